// api.cpp -- extern "C" entry points of libgpair (declared in include/gpair.h).
// Host-side argument validation, then kernel launches on the caller's stream.
// No C++ exception crosses the boundary.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "gpair_internal.h"

using namespace gpair;

namespace {

gpair_status hip_status(hipError_t e) { return e == hipSuccess ? GPAIR_OK : GPAIR_ERR_HIP; }

bool bound(const gpair_plan_s *p) { return p && p->ws; }

}  // namespace

extern "C" {

const char *gpair_status_string(gpair_status st) {
  switch (st) {
    case GPAIR_OK: return "GPAIR_OK";
    case GPAIR_NOT_CONVERGED: return "GPAIR_NOT_CONVERGED";
    case GPAIR_ERR_INVALID_ARG: return "GPAIR_ERR_INVALID_ARG";
    case GPAIR_ERR_NEAR_FIELD: return "GPAIR_ERR_NEAR_FIELD";
    case GPAIR_ERR_NONFINITE: return "GPAIR_ERR_NONFINITE";
    case GPAIR_ERR_HIP: return "GPAIR_ERR_HIP";
    case GPAIR_ERR_WORKSPACE: return "GPAIR_ERR_WORKSPACE";
    case GPAIR_ERR_SIGMA_RANGE: return "GPAIR_ERR_SIGMA_RANGE";
  }
  return "GPAIR_UNKNOWN_STATUS";
}

int gpair_abi_version(void) { return GPAIR_ABI_VERSION; }

gpair_status gpair_plan_create(const gpair_geometry *g, gpair_plan *out) {
  if (!out) return GPAIR_ERR_INVALID_ARG;
  *out = nullptr;
  gpair_plan_s *p = nullptr;
  try {
    p = new gpair_plan_s();
    p->ws = nullptr;
    p->ws_bytes = 0;
    p->timing = 0;
    p->prepared = 0;
    for (int w = 0; w < GPAIR_TIMER_KINDS; ++w) {
      p->ev_head[w] = p->ev_count[w] = 0;
      for (int i = 0; i < GPAIR_TIMER_SLOTS; ++i) p->ev_start[w][i] = p->ev_stop[w][i] = nullptr;
    }
    gpair_status st = build_plan(g, p);
    if (st != GPAIR_OK) {
      delete p;
      return st;
    }
  } catch (const std::bad_alloc &) {
    delete p;
    return GPAIR_ERR_INVALID_ARG;
  } catch (...) {
    delete p;
    return GPAIR_ERR_INVALID_ARG;
  }
  *out = p;
  return GPAIR_OK;
}

gpair_status gpair_plan_workspace_size(gpair_plan p, size_t *bytes) {
  if (!p || !bytes) return GPAIR_ERR_INVALID_ARG;
  *bytes = p->lay.total;
  return GPAIR_OK;
}

gpair_status gpair_plan_bind_workspace(gpair_plan p, void *workspace, size_t workspace_bytes,
                                       gpair_stream stream) {
  if (!p) return GPAIR_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < p->lay.total || ((uintptr_t)workspace & 255u))
    return GPAIR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  const HostTables &h = p->host;
  hipError_t e = hipSuccess;
  auto up = [&](size_t off, const void *src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, s);
  };
  up(p->lay.sens, h.sens.data(), h.sens.size() * sizeof(double));
  // Kernel records: centres now, coefficients on every operator call.
  HostVec<KernelRec> rec;
  try {
    rec.resize((size_t)p->M);
  } catch (...) {
    return GPAIR_ERR_INVALID_ARG;
  }
  // Geometry fields: the caller's float32 centre, and its float32 offset from
  // the float32-rounded centre of its adjoint tile (the filter's reference
  // block), a float32 subtraction exactly as written.
  const std::vector<TileInfo> &blocks = h.atiles;
  parallel_ranges((int64_t)blocks.size(), [&](int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) {
      const TileInfo &B = blocks[b];
      const float bx = (float)B.cx, by = (float)B.cy, bz = (float)B.cz;
      for (int64_t i = B.start; i < (int64_t)B.start + B.count; ++i) {
        KernelRec r{};
        r.fcx = (float)h.kgeo[4 * i];
        r.fcy = (float)h.kgeo[4 * i + 1];
        r.fcz = (float)h.kgeo[4 * i + 2];
        const float dx = r.fcx - bx, dy = r.fcy - by, dz = r.fcz - bz;
        r.dx = dx;
        r.dy = dy;
        r.dz = dz;
        r.dd = (float)((double)dx * dx + (double)dy * dy + (double)dz * dz);
        rec[i] = r;
      }
    }
  });
  up(p->lay.krec, rec.data(), rec.size() * sizeof(KernelRec));
  up(p->lay.perm, h.perm.data(), h.perm.size() * sizeof(int32_t));
  up(p->lay.ftiles, h.ftiles.data(), h.ftiles.size() * sizeof(TileInfo));
  up(p->lay.atiles, h.atiles.data(), h.atiles.size() * sizeof(TileInfo));
  static const unsigned long long zeros[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  up(p->lay.counters, zeros, sizeof(zeros));
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  p->ws = ws;
  p->ws_bytes = workspace_bytes;
  return GPAIR_OK;
}

void gpair_plan_destroy(gpair_plan p) {
  if (!p) return;
  for (int w = 0; w < GPAIR_TIMER_KINDS; ++w)
    for (int i = 0; i < GPAIR_TIMER_SLOTS; ++i) {
      if (p->ev_start[w][i]) (void)hipEventDestroy(p->ev_start[w][i]);
      if (p->ev_stop[w][i]) (void)hipEventDestroy(p->ev_stop[w][i]);
    }
  delete p;
}

gpair_status gpair_plan_get_info(gpair_plan p, gpair_plan_info *info) {
  if (!p || !info) return GPAIR_ERR_INVALID_ARG;
  info->n_kernels = p->M;
  info->n_sensors = p->Nd;
  info->n_samples = p->Nt;
  info->fwd_tile = p->fwd_tile;
  info->adj_tile = p->adj_tile;
  info->fwd_waves = p->fwd_waves;
  info->fwd_tiles = (int64_t)p->host.ftiles.size();
  info->adj_tiles = (int64_t)p->host.atiles.size();
  info->fwd_segment = p->Lf;
  info->adj_segment = p->La;
  info->max_taps = p->ntap_max;
  info->max_tile_radius = p->max_rho;
  info->min_distance = p->min_dist;
  info->workspace_bytes = p->lay.total;
  return GPAIR_OK;
}

gpair_status gpair_plan_tiling_slots(gpair_plan p, int32_t which, int64_t *min_first,
                                     int64_t *max_last) {
  if (!p || !min_first || !max_last || (which != 0 && which != 1)) return GPAIR_ERR_INVALID_ARG;
  return tiling_slots(p, which, min_first, max_last);
}

gpair_status gpair_plan_filter_stats(gpair_plan p, int64_t *float64_blocks, int32_t *max_steps) {
  if (!p || !float64_blocks || !max_steps) return GPAIR_ERR_INVALID_ARG;
  int64_t n = 0;
  int32_t k = 0;
  for (const TileInfo &B : p->host.atiles) {
    if (B.filter_steps < 0) ++n;
    else k = std::max(k, B.filter_steps);
  }
  *float64_blocks = n;
  *max_steps = k;
  return GPAIR_OK;
}

static void timer_begin(gpair_plan p, int which, hipStream_t s) {
  if (p->timing) (void)hipEventRecord(p->ev_start[which][p->ev_head[which]], s);
}
static void timer_end(gpair_plan p, int which, hipStream_t s) {
  if (!p->timing) return;
  (void)hipEventRecord(p->ev_stop[which][p->ev_head[which]], s);
  p->ev_head[which] = (p->ev_head[which] + 1) % GPAIR_TIMER_SLOTS;
  if (p->ev_count[which] < GPAIR_TIMER_SLOTS) ++p->ev_count[which];
}

static hipError_t prep_direct(gpair_plan p, const float *A, const float *sigma, hipStream_t s) {
  const hipError_t e = launch_prep(p, A, sigma, s);
  p->prepared = e == hipSuccess ? 1 : 0;
  return e;
}

static gpair_status forward_records(gpair_plan p, float *y, hipStream_t s) {
  hipError_t e = launch_fill(y, (int64_t)p->Nd * p->Nt, 0.0f, s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  timer_begin(p, GPAIR_TIMER_FORWARD, s);
  e = launch_forward(p, y, s);
  timer_end(p, GPAIR_TIMER_FORWARD, s);
  return hip_status(e);
}

static gpair_status adjoint_records(gpair_plan p, const float *delta, float *gA, float *gsigma,
                                    float *gcentres, hipStream_t s) {
  timer_begin(p, GPAIR_TIMER_ADJOINT, s);
  const hipError_t e = launch_adjoint(p, delta, gA, gsigma, gcentres, s);
  timer_end(p, GPAIR_TIMER_ADJOINT, s);
  return hip_status(e);
}

gpair_status gpair_forward(gpair_plan p, const float *A, const float *sigma, float *y,
                           gpair_stream stream) {
  if (!bound(p) || !A || !sigma || !y) return GPAIR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (prep_direct(p, A, sigma, s) != hipSuccess) return GPAIR_ERR_HIP;
  return forward_records(p, y, s);
}

gpair_status gpair_prepare(gpair_plan p, const float *A, const float *sigma,
                           gpair_stream stream) {
  if (!bound(p) || !sigma) return GPAIR_ERR_INVALID_ARG;
  return hip_status(prep_direct(p, A, sigma, (hipStream_t)stream));
}

gpair_status gpair_forward_prepared(gpair_plan p, float *y, gpair_stream stream) {
  if (!bound(p) || !y || !p->prepared) return GPAIR_ERR_INVALID_ARG;
  return forward_records(p, y, (hipStream_t)stream);
}

gpair_status gpair_adjoint_prepared(gpair_plan p, const float *delta, float *gA, float *gsigma,
                                    gpair_stream stream) {
  if (!bound(p) || !delta || !gA || !p->prepared) return GPAIR_ERR_INVALID_ARG;
  return adjoint_records(p, delta, gA, gsigma, nullptr, (hipStream_t)stream);
}

gpair_status gpair_adjoint(gpair_plan p, const float *A, const float *sigma,
                           const float *delta, float *gA, float *gsigma,
                           gpair_stream stream) {
  if (!bound(p) || !sigma || !delta || !gA) return GPAIR_ERR_INVALID_ARG;
  if (gsigma && !A) return GPAIR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (prep_direct(p, A, sigma, s) != hipSuccess) return GPAIR_ERR_HIP;
  return adjoint_records(p, delta, gA, gsigma, nullptr, s);
}

gpair_status gpair_adjoint_centres(gpair_plan p, const float *A, const float *sigma,
                                   const float *delta, float *gA, float *gsigma,
                                   float *gcentres, gpair_stream stream) {
  if (!bound(p) || !A || !sigma || !delta || !gA || !gcentres) return GPAIR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (prep_direct(p, A, sigma, s) != hipSuccess) return GPAIR_ERR_HIP;
  return adjoint_records(p, delta, gA, gsigma, gcentres, s);
}

gpair_status gpair_forward_aniso(gpair_plan p, const float *A, const float *sigma6, float *y,
                                 gpair_stream stream) {
  if (!bound(p) || !A || !sigma6 || !y) return GPAIR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  p->prepared = 0;  // the anisotropic records overwrite the direct coefficients
  hipError_t e = launch_aniso_prep(p, A, sigma6, s);
  if (e == hipSuccess) e = launch_fill(y, (int64_t)p->Nd * p->Nt, 0.0f, s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  timer_begin(p, GPAIR_TIMER_FORWARD, s);
  e = launch_aniso_forward(p, y, s);
  timer_end(p, GPAIR_TIMER_FORWARD, s);
  return hip_status(e);
}

gpair_status gpair_adjoint_aniso(gpair_plan p, const float *A, const float *sigma6,
                                 const float *delta, float *gA, float *gsigma6,
                                 gpair_stream stream) {
  if (!bound(p) || !sigma6 || !delta || !gA) return GPAIR_ERR_INVALID_ARG;
  if (gsigma6 && !A) return GPAIR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  p->prepared = 0;
  hipError_t e = launch_aniso_prep(p, A, sigma6, s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  timer_begin(p, GPAIR_TIMER_ADJOINT, s);
  e = launch_aniso_adjoint(p, delta, gA, gsigma6, nullptr, s);
  timer_end(p, GPAIR_TIMER_ADJOINT, s);
  return hip_status(e);
}

gpair_status gpair_adjoint_aniso_centres(gpair_plan p, const float *A, const float *sigma6,
                                         const float *delta, float *gA, float *gsigma6,
                                         float *gcentres, gpair_stream stream) {
  if (!bound(p) || !A || !sigma6 || !delta || !gA || !gcentres) return GPAIR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  p->prepared = 0;
  hipError_t e = launch_aniso_prep(p, A, sigma6, s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  timer_begin(p, GPAIR_TIMER_ADJOINT, s);
  e = launch_aniso_adjoint(p, delta, gA, gsigma6, gcentres, s);
  timer_end(p, GPAIR_TIMER_ADJOINT, s);
  return hip_status(e);
}

gpair_status gpair_assa_grid_params(gpair_plan p, double sigma, gpair_assa_grid *out) {
  if (!p || !out) return GPAIR_ERR_INVALID_ARG;
  AssaGrid g;
  const gpair_status st = assa_grid(p, sigma, &g);
  if (st != GPAIR_OK) return st;
  out->n_half = g.n_half;
  out->alpha = g.alpha;
  out->K = g.K;
  out->n_fine = g.n_fine;
  out->fwd_segment = g.F;
  out->fwd_passes = (g.Lc + g.Lch - 1) / g.Lch;
  out->adj_segment = g.Fa;
  out->adj_stage_sensors = g.S;
  return GPAIR_OK;
}

gpair_status gpair_assa_workspace_size(gpair_plan p, double sigma, size_t *bytes) {
  if (!p || !bytes) return GPAIR_ERR_INVALID_ARG;
  AssaGrid g;
  const gpair_status st = assa_grid(p, sigma, &g);
  if (st != GPAIR_OK) return st;
  *bytes = assa_work_bytes(p, g);
  return GPAIR_OK;
}

gpair_status gpair_assa_forward(gpair_plan p, const float *x, double sigma, float *y,
                                gpair_stream stream) {
  if (!bound(p) || !x || !y) return GPAIR_ERR_INVALID_ARG;
  AssaGrid g;
  const gpair_status st = assa_grid(p, sigma, &g);
  if (st != GPAIR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  p->prepared = 0;  // the ASSA prep overwrites the direct coefficients
  hipError_t e = launch_assa_prep(p, x, s);
  if (e == hipSuccess) e = launch_fill(y, (int64_t)p->Nd * p->Nt, 0.0f, s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  timer_begin(p, GPAIR_TIMER_ASSA_FORWARD, s);
  e = launch_assa_forward(p, g, y, s);
  timer_end(p, GPAIR_TIMER_ASSA_FORWARD, s);
  return hip_status(e);
}

gpair_status gpair_assa_adjoint(gpair_plan p, double sigma, const float *delta, float *g,
                                void *work, size_t work_bytes, gpair_stream stream) {
  if (!bound(p) || !delta || !g || !work) return GPAIR_ERR_INVALID_ARG;
  if (((uintptr_t)work & 255) != 0) return GPAIR_ERR_INVALID_ARG;
  AssaGrid grid;
  const gpair_status st = assa_grid(p, sigma, &grid);
  if (st != GPAIR_OK) return st;
  if (work_bytes < assa_work_bytes(p, grid)) return GPAIR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  float *dconv = (float *)work;
  hipError_t e = launch_assa_dconv(p, grid, delta, dconv, s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  timer_begin(p, GPAIR_TIMER_ASSA_ADJOINT, s);
  e = launch_assa_adjoint(p, grid, dconv, g, s);
  timer_end(p, GPAIR_TIMER_ASSA_ADJOINT, s);
  return hip_status(e);
}

gpair_status gpair_npc_map(int64_t n, const float *z, double eps, float *x,
                           gpair_stream stream) {
  if (n < 0 || (n > 0 && (!z || !x)) || !std::isfinite(eps)) return GPAIR_ERR_INVALID_ARG;
  if (n == 0) return GPAIR_OK;
  return hip_status(launch_npc_map(n, z, (float)eps, x, (hipStream_t)stream));
}

gpair_status gpair_npc_grad(int64_t n, const float *z, const float *gx, double eps, float *gz,
                            gpair_stream stream) {
  if (n < 0 || (n > 0 && (!z || !gx || !gz)) || !std::isfinite(eps))
    return GPAIR_ERR_INVALID_ARG;
  if (n == 0) return GPAIR_OK;
  return hip_status(launch_npc_grad(n, z, gx, (float)eps, gz, (hipStream_t)stream));
}

static bool vcr_dims_ok(int32_t nx, int32_t ny, int32_t nz) {
  return nx >= 1 && ny >= 1 && nz >= 1 && (int64_t)nx * ny * nz <= (int64_t(1) << 31) / 16;
}

gpair_status gpair_vcr_workspace_size(int32_t nx, int32_t ny, int32_t nz, size_t *bytes) {
  if (!bytes || !vcr_dims_ok(nx, ny, nz)) return GPAIR_ERR_INVALID_ARG;
  *bytes = vcr_work_bytes(nx, ny, nz);
  return GPAIR_OK;
}

gpair_status gpair_vcr(int32_t nx, int32_t ny, int32_t nz, const float *x, double beta,
                       double eps, double lambda, float *grad, double *value, void *work,
                       size_t work_bytes, gpair_stream stream) {
  if (!vcr_dims_ok(nx, ny, nz) || !x || !std::isfinite(beta) || !(eps >= 0.0) ||
      !std::isfinite(eps) || !std::isfinite(lambda))
    return GPAIR_ERR_INVALID_ARG;
  if (!work || work_bytes < vcr_work_bytes(nx, ny, nz) || ((uintptr_t)work & 255u))
    return GPAIR_ERR_WORKSPACE;
  if (!grad && !value) return GPAIR_OK;
  return hip_status(
      launch_vcr(nx, ny, nz, x, beta, eps, lambda, grad, value, work, (hipStream_t)stream));
}

gpair_status gpair_cawr_rate(int64_t t, double eta_min, double eta_max, int64_t T0,
                             int32_t Tmult, double *rate) {
  if (!rate || t < 0 || T0 < 1 || Tmult < 1 || !std::isfinite(eta_min) ||
      !std::isfinite(eta_max))
    return GPAIR_ERR_INVALID_ARG;
  int64_t start = 0, period = T0;
  while (t >= start + period) {
    start += period;
    if (period > (int64_t(1) << 40) / Tmult) break;  // t lies in this (huge) period
    period *= Tmult;
  }
  const double tc = (double)(t - start), ti = (double)period;
  *rate = eta_min + 0.5 * (eta_max - eta_min) * (1.0 + std::cos(M_PI * tc / ti));
  return GPAIR_OK;
}

gpair_status gpair_sigma_violations(gpair_plan p, int64_t *count, gpair_stream stream) {
  if (!bound(p) || !count) return GPAIR_ERR_INVALID_ARG;
  unsigned long long v = 0;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(&v, ws_counters(p), sizeof(v), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  *count = (int64_t)v;
  return GPAIR_OK;
}

gpair_status gpair_residual(gpair_plan p, const float *y, const float *b, float scale,
                            float *delta, double *norms, gpair_stream stream) {
  if (!bound(p) || !y || !b || !norms || !std::isfinite(scale)) return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_residual(p, y, b, scale, delta, norms, (hipStream_t)stream));
}

gpair_status gpair_warm_rescale(gpair_plan p, float *A, const float *sigma, const float *b,
                                float *y_scratch, gpair_warm_report *report,
                                gpair_stream stream) {
  if (!bound(p) || !A || !sigma || !b || !y_scratch || !report) return GPAIR_ERR_INVALID_ARG;
  const hipStream_t s = (hipStream_t)stream;
  gpair_status st = gpair_forward(p, A, sigma, y_scratch, stream);
  if (st != GPAIR_OK) return st;
  double *dots = ws_partials(p) + 3 * kResidualBlocks;  // the 64-byte tail
  if (launch_dot3(p, y_scratch, b, dots, s) != hipSuccess) return GPAIR_ERR_HIP;
  double h[3];
  if (hipMemcpyAsync(h, dots, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GPAIR_ERR_HIP;
  const double yb = h[0], yy = h[1], bb = h[2];
  if (!std::isfinite(yb) || !std::isfinite(yy) || !std::isfinite(bb)) return GPAIR_ERR_NONFINITE;
  if (!(bb > 0.0)) return GPAIR_ERR_INVALID_ARG;
  const int64_t M = p->M;
  double c = (yy > 0.0 && yb > 0.0) ? yb / yy : 0.0;
  // ||c y - b||^2 / ||b||^2 at the optimal c: 1 - <y,b>^2 / (||y||^2 ||b||^2)
  double rho = c > 0.0 ? std::sqrt(std::fmax(0.0, 1.0 - (yb / yy) * (yb / bb))) : 1.0;
  const bool fall = !(c > 0.0) || !(rho < 1.0);
  if (fall) {
    c = 0.0;
    rho = 1.0;
    if (launch_fill(A, M, 0.0f, s) != hipSuccess) return GPAIR_ERR_HIP;
  } else if (launch_scale(A, M, (float)c, s) != hipSuccess) {
    return GPAIR_ERR_HIP;
  }
  report->c_star = c;
  report->rho = rho;
  report->fell_back = fall ? 1 : 0;
  report->pad = 0;
  return GPAIR_OK;
}

gpair_status gpair_pgd_update(int64_t n, float *x, const float *g, float step, float lo,
                              float hi, gpair_stream stream) {
  if (n < 0 || (n > 0 && (!x || !g)) || !std::isfinite(step) || std::isnan(lo) ||
      std::isnan(hi) || lo > hi)
    return GPAIR_ERR_INVALID_ARG;
  if (n == 0) return GPAIR_OK;
  return hip_status(launch_pgd(n, x, g, step, lo, hi, (hipStream_t)stream));
}

gpair_status gpair_adam_update(int64_t n, float *x, const float *g, float *m, float *v,
                               float grad_scale, float lr, float beta1, float beta2,
                               float eps, int32_t t, float lo, float hi,
                               gpair_stream stream) {
  if (n < 0 || (n > 0 && (!x || !g || !m || !v)) || t < 1 || !std::isfinite(grad_scale) ||
      !std::isfinite(lr) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f) || std::isnan(lo) ||
      std::isnan(hi) || lo > hi)
    return GPAIR_ERR_INVALID_ARG;
  if (n == 0) return GPAIR_OK;
  return hip_status(launch_adam(n, x, g, m, v, grad_scale, lr, beta1, beta2, eps, t, lo, hi,
                                (hipStream_t)stream));
}

gpair_status gpair_plan_set_timing(gpair_plan p, int enable) {
  if (!p) return GPAIR_ERR_INVALID_ARG;
  if (enable) {
    for (int w = 0; w < GPAIR_TIMER_KINDS; ++w)
      for (int i = 0; i < GPAIR_TIMER_SLOTS; ++i) {
        if (!p->ev_start[w][i] && hipEventCreate(&p->ev_start[w][i]) != hipSuccess)
          return GPAIR_ERR_HIP;
        if (!p->ev_stop[w][i] && hipEventCreate(&p->ev_stop[w][i]) != hipSuccess)
          return GPAIR_ERR_HIP;
      }
  }
  p->timing = enable ? 1 : 0;
  for (int w = 0; w < GPAIR_TIMER_KINDS; ++w) p->ev_head[w] = p->ev_count[w] = 0;
  return GPAIR_OK;
}

gpair_status gpair_plan_kernel_times(gpair_plan p, int which, float *ms, int32_t capacity,
                                     int32_t *count) {
  if (!p || !count || capacity < 0 || (capacity > 0 && !ms) ||
      which < 0 || which >= GPAIR_TIMER_KINDS || !p->timing)
    return GPAIR_ERR_INVALID_ARG;
  const int n = p->ev_count[which];
  const int first = (p->ev_head[which] - n + GPAIR_TIMER_SLOTS) % GPAIR_TIMER_SLOTS;
  if (n > 0) {
    const int last = (p->ev_head[which] - 1 + GPAIR_TIMER_SLOTS) % GPAIR_TIMER_SLOTS;
    if (hipEventSynchronize(p->ev_stop[which][last]) != hipSuccess) return GPAIR_ERR_HIP;
  }
  for (int i = 0; i < n && i < capacity; ++i) {
    const int slot = (first + i) % GPAIR_TIMER_SLOTS;
    if (hipEventElapsedTime(ms + i, p->ev_start[which][slot], p->ev_stop[which][slot]) !=
        hipSuccess)
      return GPAIR_ERR_HIP;
  }
  *count = n;
  p->ev_count[which] = 0;
  return GPAIR_OK;
}

}  // extern "C"
