// solve.cpp -- the reconstruction driver gpair_solve (arXiv 2602.03893,
// Algorithm 2 without its regulariser, non-negativity reparameterisation and
// learning-rate schedule): forward -> residual -> adjoint -> update, with one
// host synchronisation every check_every iterations to read the two norms.
#include <chrono>
#include <cmath>

#include "gpair_internal.h"

using namespace gpair;

namespace {

struct SolveLayout {
  size_t y, gA, gS, mA, vA, mS, vS, norms, z, vcr, total;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

SolveLayout solve_layout(const gpair_plan_s *p, const gpair_solve_opts *o) {
  SolveLayout l{};
  const size_t M = (size_t)p->M, N = (size_t)p->Nd * (size_t)p->Nt;
  const bool adam = o->method == GPAIR_SOLVE_ADAM;
  const bool sig = adam && o->learn_sigma;
  size_t off = 0;
  l.y = off;     off = a256(off + N * 4);
  l.gA = off;    off = a256(off + M * 4);
  l.gS = off;    off = a256(off + (sig ? M * 4 : 0));
  l.mA = off;    off = a256(off + (adam ? M * 4 : 0));
  l.vA = off;    off = a256(off + (adam ? M * 4 : 0));
  l.mS = off;    off = a256(off + (sig ? M * 4 : 0));
  l.vS = off;    off = a256(off + (sig ? M * 4 : 0));
  l.norms = off; off = a256(off + 2 * sizeof(double));
  l.z = off;     off = a256(off + (o->npc ? M * 4 : 0));
  l.vcr = off;
  off = a256(off + (o->reg_lambda != 0.0 ? vcr_work_bytes(o->grid_nx, o->grid_ny, o->grid_nz)
                                         : 0));
  l.total = off;
  return l;
}

bool valid_opts(const gpair_plan_s *p, const gpair_solve_opts *o) {
  if (!o) return false;
  if (o->method != GPAIR_SOLVE_PGD && o->method != GPAIR_SOLVE_ADAM) return false;
  if (o->max_iters < 0 || o->check_every < 1) return false;
  if (!(o->tol >= 0.0) || std::isnan(o->a_lo) || std::isnan(o->a_hi) || o->a_lo > o->a_hi)
    return false;
  if (o->method == GPAIR_SOLVE_PGD && !std::isfinite(o->step)) return false;
  if (o->npc && (o->method != GPAIR_SOLVE_ADAM || !std::isfinite(o->npc_eps))) return false;
  if (!std::isfinite(o->reg_lambda)) return false;
  if (o->reg_lambda != 0.0) {
    if (!std::isfinite(o->reg_beta) || !(o->reg_eps >= 0.0) || !std::isfinite(o->reg_eps))
      return false;
    if (o->grid_nx < 1 || o->grid_ny < 1 || o->grid_nz < 1 ||
        (int64_t)o->grid_nx * o->grid_ny * o->grid_nz != p->M)
      return false;
  }
  if (o->cawr_T0 < 0 || (o->cawr_T0 > 0 && (o->cawr_Tmult < 1 || !std::isfinite(o->lr_min))))
    return false;
  if (o->method == GPAIR_SOLVE_ADAM) {
    if (!std::isfinite(o->lr_A) || !(o->beta1 >= 0 && o->beta1 < 1) ||
        !(o->beta2 >= 0 && o->beta2 < 1) || !(o->eps >= 0))
      return false;
    if (o->learn_sigma) {
      if (!std::isfinite(o->lr_sigma) || !(o->sigma_lo > 0) || !(o->sigma_hi >= o->sigma_lo) ||
          !(o->sigma_hi <= p->sigma_max))
        return false;
    }
  }
  return true;
}

}  // namespace

extern "C" {

gpair_status gpair_solve_workspace_size(gpair_plan p, const gpair_solve_opts *o,
                                        size_t *bytes) {
  if (!p || !bytes || !valid_opts(p, o)) return GPAIR_ERR_INVALID_ARG;
  *bytes = solve_layout(p, o).total;
  return GPAIR_OK;
}

gpair_status gpair_solve(gpair_plan p, const float *b, float *A, float *sigma,
                         const gpair_solve_opts *o, void *workspace, size_t workspace_bytes,
                         gpair_solve_report *r, gpair_stream stream) {
  if (!p || !p->ws || !b || !A || !sigma || !r || !valid_opts(p, o))
    return GPAIR_ERR_INVALID_ARG;
  const SolveLayout L = solve_layout(p, o);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace & 255u))
    return GPAIR_ERR_WORKSPACE;
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  float *y = (float *)(ws + L.y);
  float *gA = (float *)(ws + L.gA);
  const bool adam = o->method == GPAIR_SOLVE_ADAM;
  const bool sig = adam && o->learn_sigma;
  float *gS = sig ? (float *)(ws + L.gS) : nullptr;
  double *norms = (double *)(ws + L.norms);
  const int64_t M = p->M;
  const float a_lo = (float)o->a_lo, a_hi = (float)o->a_hi;

  if (r->history)
    for (int i = 0; i <= o->max_iters; ++i) r->history[i] = -1.0;
  r->iters = 0;
  r->converged = 0;
  r->rel_residual = -1.0;
  r->seconds = 0.0;

  const bool npc = o->npc != 0;
  const bool reg = o->reg_lambda != 0.0;
  float *z = npc ? (float *)(ws + L.z) : nullptr;
  const float npc_eps = (float)o->npc_eps;
  hipError_t e = hipSuccess;
  // NPC: the latent starts from the caller's A; A then holds x = phi(z).
  if (npc) e = hipMemcpyAsync(z, A, (size_t)p->M * 4, hipMemcpyDeviceToDevice, s);
  if (adam && e == hipSuccess) {
    e = launch_fill((float *)(ws + L.mA), M, 0.0f, s);
    if (e == hipSuccess) e = launch_fill((float *)(ws + L.vA), M, 0.0f, s);
    if (sig && e == hipSuccess) e = launch_fill((float *)(ws + L.mS), M, 0.0f, s);
    if (sig && e == hipSuccess) e = launch_fill((float *)(ws + L.vS), M, 0.0f, s);
  }
  // ||b||^2 (norms[1] of a residual of b against itself).
  double hn[2] = {0, 0};
  if (e == hipSuccess) e = launch_residual(p, b, b, 0.0f, nullptr, norms, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hn, norms, sizeof(hn), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return GPAIR_ERR_HIP;
  const double nb2 = hn[1];
  if (!std::isfinite(nb2)) return GPAIR_ERR_NONFINITE;
  if (!(nb2 > 0.0)) return GPAIR_ERR_INVALID_ARG;  // b == 0: residual undefined
  // Adam minimises 0.5 ||Ax - b||^2 / ||b||^2, PGD 0.5 ||Ax - b||^2.
  const float scale = adam ? (float)(1.0 / nb2) : 1.0f;

  auto read_rho = [&](double *rho) -> gpair_status {
    double h2[2];
    hipError_t ee = hipMemcpyAsync(h2, norms, sizeof(h2), hipMemcpyDeviceToHost, s);
    if (ee == hipSuccess) ee = hipStreamSynchronize(s);
    if (ee != hipSuccess) return GPAIR_ERR_HIP;
    *rho = std::sqrt(h2[0] / nb2);
    return std::isfinite(*rho) ? GPAIR_OK : GPAIR_ERR_NONFINITE;
  };

  gpair_status st = GPAIR_OK;
  int it = 0;
  bool converged = false;
  double rho = -1.0;
  for (; it < o->max_iters; ++it) {
    if (npc && launch_npc_map(M, z, npc_eps, A, s) != hipSuccess) return GPAIR_ERR_HIP;
    // (A, sigma) are the same for the forward and the adjoint of an
    // iteration: their coefficient records are built once.
    st = gpair_prepare(p, A, sigma, stream);
    if (st == GPAIR_OK) st = gpair_forward_prepared(p, y, stream);
    if (st != GPAIR_OK) return st;
    if (launch_residual(p, y, b, scale, y, norms, s) != hipSuccess) return GPAIR_ERR_HIP;
    if (it % o->check_every == 0) {
      st = read_rho(&rho);
      if (st != GPAIR_OK) {
        r->iters = it;
        return st;
      }
      if (r->history) r->history[it] = rho;
      if (o->tol > 0.0 && rho <= o->tol) {
        converged = true;
        break;
      }
    }
    st = gpair_adjoint_prepared(p, y, gA, gS, stream);
    if (st != GPAIR_OK) return st;
    if (reg && launch_vcr(o->grid_nx, o->grid_ny, o->grid_nz, A, o->reg_beta, o->reg_eps,
                          o->reg_lambda, gA, nullptr, ws + L.vcr, s) != hipSuccess)
      return GPAIR_ERR_HIP;
    double lr = o->lr_A;
    if (o->cawr_T0 > 0 &&
        gpair_cawr_rate(it, o->lr_min, o->lr_A, o->cawr_T0, o->cawr_Tmult, &lr) != GPAIR_OK)
      return GPAIR_ERR_INVALID_ARG;
    if (npc) {
      e = launch_npc_grad(M, z, gA, npc_eps, gA, s);
      if (e == hipSuccess)
        e = launch_adam(M, z, gA, (float *)(ws + L.mA), (float *)(ws + L.vA), 1.0f, (float)lr,
                        (float)o->beta1, (float)o->beta2, (float)o->eps, it + 1, -INFINITY,
                        INFINITY, s);
      if (e == hipSuccess && sig)
        e = launch_adam(M, sigma, gS, (float *)(ws + L.mS), (float *)(ws + L.vS), 1.0f,
                        (float)o->lr_sigma, (float)o->beta1, (float)o->beta2, (float)o->eps,
                        it + 1, (float)o->sigma_lo, (float)o->sigma_hi, s);
    } else if (adam) {
      e = launch_adam(M, A, gA, (float *)(ws + L.mA), (float *)(ws + L.vA), 1.0f, (float)lr,
                      (float)o->beta1, (float)o->beta2, (float)o->eps, it + 1, a_lo, a_hi, s);
      if (e == hipSuccess && sig)
        e = launch_adam(M, sigma, gS, (float *)(ws + L.mS), (float *)(ws + L.vS), 1.0f,
                        (float)o->lr_sigma, (float)o->beta1, (float)o->beta2, (float)o->eps,
                        it + 1, (float)o->sigma_lo, (float)o->sigma_hi, s);
    } else {
      e = launch_pgd(M, A, gA, (float)o->step, a_lo, a_hi, s);
    }
    if (e != hipSuccess) return GPAIR_ERR_HIP;
  }
  if (npc && launch_npc_map(M, z, npc_eps, A, s) != hipSuccess) return GPAIR_ERR_HIP;
  if (!converged) {
    st = gpair_forward(p, A, sigma, y, stream);
    if (st != GPAIR_OK) return st;
    if (launch_residual(p, y, b, scale, nullptr, norms, s) != hipSuccess) return GPAIR_ERR_HIP;
    st = read_rho(&rho);
    if (st != GPAIR_OK) {
      r->iters = it;
      return st;
    }
    if (r->history) r->history[it] = rho;
    converged = o->tol > 0.0 && rho <= o->tol;
  }
  r->iters = it;
  r->rel_residual = rho;
  r->converged = converged ? 1 : 0;
  r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return converged ? GPAIR_OK : GPAIR_NOT_CONVERGED;
}

}  // extern "C"
