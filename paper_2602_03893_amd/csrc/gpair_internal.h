// gpair_internal.h -- data layout shared by the host planner, the C ABI layer
// and the gfx950 kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <memory>
#include <thread>
#include <utility>
#include <vector>

#include "gpair.h"

namespace gpair {

// std::allocator that leaves trivially constructible elements uninitialised:
// the planner's large host tables (GBs at 67 M kernels) are then first
// written by parallel fill loops instead of a serial zero fill.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U> &) {}
  template <class U>
  void construct(U *p) {
    ::new ((void *)p) U;
  }
  template <class U, class... A>
  void construct(U *p, A &&...a) {
    ::new ((void *)p) U(std::forward<A>(a)...);
  }
};
template <class T>
using HostVec = std::vector<T, NoInitAlloc<T>>;

// Host threads for the planner's O(M) passes.
inline int host_threads() {
  const unsigned n = std::thread::hardware_concurrency();
  return (int)std::min<unsigned>(std::max<unsigned>(n, 1u), 16u);
}

// f(begin, end) over [0, n) in contiguous chunks, one per thread.
template <class F>
void parallel_ranges(int64_t n, F f) {
  const int T = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, n / 65536));
  if (T <= 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t) th.emplace_back(f, n * t / T, n * (t + 1) / T);
  for (auto &x : th) x.join();
}

// Bounding sphere and kernel range of one tile (a compact spatial block of
// kernels, consecutive in the plan's permuted kernel order).  Adjoint tiles
// are nested in forward tiles; they are also the reference blocks of the
// float32 distance filter (the float32-rounded centre of an adjoint tile is
// the reference point of its members).
struct alignas(16) TileInfo {
  double cx, cy, cz;  // sphere centre (m)
  double rho;         // sphere radius (m): every member is within rho
  int32_t start;      // first member in permuted order
  int32_t count;      // number of members (<= the tile size)
  float asum;         // per-call scratch of the ASSA forward: sum of |x| over
                      // the members (forward tiles only)
  union {
    int32_t first_block;   // forward tiles: index of the first adjoint tile inside
    int32_t filter_steps;  // adjoint tiles: fixed-point steps of the float32
                           // window filter, or -1: every pair in float64
  };
};
static_assert(sizeof(TileInfo) == 48, "TileInfo layout");

// One 64-byte record per kernel (permuted order), read by the forward as a
// single scalar load.  The geometry fields (d*, dd, fc*) are written once
// when the plan is bound; the coefficients are rebuilt on every operator
// call from (A, sigma).  Offsets along a window are in samples: with
// Delta = v dt, h = n_sigma sigma / Delta and c = -log2(e) Delta^2 /
// (2 sigma^2),
//   exp(-d^2/(2 sigma^2)) = exp2(c u^2) for d = u Delta;
//   the ratio of consecutive taps (u -> u - 1) is q(u) = exp2(k1 u + c) with
//   k1 = -2c, and q itself is multiplied by rq = exp2(2c) from one tap to
//   the next.
struct alignas(64) KernelRec {
  float dx, dy, dz;  // float32 centre minus the float32 reference point of
                     // its adjoint tile (a float32 subtraction)
  float dd;          // |(dx, dy, dz)|^2
  float hf;          // h (float32)
  float H;           // (ntap - 1) - 2h: tap ntap-1 is in the window iff the
                     // first tap's offset minus h is >= H
  float amp;         // A_k
  float c;           // -log2(e) Delta^2 / (2 sigma_k^2)
  float k1;          // -2 c
  float rq;          // exp2(2 c)
  int32_t ntap;      // floor(2 h) + 1: most samples a window can hold
  float fcz;         // the caller's float32 centre (z)
  double h;          // n_sigma sigma_k / Delta (float64, the exact path)
  float fcx, fcy;    // the caller's float32 centre (x, y)
};
static_assert(sizeof(KernelRec) == 64, "KernelRec layout");

// The same 64 bytes as the ASSA operators use them (rebuilt by the ASSA
// prep on every call; the geometry fields are shared with KernelRec).
struct alignas(64) AssaRec {
  float dx, dy, dz, dd;  // geometry (unused by ASSA)
  double cx, cy;         // float64 copy of the float32 centre
  double cz;
  float amp;             // x_k
  float fcz;             // geometry
  double cc;             // |c|^2
  float fcx, fcy;        // geometry
};
static_assert(sizeof(AssaRec) == 64, "AssaRec layout");
static_assert(offsetof(AssaRec, fcz) == offsetof(KernelRec, fcz) &&
                  offsetof(AssaRec, fcx) == offsetof(KernelRec, fcx) &&
                  offsetof(AssaRec, dd) == offsetof(KernelRec, dd),
              "shared geometry fields");

constexpr int kWave = 64;
constexpr int kAdjSensorsPerStage = 64; // sensors staged per LDS refill
// Cap of the dynamic LDS segment per workgroup.  The kernels' static LDS comes
// on top (at most 4.25 KiB: the direct adjoint's staged sensors, tap counts
// and ranking), so a workgroup asks for at most 67.25 KiB of gfx950's 160 KiB;
// the planner shrinks tiles until their segments fit the cap.
constexpr int kMaxSegmentBytes = 63 * 1024;
constexpr int kResidualBlocks = 1024;
constexpr int kXcds = 8;                // MI355X: 8 accelerator dies

// Offsets (bytes) of each table inside the plan workspace.
struct WorkspaceLayout {
  size_t sens, perm, ftiles, atiles, krec, counters, partials;
  size_t det;  // deterministic forward: int64 [Nd][Nt] trace accumulator (0 bytes otherwise)
  size_t total;
};

struct HostTables {
  std::vector<double> sens;      // [Nd][4]: x, y, z, |s|^2
  HostVec<double> kgeo;          // [M][4] permuted centres
  HostVec<int32_t> perm;         // [M] permuted index -> caller index
  std::vector<TileInfo> ftiles;  // forward tiles
  std::vector<TileInfo> atiles;  // adjoint tiles
};

}  // namespace gpair

struct gpair_plan_s {
  // geometry constants
  int64_t M;
  int32_t Nd, Nt;
  double dt, t0, v, nsig, sigma_max;
  double vdt, inv_vdt, t0_over_dt, hmax;
  int32_t ntap_max;
  // tiling
  int32_t fwd_tile, adj_tile;
  int32_t fwd_waves;  // waves (sensor groups of 64) per forward workgroup
  int32_t deterministic;  // forward flush through a global int64 fixed point
  int32_t prepared;       // the records hold the direct operators' coefficients
                          // (set by their prep, cleared by the ASSA prep)
  int32_t Lf, La;     // samples per forward / adjoint LDS segment
  double max_rho, min_dist;
  gpair::HostTables host;
  gpair::WorkspaceLayout lay;
  // bound workspace (device)
  char *ws;
  size_t ws_bytes;
  // timing: per kind (forward, adjoint) a ring of event pairs
  int timing;
  hipEvent_t ev_start[GPAIR_TIMER_KINDS][GPAIR_TIMER_SLOTS];
  hipEvent_t ev_stop[GPAIR_TIMER_KINDS][GPAIR_TIMER_SLOTS];
  int ev_head[GPAIR_TIMER_KINDS];
  int ev_count[GPAIR_TIMER_KINDS];
};

namespace gpair {

// The float32 window filter of the operators for a reference block of
// radius rho (about its float32-rounded centre) seen from sensors at
// distance >= R: the number of fixed-point steps for the distance offset
// that brings its truncation below kFilterIterTol samples, or -1 when the
// filter's error bound is not below kFilterGuard / 2 (then the operators
// decide every pair of the block in float64).
constexpr double kFilterGuard = 0x1p-14;  // samples
constexpr double kFilterIterTol = 1e-6;   // samples
constexpr int kFilterMaxSteps = 8;
int filter_steps(double R, double rho, double inv_vdt, double hmax);

// Kernel launchers (operators.hip, vector_ops.hip).  All return hipSuccess or
// the launch error.
hipError_t launch_prep(const gpair_plan_s *p, const float *A, const float *sigma,
                       hipStream_t s);
hipError_t launch_fill(float *x, int64_t n, float value, hipStream_t s);
hipError_t launch_scale(float *x, int64_t n, float alpha, hipStream_t s);
// (<y, b>, ||y||^2, ||b||^2) in float64, fixed summation order, into out[3]
// (device); partial sums in the plan workspace.
hipError_t launch_dot3(const gpair_plan_s *p, const float *y, const float *b, double *out,
                       hipStream_t s);
// The forward into y (zeroed by the caller); with p->deterministic, y need
// not be zeroed and the flush goes through the int64 accumulator.
hipError_t launch_forward(const gpair_plan_s *p, float *y, hipStream_t s);
// gsigma and gcentres may be null (not computed / not written).
hipError_t launch_adjoint(const gpair_plan_s *p, const float *delta, float *gA,
                          float *gsigma, float *gcentres, hipStream_t s);
// Anisotropic kernels (aniso.hip): records from (A, Sigma), forward into y
// (zeroed by the caller), adjoint (gsig6 and gcentres may be null).
hipError_t launch_aniso_prep(const gpair_plan_s *p, const float *A, const float *sig6,
                             hipStream_t s);
hipError_t launch_aniso_forward(const gpair_plan_s *p, float *y, hipStream_t s);
hipError_t launch_aniso_adjoint(const gpair_plan_s *p, const float *delta, float *gA,
                                float *gsig6, float *gcentres, hipStream_t s);
hipError_t launch_residual(const gpair_plan_s *p, const float *y, const float *b,
                           float scale, float *delta, double *norms,
                           hipStream_t s);
hipError_t launch_pgd(int64_t n, float *x, const float *g, float step, float lo,
                      float hi, hipStream_t s);
hipError_t launch_adam(int64_t n, float *x, const float *g, float *m, float *v,
                       float grad_scale, float lr, float beta1, float beta2,
                       float eps, int32_t t, float lo, float hi, hipStream_t s);

// ASSA operators (assa.hip).  AssaGrid holds the grid of one shared sigma and
// the LDS segment sizes that follow from the plan's tiles.
constexpr int kAssaMaxK = 120;  // h has at most 2 kAssaMaxK + 1 taps (fits the LDS rows)
struct AssaGrid {
  int32_t n_half, alpha, K, n_fine;
  int32_t Lc;   // coarse samples of a forward (tile, sensor) shell
  int32_t Lch;  // coarse samples per forward pass
  int32_t F;    // fine rows per forward LDS segment (alpha (Lch - 1) + 2K + 1)
  int32_t Fa;   // fine samples per adjoint stage row
  int32_t S;    // sensors per adjoint stage
  double sigma;
};
// Grid of `sigma` for plan p; GPAIR_OK or the status to return.
gpair_status assa_grid(const gpair_plan_s *p, double sigma, AssaGrid *g);
size_t assa_work_bytes(const gpair_plan_s *p, const AssaGrid &g);
hipError_t launch_assa_prep(const gpair_plan_s *p, const float *x, hipStream_t s);
hipError_t launch_assa_forward(const gpair_plan_s *p, const AssaGrid &g, float *y,
                               hipStream_t s);
hipError_t launch_assa_dconv(const gpair_plan_s *p, const AssaGrid &g, const float *delta,
                             float *dconv, hipStream_t s);
hipError_t launch_assa_adjoint(const gpair_plan_s *p, const AssaGrid &g, const float *dconv,
                               float *out, hipStream_t s);

// The full objective (objective.hip).
hipError_t launch_npc_map(int64_t n, const float *z, float eps, float *x, hipStream_t s);
hipError_t launch_npc_grad(int64_t n, const float *z, const float *gx, float eps, float *gz,
                           hipStream_t s);
size_t vcr_work_bytes(int32_t nx, int32_t ny, int32_t nz);
hipError_t launch_vcr(int32_t nx, int32_t ny, int32_t nz, const float *x, double beta,
                      double eps, double lambda, float *grad, double *value, void *work,
                      hipStream_t s);

// Workspace pointers of a bound plan.
inline double *ws_sens(const gpair_plan_s *p) { return (double *)(p->ws + p->lay.sens); }
inline int32_t *ws_perm(const gpair_plan_s *p) { return (int32_t *)(p->ws + p->lay.perm); }
inline TileInfo *ws_ftiles(const gpair_plan_s *p) { return (TileInfo *)(p->ws + p->lay.ftiles); }
inline TileInfo *ws_atiles(const gpair_plan_s *p) { return (TileInfo *)(p->ws + p->lay.atiles); }
inline KernelRec *ws_krec(const gpair_plan_s *p) { return (KernelRec *)(p->ws + p->lay.krec); }
inline unsigned long long *ws_counters(const gpair_plan_s *p) {
  return (unsigned long long *)(p->ws + p->lay.counters);
}
inline double *ws_partials(const gpair_plan_s *p) { return (double *)(p->ws + p->lay.partials); }
inline long long *ws_det(const gpair_plan_s *p) { return (long long *)(p->ws + p->lay.det); }

// Host planner (plan.cpp).
gpair_status build_plan(const gpair_geometry *g, gpair_plan_s *p);
// Exhaustive host check of the binning invariant over every (tile member,
// sensor) pair of the forward (which = 0) or adjoint (1) tiling.
gpair_status tiling_slots(const gpair_plan_s *p, int which, int64_t *min_first,
                          int64_t *max_last);
WorkspaceLayout layout_for(int64_t M, int32_t Nd, size_t nft, size_t nat, int64_t det_words);

}  // namespace gpair
