// aniso.hip -- gfx950 kernels of the direct operators for anisotropic
// Gaussian kernels (learnable anisotropic Gaussians: the future work named in
// the Discussion of arXiv 2602.03893).
//
// Kernel k has p0 = A_k exp(-(x - c_k)^T Sigma_k^-1 (x - c_k) / 2), Sigma_k
// given as six numbers (xx, yy, zz, xy, xz, yz).  Far field: the detector's
// sphere is taken as flat across the kernel (the same step that keeps only
// the outgoing term of Eq. (single_forward)), so the sphere integral of p0 is
// the kernel's marginal along n = (s - c)/r and Eq. (pa_wave) gives
//     p = A sqrt(det Sigma) / sigma_n^3 * d / (2r) * exp(-d^2 / (2 sigma_n^2)),
//     sigma_n^2 = n^T Sigma n,  d = r - v t,  kept inside |d| <= n_sigma sigma_n
// (Eq. (single_forward) exactly when Sigma = sigma^2 I).  The window depends
// on the pair through sigma_n: each pair goes through the isotropic
// operators' float32 filter (filter.h) extended by sigma_n, and a pair whose
// window end lies within the guard of a sample, or a block the planner keeps
// in float64, is decided in float64 as the definition (distance, sigma_n,
// first and last in-window sample).  Taps run in float32 with the same
// Gaussian recurrence as the isotropic operators.
//
// Forward: one workgroup per (forward tile, 64 sensors), lane = sensor, the
// waves take the tile's reference blocks in turn (wave-uniform kernel loop);
// taps go into the shared fixed-point LDS segment of the tile's time shell as
// in the isotropic forward (the same segment bounds hold since every sigma_n
// is at most sigma_max), then one float atomic per sample into y.
// Adjoint: one workgroup per adjoint tile, lane = kernel; per stage of 64
// sensors the residual over the tile's time shell is staged in LDS; per pair
// the lane gathers its taps.  float32 within a stage, float64 across stages.
// Gradient with respect to the six covariance parameters at fixed windows:
//   dp/dSigma = p [Sigma^-1 / 2 + (d^2 / (2 sigma_n^4) - 3 / (2 sigma_n^2)) n n^T],
// an off-diagonal parameter standing for both symmetric entries (twice the
// matrix entry).
#include <algorithm>
#include <cmath>

#include "filter.h"
#include "gpair_internal.h"

namespace gpair {
namespace {

// The 64-byte record as the anisotropic operators use it (rebuilt by their
// prep on every call; the geometry fields are shared with KernelRec).
struct alignas(64) AnisoRec {
  float dx, dy, dz, dd;                // geometry (unused here)
  float sxx, syy, szz, sxy, sxz, syz;  // covariance (m^2)
  float A;                             // amplitude
  float fcz;                           // geometry: float32 centre (z)
  float sq;                            // sqrt(det Sigma)
  float pk;                            // bound of |A| sqrt(det Sigma) / lambda_min; sign
                                       // bit set: every pair in float64 (ill-conditioned)
  float fcx, fcy;                      // geometry: float32 centre (x, y)
};
static_assert(sizeof(AnisoRec) == 64, "AnisoRec layout");
static_assert(offsetof(AnisoRec, fcz) == offsetof(KernelRec, fcz) &&
                  offsetof(AnisoRec, fcx) == offsetof(KernelRec, fcx) &&
                  offsetof(AnisoRec, fcy) == offsetof(KernelRec, fcy) &&
                  offsetof(AnisoRec, dd) == offsetof(KernelRec, dd),
              "shared geometry fields");

constexpr int kAnisoWaves = 4;   // forward waves per workgroup
constexpr int kTapRunAniso = 16; // taps between exact Gaussian factors
// Floats of LDS past the adjoint's stage: the unrolled gather (at most 18
// taps) reads its whole unrolled length from a window that starts inside its
// row, and masks what lies past the lane's own window.
constexpr int kAnisoStagePad = 32;
// Largest condition number lambda_max/lambda_min of a covariance whose pairs
// go through the float32 filter: sigma_n^2 from the float32 quadratic form is
// then within about 24 kappa float32 units (6e-6 relative at 2.5), which keeps
// the window ends inside the guard's margin and the taps near float32 accuracy.
constexpr double kAnisoFilterKappa = 2.5;

__device__ __forceinline__ int64_t xcd_logical_a(int64_t nlogical) {
  const int64_t per = (nlogical + kXcds - 1) / kXcds;
  const int64_t b = blockIdx.x;
  return (b % kXcds) * per + b / kXcds;
}

inline unsigned int xcd_grid_a(int64_t nlogical) {
  const int64_t per = (nlogical + kXcds - 1) / kXcds;
  return (unsigned int)(per * kXcds);
}

// ---------------------------------------------------------------------------
// Records: covariance checks, sqrt(det), the fixed-point bound factor.
// ---------------------------------------------------------------------------
// A covariance is admitted when it is symmetric positive definite (leading
// minors > 0) and smax2 I - Sigma is positive semidefinite (every principal
// minor >= 0), i.e. its largest eigenvalue is at most smax2.  Anything else
// is counted and replaced by smax2 I for that kernel.
__global__ __launch_bounds__(256) void aniso_prep_kernel(
    const float *__restrict__ A, const float *__restrict__ sig6,
    const int32_t *__restrict__ perm, AnisoRec *__restrict__ rec, int64_t M, double smax2,
    unsigned long long *viol) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int32_t k = perm[i];
  float s[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) s[c] = sig6[(int64_t)c * M + k];
  double xx = s[0], yy = s[1], zz = s[2], xy = s[3], xz = s[4], yz = s[5];
  double det = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
  const bool spd = xx > 0.0 && xx * yy - xy * xy > 0.0 && det > 0.0;
  // B = smax2 I - Sigma: its off-diagonal entries are -xy, -xz, -yz.
  const double bxx = smax2 - xx, byy = smax2 - yy, bzz = smax2 - zz;
  const double bdet =
      bxx * (byy * bzz - yz * yz) - xy * (xy * bzz + yz * xz) - xz * (xy * yz + byy * xz);
  const bool below = bxx >= 0.0 && byy >= 0.0 && bzz >= 0.0 && bxx * byy - xy * xy >= 0.0 &&
                     bxx * bzz - xz * xz >= 0.0 && byy * bzz - yz * yz >= 0.0 && bdet >= 0.0;
  if (!(spd && below)) {
    atomicAdd(viol, 1ULL);
    xx = yy = zz = smax2;
    xy = xz = yz = 0.0;
    det = smax2 * smax2 * smax2;
#pragma unroll
    for (int c = 0; c < 6; ++c) s[c] = c < 3 ? (float)smax2 : 0.0f;
  }
  const float a = A ? A[k] : 0.0f;
  const double sq = sqrt(det);
  const double tr = xx + yy + zz;
  // 1/lambda_min for the fixed-point bound: the closed-form (trigonometric)
  // smallest eigenvalue, lowered by 1e-6 and accepted only if Sigma - l I is
  // then positive semidefinite; otherwise (or when it would be looser) the
  // always valid tr^2 / (4 det) >= lambda_mid lambda_max / det = 1/lambda_min.
  double inv_lmin = tr * tr / (4.0 * det);
  double l1 = tr;  // largest eigenvalue (tr bounds it)
  {
    const double p1 = xy * xy + xz * xz + yz * yz;
    const double q = tr / 3.0;
    const double p2 = (xx - q) * (xx - q) + (yy - q) * (yy - q) + (zz - q) * (zz - q) + 2.0 * p1;
    double l3 = q;
    l1 = q;
    if (p2 > 0.0) {
      const double pp = sqrt(p2 / 6.0);
      const double b11 = (xx - q) / pp, b22 = (yy - q) / pp, b33 = (zz - q) / pp;
      const double b12 = xy / pp, b13 = xz / pp, b23 = yz / pp;
      double rr = 0.5 * (b11 * (b22 * b33 - b23 * b23) - b12 * (b12 * b33 - b23 * b13) +
                         b13 * (b12 * b23 - b22 * b13));
      rr = fmin(1.0, fmax(-1.0, rr));
      const double phi = acos(rr) / 3.0;
      l3 = q + 2.0 * pp * cos(phi + 2.0943951023931957);
      l1 = q + 2.0 * pp * cos(phi);
    }
    l1 *= 1.0 + 1e-6;
    const double l = l3 * (1.0 - 1e-6);
    const double cxx = xx - l, cyy = yy - l, czz = zz - l;
    const double cdet =
        cxx * (cyy * czz - yz * yz) - xy * (xy * czz - yz * xz) + xz * (xy * yz - cyy * xz);
    if (l > 0.0 && cxx >= 0.0 && cyy >= 0.0 && czz >= 0.0 && cxx * cyy - xy * xy >= 0.0 &&
        cxx * czz - xz * xz >= 0.0 && cyy * czz - yz * yz >= 0.0 && cdet >= 0.0)
      inv_lmin = fmin(inv_lmin, 1.0 / l);
  }
  AnisoRec &r = rec[i];
  r.sxx = s[0];
  r.syy = s[1];
  r.szz = s[2];
  r.sxy = s[3];
  r.sxz = s[4];
  r.syz = s[5];
  r.A = a;
  r.sq = (float)sq;
  // A kernel whose condition number exceeds kAnisoFilterKappa is decided in
  // float64 for every pair (its sign bit of pk set): the float32 quadratic form
  // u^T Sigma u loses about kappa float32 units of sigma_n^2 to cancellation,
  // which would break the filter's error bound and the taps' accuracy.
  const float pk = (float)(fabs((double)a) * sq * inv_lmin * (1.0 + 1e-6));
  r.pk = l1 * inv_lmin > kAnisoFilterKappa ? -pk : pk;
}

// sqrt(x) and 1/(2 sqrt(x)) for a positive normal float64 x: the float64
// reciprocal-square-root seed, one coupled Newton step on both and two
// corrections of the root (the sequence the compiler uses for sqrt, without
// its rescaling of tiny or huge inputs, which these distances never are).
__device__ __forceinline__ double sqrt_and_half_rinv(double x, double &h) {
  const double g = __builtin_amdgcn_rsq(x);
  double sr = x * g;
  h = 0.5 * g;
  const double e = fma(-h, sr, 0.5);
  sr = fma(sr, e, sr);
  h = fma(h, e, h);
  double d = fma(-sr, sr, x);
  sr = fma(d, h, sr);
  d = fma(-sr, sr, x);
  return fma(d, h, sr);
}

// One pair's window (slot of its first sample relative to the segment base,
// sample count, offset of that sample from the pulse centre) and its float32
// tap constants.
struct AnisoPair {
  int o;           // first in-window sample minus the segment base nb
  int ntap;        // in-window samples (>= 0)
  float d0;        // offset of sample o from the pulse centre, samples
  float rinv;      // 1/r
  float isn;       // 1/sigma_n (1/m)
  float nx, ny, nz;  // n = (s - c)/r (adjoint only)
};

// exp2(c u^2) = exp(-d^2/(2 sigma_n^2)) for u = d / Delta; the ratio of
// consecutive taps is exp2(k1 u + c), itself multiplied by rq each tap.
struct AnisoGauss {
  float c, k1, rq;
};

__device__ __forceinline__ AnisoGauss aniso_gauss(float isn, float vdt_f) {
  AnisoGauss g;
  const float iu = vdt_f * isn;  // Delta / sigma_n
  g.c = -0.72134752044448170f * iu * iu;  // -log2(e)/2 (Delta/sigma_n)^2
  g.k1 = -2.0f * g.c;
  g.rq = __builtin_amdgcn_exp2f(2.0f * g.c);
  return g;
}

// The float64 decision, as the definition: u = s - c from the caller's
// float32 centre, r, sigma_n^2 = u^T Sigma u / r^2 (clamped to smax2: the
// records admit no more, the clamp only absorbs rounding, so no window
// exceeds the plan's widest), the first and last sample with
// |r - v t| <= n_sigma sigma_n.
__device__ __forceinline__ void aniso_exact(const double4 &s, const AnisoRec &k, int nb,
                                            double inv_vdt, double t0_over_dt,
                                            double nsig_inv_vdt, double smax2, AnisoPair &p) {
  const double ux = s.x - (double)k.fcx, uy = s.y - (double)k.fcy, uz = s.z - (double)k.fcz;
  const double r2 = fma(uz, uz, fma(uy, uy, ux * ux));
  double hr;
  const double r = sqrt_and_half_rinv(r2, hr);
  const double rinv = 2.0 * hr;
  const double q = fma((double)k.sxx * ux, ux,
                   fma((double)k.syy * uy, uy,
                   fma((double)k.szz * uz, uz,
                       2.0 * fma((double)k.sxy * ux, uy,
                             fma((double)k.sxz * ux, uz, (double)k.syz * uy * uz)))));
  double sn2 = q * rinv * rinv;
  sn2 = (sn2 > 0.0 && sn2 <= smax2) ? sn2 : smax2;
  double hs_;
  const double sn = sqrt_and_half_rinv(sn2, hs_);
  const double hs = nsig_inv_vdt * sn;
  const double nc = fma(r, inv_vdt, -t0_over_dt);
  const double lo = ceil(nc - hs);
  const double hi = floor(nc + hs);
  p.o = (int)lo - nb;
  p.ntap = hi >= lo ? (int)(hi - lo) + 1 : 0;
  p.d0 = (float)(nc - lo);
  p.rinv = (float)rinv;
  p.isn = (float)(2.0 * hs_);
  p.nx = (float)(ux * rinv);
  p.ny = (float)(uy * rinv);
  p.nz = (float)(uz * rinv);
}

// The float32 filter from the block's constants (filter.h): dr = r - R by
// the block's fixed-point steps as in the isotropic operators, u = s - c_k =
// (s - c_B) - dk, sigma_n from u^T Sigma u and 1/r, then both window ends
// z -+ h_n about the pulse centre z (samples past Xi).  Returns true when an
// end lies within kGuard of a sample (then the caller decides with
// aniso_exact).  Its error is the isotropic filter's in z (below kGuard / 2 by
// the planner's bound) plus the float32 error of h_n, at most about 12 kappa
// float32 units of h_n <= h_max for kappa <= kAnisoFilterKappa (worse
// conditioned kernels never come here), so a decision outside the guard
// equals the float64 one.
__device__ __forceinline__ bool aniso_filter(const BlockLane &bl, int kit, const AnisoRec &k,
                                             float nsig_inv_vdt, float inv_vdt_f, float smax2f,
                                             AnisoPair &p) {
  const float D = fmaf(bl.m2ux, k.dx, fmaf(bl.m2uy, k.dy, fmaf(bl.m2uz, k.dz, k.dd)));
  float dr = D * bl.inv2R;
  for (int it = 0; it < kit; ++it) dr = fmaf(-dr, dr, D) * bl.inv2R;
  const float ux = fmaf(-0.5f, bl.m2ux, -k.dx);
  const float uy = fmaf(-0.5f, bl.m2uy, -k.dy);
  const float uz = fmaf(-0.5f, bl.m2uz, -k.dz);
  const float q = fmaf(k.sxx * ux, ux,
                  fmaf(k.syy * uy, uy,
                  fmaf(k.szz * uz, uz,
                       2.0f * fmaf(k.sxy * ux, uy, fmaf(k.sxz * ux, uz, k.syz * uy * uz)))));
  const float rinv = __builtin_amdgcn_rcpf(bl.Rf + dr);
  float sn2 = q * rinv * rinv;
  sn2 = (sn2 > 0.0f && sn2 <= smax2f) ? sn2 : smax2f;
  const float isn = __builtin_amdgcn_rsqf(sn2);
  const float hs = nsig_inv_vdt * (sn2 * isn);
  const float zc = fmaf(dr, inv_vdt_f, bl.Xf);
  const float zl = zc - hs, zh = zc + hs;
  const float cl = ceilf(zl), fh = floorf(zh);
  p.o = bl.Xi + (int)cl;
  p.ntap = fh >= cl ? (int)(fh - cl) + 1 : 0;
  p.d0 = zc - cl;
  p.rinv = rinv;
  p.isn = isn;
  p.nx = ux * rinv;
  p.ny = uy * rinv;
  p.nz = uz * rinv;
  const float m = fminf(fminf(cl - zl, zl + 1.0f - cl), fminf(zh - fh, fh + 1.0f - zh));
  return m < kGuard;
}

// ---------------------------------------------------------------------------
// Forward.
// ---------------------------------------------------------------------------
struct AnisoFwdArgs {
  const double4 *sens;
  const TileInfo *tiles;
  const TileInfo *blocks;  // adjoint tiles: the filter's reference blocks
  float *y;
  int64_t nlogical;
  int32_t ntiles, nblocks;
  int32_t Nd, Nt, nsg, L;
  double inv_vdt, t0_over_dt, hmax, vdt, nsig, smax2, min_dist;
  long long *y64;          // deterministic flush: int64 [Nd][Nt] in units of *det_unit
  const double *det_unit;  // the global unit (device), set before the launch
};

// Deterministic forward: the global unit G = 2^-62 e^{-1/2}/(2 min_dist)
// sum_k |pk_k| (a bound on every sample of y), from per-block partial sums
// reduced in a fixed order; then y = G y64.
__global__ __launch_bounds__(256) void aniso_det_partial_kernel(const AnisoRec *__restrict__ rec,
                                                               int64_t M, double *partials) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (int64_t)gridDim.x * 256)
    acc += fabs((double)rec[i].pk);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void aniso_det_unit_kernel(const double *partials, int nblocks, double scale,
                                      double *unit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double sum = 0.0;
  for (int b = 0; b < nblocks; ++b) sum += partials[b];
  *unit = sum * scale;
}

__global__ __launch_bounds__(256) void aniso_det_finish_kernel(const long long *__restrict__ y64,
                                                              const double *unit, float *y,
                                                              int64_t n) {
  const double G = *unit;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    y[i] = (float)((double)y64[i] * G);
}

// The largest n over the wave's active lanes when it is below 32 (31
// otherwise), by five ballots: no cross-lane data movement, and the result is
// wave-uniform.
__device__ __forceinline__ int wave_max_small(int n) {
  int m = 0;
#pragma unroll
  for (int b = 16; b > 0; b >>= 1)
    if (__ballot(n >= m + b) != 0) m += b;
  return m;
}

__device__ __forceinline__ void lds_add_fx(int *p, float v) {
  int n;
  asm volatile("v_cvt_rpi_i32_f32 %0, %1" : "=v"(n) : "v"(v));
  __hip_atomic_fetch_add(p, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The taps of one pair when the wave's longest window has NT samples (fully
// unrolled, compile-time LDS offsets): t_i = f_i u_i by the fused
// recurrence t_{i+1} = q_i t_i - f_{i+1}; the lane adds only its own n.
template <int NT>
__device__ __forceinline__ void aniso_taps(int *pa, float f, float q, float d, float rq, int n) {
  float tv = f * d;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    if (i < n) lds_add_fx(pa + i * kWave, tv);
    if (i + 1 < NT) {
      f *= q;
      tv = fmaf(q, tv, -f);
      q *= rq;
    }
  }
}

// The taps of one pair from a staged residual row (rp at the pair's first
// sample), unrolled for NT samples of which the lane's own n are read:
// s1 += delta e u, with S3 s3 += delta e u^3, with CEN s0 += delta e and
// s2 += delta e u^2 (u in samples, e by the ratio recurrence).
template <int NT, bool S3, bool CEN>
__device__ __forceinline__ void aniso_gather(const float *rp, float f, float q, float d, float rq,
                                             int n, float &s0, float &s1, float &s2, float &s3) {
  float dl[NT];
  // Every read stays in the stage: the window starts inside its row and the
  // stage carries kAnisoStagePad floats past its last row.
#pragma unroll
  for (int i = 0; i < NT; ++i) dl[i] = rp[i];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    if (i >= n) dl[i] = 0.0f;
    const float t = dl[i] * f;
    const float pd = t * d;
    s1 += pd;
    if (S3) s3 = fmaf(pd, d * d, s3);
    if (CEN) {
      s0 += t;
      s2 = fmaf(pd, d, s2);
    }
    d -= 1.0f;
    f *= q;
    q *= rq;
  }
}

template <int WAVES, bool DET>
__global__ __launch_bounds__(WAVES * kWave) void aniso_forward_kernel(
    const AnisoRec *__restrict__ rec, AnisoFwdArgs a) {
  extern __shared__ int seg[];  // [L][64]
  const int64_t logical = xcd_logical_a(a.nlogical);
  if (logical >= a.nlogical) return;
  const int64_t tile = logical / a.nsg;
  const int sg = (int)(logical - tile * a.nsg);
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int j = sg * kWave + lane;
  const double4 s = a.sens[j < a.Nd ? j : a.Nd - 1];
  const TileInfo T = a.tiles[tile];
  double R;
  {
    const double dx = s.x - T.cx, dy = s.y - T.cy, dz = s.z - T.cz;
    R = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
  }
  const int nb = (int)floor((R - T.rho) * a.inv_vdt - a.t0_over_dt - a.hmax) - 1;
  for (int i = t; i < a.L * kWave; i += WAVES * kWave) seg[i] = 0;

  // Fixed-point unit: every tap of kernel k at distance r is at most
  // pk_k e^{-1/2} / (2 r) in magnitude, so B = e^{-1/2}/(2 r_low) sum pk
  // bounds any sample's tile sum; every wave adds the same values in the same
  // order, so all waves use the same unit.
  float psum = 0.0f;
  for (int i = T.start + lane; i < T.start + T.count; i += kWave) psum += fabsf(rec[i].pk);
  for (int off = 32; off > 0; off >>= 1) psum += __shfl_xor(psum, off, kWave);
  const double r_low = fmax(R - T.rho, a.min_dist);
  const double bound = (double)psum * (1.0 + 1e-5) * 0.60653065971263342 / (2.0 * r_low);
  const float unit = (float)(bound * 0x1p-30);
  const double iuw = bound > 0.0 ? 0x1p30 / bound : 0.0;
  __syncthreads();

  // Slots: o >= 1 and o + ntap - 1 <= L - 1 for every pair (the plan's slot
  // bound with the widest admitted window, which no sigma_n exceeds); a lane
  // adds only its own window's taps while the wave runs to its longest.
  int *const col = seg + lane;
  const float wsc = (float)(0.5 * a.vdt * iuw);  // Delta/2 in fixed-point units
  const float vdt_f = (float)a.vdt, inv_vdt_f = (float)a.inv_vdt;
  const double nsig_inv_vdt = a.nsig * a.inv_vdt;
  const float nsig_inv_vdt_f = (float)nsig_inv_vdt, smax2f = (float)a.smax2;
  // The waves take the tile's reference blocks (the adjoint tiles nested in
  // it) in turn; each sets up its block's filter constants per lane.
  const int bend = tile + 1 < a.ntiles ? a.tiles[tile + 1].first_block : a.nblocks;
  for (int b = T.first_block + wave; b < bend; b += WAVES) {
    const TileInfo B = a.blocks[b];
    BlockLane bl;
    block_lane(s, B, nb, a.inv_vdt, a.t0_over_dt, bl);
    const int kit = B.filter_steps;
    for (int k = B.start; k < B.start + B.count; ++k) {
      const AnisoRec r = rec[k];
      AnisoPair p;
      if (kit < 0 || signbit(r.pk) || aniso_filter(bl, kit, r, nsig_inv_vdt_f, inv_vdt_f, smax2f, p))
        aniso_exact(s, r, nb, a.inv_vdt, a.t0_over_dt, nsig_inv_vdt, a.smax2, p);
      const AnisoGauss gs = aniso_gauss(p.isn, vdt_f);
      // p = A sq / sigma_n^3 * (u Delta) / (2r) * exp2(c u^2), u in samples
      const float w = r.A * r.sq * (p.isn * p.isn * p.isn) * wsc * p.rinv;
      int *const pa = col + p.o * kWave;
      const int n = p.ntap;
      const int nmax = wave_max_small(n);
      if (nmax <= 18) {
        const float f0 = w * __builtin_amdgcn_exp2f(gs.c * p.d0 * p.d0);
        const float q0 = __builtin_amdgcn_exp2f(fmaf(gs.k1, p.d0, gs.c));
        switch (nmax) {
#define GPAIR_ANISO_TAPS(k) \
  case k: aniso_taps<k>(pa, f0, q0, p.d0, gs.rq, n); break;
          GPAIR_ANISO_TAPS(1) GPAIR_ANISO_TAPS(2) GPAIR_ANISO_TAPS(3) GPAIR_ANISO_TAPS(4)
          GPAIR_ANISO_TAPS(5) GPAIR_ANISO_TAPS(6) GPAIR_ANISO_TAPS(7) GPAIR_ANISO_TAPS(8)
          GPAIR_ANISO_TAPS(9) GPAIR_ANISO_TAPS(10) GPAIR_ANISO_TAPS(11) GPAIR_ANISO_TAPS(12)
          GPAIR_ANISO_TAPS(13) GPAIR_ANISO_TAPS(14) GPAIR_ANISO_TAPS(15) GPAIR_ANISO_TAPS(16)
          GPAIR_ANISO_TAPS(17) GPAIR_ANISO_TAPS(18)
#undef GPAIR_ANISO_TAPS
          default: break;
        }
        continue;
      }
      // Longer windows: each lane runs its own count.
      for (int i0 = 0; i0 < n; i0 += kTapRunAniso) {
        const float d = p.d0 - (float)i0;
        float f = w * __builtin_amdgcn_exp2f(gs.c * d * d);
        float q = __builtin_amdgcn_exp2f(fmaf(gs.k1, d, gs.c));
        float tv = f * d;  // t_i = f_i u_i; t_{i+1} = q_i t_i - f_{i+1}
        const int iend = min(i0 + kTapRunAniso, n);
        for (int i = i0; i < iend; ++i) {
          lds_add_fx(pa + i * kWave, tv);
          f *= q;
          tv = fmaf(q, tv, -f);
          q *= gs.rq;
        }
      }
    }
  }
  __syncthreads();

  // Back to float32 (each lane's own unit; DET: kept as integers), row c
  // rotated by c columns, then one coalesced atomic per sample (as the
  // isotropic forward).
  for (int cr = wave; cr < a.L; cr += WAVES) {
    const int v = col[cr * kWave];
    seg[cr * kWave + ((lane + cr) & (kWave - 1))] = DET ? v : __float_as_int((float)v * unit);
  }
  __syncthreads();
  if (DET) {
    // Each sample's tile sum (an integer in units of bound 2^-30) goes to the
    // global unit G, rounded to the nearest integer, and is added with a
    // 64-bit integer atomic: the rounding depends only on the tile's own sum
    // and integer addition is exact, so y is the same bit for bit whatever the
    // order of the tiles.  G is 2^-62 of a bound on every sample of y.
    const double fac = bound * 0x1p-30 / *a.det_unit;
    for (int row = wave; row < kWave; row += WAVES) {
      const int jr = sg * kWave + row;
      if (jr >= a.Nd) break;
      const int nbr = __builtin_amdgcn_readlane(nb, row);
      const double fr = __shfl(fac, row, kWave);
      long long *yrow = a.y64 + (int64_t)jr * a.Nt;
      for (int cs = lane; cs < a.L; cs += kWave) {
        const int n = nbr + cs;
        const int v = seg[cs * kWave + ((row + cs) & (kWave - 1))];
        if (n >= 0 && n < a.Nt && v != 0)
          __hip_atomic_fetch_add(yrow + n, (long long)llrint((double)v * fr), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    return;
  }
  for (int row = wave; row < kWave; row += WAVES) {
    const int jr = sg * kWave + row;
    if (jr >= a.Nd) break;
    const int nbr = __builtin_amdgcn_readlane(nb, row);
    float *yrow = a.y + (int64_t)jr * a.Nt;
    for (int cs = lane; cs < a.L; cs += kWave) {
      const int n = nbr + cs;
      const float v = __int_as_float(seg[cs * kWave + ((row + cs) & (kWave - 1))]);
      if (n >= 0 && n < a.Nt && v != 0.0f) unsafeAtomicAdd(yrow + n, v);
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint.
// ---------------------------------------------------------------------------
struct AnisoAdjArgs {
  const AnisoRec *rec;
  const TileInfo *tiles;
  const int32_t *perm;
  const float *delta;
  float *gA;
  float *gS;  // [6][M] caller order, or null
  float *gC;  // [M][3] caller order (centre gradient), or null
  int64_t nlogical, M;
  int32_t Nd, Nt, L;
  double inv_vdt, t0_over_dt, hmax, vdt, nsig, smax2;
};

// SIGMA: also the covariance gradient; CENTRES: also the centre gradient,
// -sum delta (dp/dr n + dp/d(sigma_n^2) (2/r)(Sigma n - sigma_n^2 n)), whose
// direction terms are formed in float64 (Sigma n - sigma_n^2 n cancels by
// about the condition number of Sigma).
template <int BLOCK, bool SIGMA, bool CENTRES = false>
__global__ __launch_bounds__(BLOCK) void aniso_adjoint_kernel(const double4 *__restrict__ sens,
                                                              AnisoAdjArgs a) {
  extern __shared__ float stage[];  // [kAdjSensorsPerStage][L]
  __shared__ int nbs[kAdjSensorsPerStage];
  __shared__ float4 su[kAdjSensorsPerStage];  // -2u (x, y, z), 1/(2R)
  __shared__ float4 sv[kAdjSensorsPerStage];  // R, Xf, Xi (bits), unused

  const int64_t logical = xcd_logical_a(a.nlogical);
  if (logical >= a.nlogical) return;
  const TileInfo T = a.tiles[logical];
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  const int wave = t >> 6;
  const bool live = t < T.count;
  const int64_t i = T.start + (live ? t : 0);
  const AnisoRec r = a.rec[i];
  const int kit = T.filter_steps;
  const float vdt_f = (float)a.vdt, hvdt = 0.5f * (float)a.vdt, inv_vdt_f = (float)a.inv_vdt;
  const double nsig_inv_vdt = a.nsig * a.inv_vdt;
  const float nsig_inv_vdt_f = (float)nsig_inv_vdt, smax2f = (float)a.smax2;

  double accA = 0.0, accN[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double accC[3] = {0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < a.Nd; j0 += kAdjSensorsPerStage) {
    const int nsb = min(kAdjSensorsPerStage, a.Nd - j0);
    __syncthreads();  // the previous stage has been consumed
    if (t < nsb) {
      const double4 s = sens[j0 + t];
      const double dx = s.x - T.cx, dy = s.y - T.cy, dz = s.z - T.cz;
      const double R = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
      const int nb = (int)floor((R - T.rho) * a.inv_vdt - a.t0_over_dt - a.hmax) - 1;
      nbs[t] = nb;
      BlockLane bl;
      block_lane(s, T, nb, a.inv_vdt, a.t0_over_dt, bl);
      su[t] = make_float4(bl.m2ux, bl.m2uy, bl.m2uz, bl.inv2R);
      sv[t] = make_float4(bl.Rf, bl.Xf, __int_as_float(bl.Xi), 0.0f);
    }
    __syncthreads();
    for (int js = wave; js < nsb; js += BLOCK / kWave) {
      const float *drow = a.delta + (int64_t)(j0 + js) * a.Nt;
      const int nb = nbs[js];
      for (int c = lane; c < a.L; c += kWave) {
        const int n = nb + c;
        stage[js * a.L + c] = (n >= 0 && n < a.Nt) ? drow[n] : 0.0f;
      }
    }
    __syncthreads();

    float sA = 0.0f, sN[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int js = 0; js < nsb; ++js) {
      AnisoPair p;
      bool exact = kit < 0 || signbit(r.pk);
      if (!exact) {
        const float4 U = su[js];
        const float4 V = sv[js];
        BlockLane bl;
        bl.m2ux = U.x;
        bl.m2uy = U.y;
        bl.m2uz = U.z;
        bl.inv2R = U.w;
        bl.Rf = V.x;
        bl.Xf = V.y;
        bl.Xi = __float_as_int(V.z);
        exact = aniso_filter(bl, kit, r, nsig_inv_vdt_f, inv_vdt_f, smax2f, p);
      }
      if (exact)
        aniso_exact(sens[j0 + js], r, nbs[js], a.inv_vdt, a.t0_over_dt, nsig_inv_vdt, a.smax2, p);
      const AnisoGauss gs = aniso_gauss(p.isn, vdt_f);
      const float *rp = stage + js * a.L + p.o;
      // In samples: s0 = sum delta e, s1 = sum delta u e, s2 = sum delta u^2 e,
      // s3 = sum delta u^3 e.
      float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
      const int nmax = wave_max_small(p.ntap);
      if (nmax <= 18) {
        // Unrolled for the wave's longest window, each lane masked to its own.
        const float f0 = __builtin_amdgcn_exp2f(gs.c * p.d0 * p.d0);
        const float q0 = __builtin_amdgcn_exp2f(fmaf(gs.k1, p.d0, gs.c));
        switch (nmax) {
#define GPAIR_ANISO_GATHER(k)                                                          \
  case k:                                                                              \
    aniso_gather<k, SIGMA || CENTRES, CENTRES>(rp, f0, q0, p.d0, gs.rq, p.ntap, s0, s1, \
                                               s2, s3);                                \
    break;
          GPAIR_ANISO_GATHER(1) GPAIR_ANISO_GATHER(2) GPAIR_ANISO_GATHER(3)
          GPAIR_ANISO_GATHER(4) GPAIR_ANISO_GATHER(5) GPAIR_ANISO_GATHER(6)
          GPAIR_ANISO_GATHER(7) GPAIR_ANISO_GATHER(8) GPAIR_ANISO_GATHER(9)
          GPAIR_ANISO_GATHER(10) GPAIR_ANISO_GATHER(11) GPAIR_ANISO_GATHER(12)
          GPAIR_ANISO_GATHER(13) GPAIR_ANISO_GATHER(14) GPAIR_ANISO_GATHER(15)
          GPAIR_ANISO_GATHER(16) GPAIR_ANISO_GATHER(17) GPAIR_ANISO_GATHER(18)
#undef GPAIR_ANISO_GATHER
          default: break;
        }
      }
      for (int i0 = nmax <= 18 ? p.ntap : 0; i0 < p.ntap; i0 += kTapRunAniso) {
        float d = p.d0 - (float)i0;
        float f = __builtin_amdgcn_exp2f(gs.c * d * d);
        float q = __builtin_amdgcn_exp2f(fmaf(gs.k1, d, gs.c));
        const int iend = min(i0 + kTapRunAniso, p.ntap);
        for (int ii = i0; ii < iend; ++ii) {
          const float t = rp[ii] * f;
          const float pd = t * d;
          s1 += pd;
          if (SIGMA || CENTRES) s3 = fmaf(pd, d * d, s3);
          if (CENTRES) {
            s0 += t;
            s2 = fmaf(pd, d, s2);
          }
          d -= 1.0f;
          f *= q;
          q *= gs.rq;
        }
      }
      // W = sqrt(det) / sigma_n^3 * Delta / (2r): gA += W s1
      const float W = r.sq * (p.isn * p.isn * p.isn) * hvdt * p.rinv;
      sA = fmaf(W, s1, sA);
      const float iu = vdt_f * p.isn;
      // W / (2 sigma_n^2) (s3 (Delta/sigma_n)^2 - 3 s1): the sigma_n^2 factor
      const float G = W * 0.5f * (p.isn * p.isn) * fmaf(s3, iu * iu, -3.0f * s1);
      if (CENTRES) {
        // dp/dr part: A sqrt(det)/sigma_n^3/(2r) (s0 - (Delta/sigma_n)^2 s2 - (Delta/r) s1)
        const float dpr = r.A * W * inv_vdt_f *
                          (s0 - iu * iu * s2 - vdt_f * p.rinv * s1);
        const double dps = (double)r.A * (double)G;
        const double4 sj = sens[j0 + js];
        const double ux = sj.x - (double)r.fcx, uy = sj.y - (double)r.fcy,
                     uz = sj.z - (double)r.fcz;
        double hr;
        sqrt_and_half_rinv(fma(uz, uz, fma(uy, uy, ux * ux)), hr);
        const double ri = 2.0 * hr;
        const double nx = ux * ri, ny = uy * ri, nz = uz * ri;
        const double Snx = fma((double)r.sxx, nx, fma((double)r.sxy, ny, (double)r.sxz * nz));
        const double Sny = fma((double)r.sxy, nx, fma((double)r.syy, ny, (double)r.syz * nz));
        const double Snz = fma((double)r.sxz, nx, fma((double)r.syz, ny, (double)r.szz * nz));
        const double sn2 = fma(nx, Snx, fma(ny, Sny, nz * Snz));
        const double f2 = dps * 2.0 * ri;
        accC[0] -= fma((double)dpr, nx, f2 * fma(-sn2, nx, Snx));
        accC[1] -= fma((double)dpr, ny, f2 * fma(-sn2, ny, Sny));
        accC[2] -= fma((double)dpr, nz, f2 * fma(-sn2, nz, Snz));
      }
      if (SIGMA) {
        // G along n n^T
        sN[0] = fmaf(G * p.nx, p.nx, sN[0]);
        sN[1] = fmaf(G * p.ny, p.ny, sN[1]);
        sN[2] = fmaf(G * p.nz, p.nz, sN[2]);
        sN[3] = fmaf(G * p.nx, p.ny, sN[3]);
        sN[4] = fmaf(G * p.nx, p.nz, sN[4]);
        sN[5] = fmaf(G * p.ny, p.nz, sN[5]);
      }
    }
    accA += (double)sA;
    if (SIGMA) {
#pragma unroll
      for (int c = 0; c < 6; ++c) accN[c] += (double)sN[c];
    }
  }
  if (!live) return;
  const int32_t k = a.perm[i];
  a.gA[k] = (float)accA;
  if (CENTRES) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.gC[3 * (int64_t)k + c] = (float)accC[c];
  }
  if (SIGMA) {
    const double xx = r.sxx, yy = r.syy, zz = r.szz, xy = r.sxy, xz = r.sxz, yz = r.syz;
    const double det = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
    const double inv[6] = {(yy * zz - yz * yz) / det, (xx * zz - xz * xz) / det,
                           (xx * yy - xy * xy) / det, (xz * yz - xy * zz) / det,
                           (xy * yz - xz * yy) / det, (xy * xz - xx * yz) / det};
    const double A = r.A, h = 0.5 * A * accA;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double g = h * inv[c] + A * accN[c];
      a.gS[(int64_t)c * a.M + k] = (float)(c < 3 ? g : 2.0 * g);
    }
  }
}

}  // namespace

hipError_t launch_aniso_prep(const gpair_plan_s *p, const float *A, const float *sig6,
                             hipStream_t s) {
  const int64_t M = p->M;
  const double smax = p->sigma_max * (1.0 + 1e-6);
  aniso_prep_kernel<<<(unsigned int)((M + 255) / 256), 256, 0, s>>>(
      A, sig6, ws_perm(p), (AnisoRec *)ws_krec(p), M, smax * smax, ws_counters(p));
  return hipGetLastError();
}

hipError_t launch_aniso_forward(const gpair_plan_s *p, float *y, hipStream_t s) {
  AnisoFwdArgs a;
  a.sens = (const double4 *)ws_sens(p);
  a.tiles = ws_ftiles(p);
  a.blocks = ws_atiles(p);
  a.y = y;
  a.ntiles = (int32_t)p->host.ftiles.size();
  a.nblocks = (int32_t)p->host.atiles.size();
  a.Nd = p->Nd;
  a.Nt = p->Nt;
  a.nsg = (p->Nd + kWave - 1) / kWave;
  a.nlogical = (int64_t)p->host.ftiles.size() * a.nsg;
  a.L = p->Lf;
  a.inv_vdt = p->inv_vdt;
  a.t0_over_dt = p->t0_over_dt;
  a.hmax = p->hmax;
  a.vdt = p->vdt;
  a.nsig = p->nsig;
  const double smax = p->sigma_max * (1.0 + 1e-6);
  a.smax2 = smax * smax;
  a.min_dist = p->min_dist;
  a.y64 = nullptr;
  a.det_unit = nullptr;
  const size_t lds = (size_t)p->Lf * kWave * sizeof(int);
  const unsigned int grid = xcd_grid_a(a.nlogical);
  const AnisoRec *rec = (const AnisoRec *)ws_krec(p);
  if (!p->deterministic) {
    aniso_forward_kernel<kAnisoWaves, false><<<grid, kAnisoWaves * kWave, lds, s>>>(rec, a);
    return hipGetLastError();
  }
  const int64_t n = (int64_t)p->Nd * p->Nt;
  a.y64 = ws_det(p);
  double *unit = (double *)(a.y64 + n);
  double *partials = ws_partials(p);
  aniso_det_partial_kernel<<<kResidualBlocks, 256, 0, s>>>(rec, p->M, partials);
  aniso_det_unit_kernel<<<1, 64, 0, s>>>(
      partials, kResidualBlocks, (1.0 + 1e-5) * 0.60653065971263342 / (2.0 * p->min_dist) * 0x1p-62,
      unit);
  a.det_unit = unit;
  hipError_t e = launch_fill((float *)a.y64, 2 * n, 0.0f, s);  // int64 zero = two float zeros
  if (e != hipSuccess) return e;
  aniso_forward_kernel<kAnisoWaves, true><<<grid, kAnisoWaves * kWave, lds, s>>>(rec, a);
  aniso_det_finish_kernel<<<(unsigned int)std::min<int64_t>((n + 255) / 256, 16384), 256, 0, s>>>(
      a.y64, a.det_unit, y, n);
  return hipGetLastError();
}

hipError_t launch_aniso_adjoint(const gpair_plan_s *p, const float *delta, float *gA,
                                float *gsig6, float *gcentres, hipStream_t s) {
  AnisoAdjArgs a;
  a.rec = (const AnisoRec *)ws_krec(p);
  a.tiles = ws_atiles(p);
  a.perm = ws_perm(p);
  a.delta = delta;
  a.gA = gA;
  a.gS = gsig6;
  a.gC = gcentres;
  a.nlogical = (int64_t)p->host.atiles.size();
  a.M = p->M;
  a.Nd = p->Nd;
  a.Nt = p->Nt;
  a.L = p->La;
  a.inv_vdt = p->inv_vdt;
  a.t0_over_dt = p->t0_over_dt;
  a.hmax = p->hmax;
  a.vdt = p->vdt;
  a.nsig = p->nsig;
  const double smax = p->sigma_max * (1.0 + 1e-6);
  a.smax2 = smax * smax;
  const size_t lds = ((size_t)p->La * kAdjSensorsPerStage + kAnisoStagePad) * sizeof(float);
  const unsigned int grid = xcd_grid_a(a.nlogical);
  const double4 *sens = (const double4 *)ws_sens(p);
#define GPAIR_ANISO_ADJ(B)                                                                 \
  if (gcentres && gsig6)                                                                   \
    aniso_adjoint_kernel<B, true, true><<<grid, B, lds, s>>>(sens, a);                     \
  else if (gcentres)                                                                       \
    aniso_adjoint_kernel<B, false, true><<<grid, B, lds, s>>>(sens, a);                    \
  else if (gsig6)                                                                          \
    aniso_adjoint_kernel<B, true><<<grid, B, lds, s>>>(sens, a);                           \
  else                                                                                     \
    aniso_adjoint_kernel<B, false><<<grid, B, lds, s>>>(sens, a);
  switch (p->adj_tile) {
    case 64: GPAIR_ANISO_ADJ(64) break;
    case 128: GPAIR_ANISO_ADJ(128) break;
    default: GPAIR_ANISO_ADJ(256) break;
  }
#undef GPAIR_ANISO_ADJ
  return hipGetLastError();
}

}  // namespace gpair
