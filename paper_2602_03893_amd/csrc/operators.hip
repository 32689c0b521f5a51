// operators.hip -- gfx950 kernels of the direct GPAIR operators.
//
// Forward (arXiv 2602.03893, Eq. (single_forward) summed over kernels, inside
// the n_sigma window that follows it):
//   y_j[n] = sum_k [|d| <= n_sigma sigma_k] A_k/(2 r_jk) d exp(-d^2/(2 sigma_k^2)),
//   d = r_jk - v (t0 + n dt).
// Adjoint: its transpose, plus the sigma-derivative of Eq. (single_forward).
//
// Work decomposition (VALU-bound; no MFMA: nothing here is a contraction).
//  * Pair stage.  A kernel k of reference block B (an adjoint tile, of
//    float32-rounded centre c_B) at offset dk = c_k - c_B, seen from sensor s
//    with u = s - c_B and R = |u| (float64, once per block and sensor), has
//    r^2 - R^2 = D = |dk|^2 - 2 u.dk, so its distance offset dr = r - R
//    solves dr = (D - dr^2) / (2R): a few float32 fixed-point steps from
//    dr = D / (2R), converging by a factor ~rho_B/R per step.  The pulse
//    position in samples relative to the segment base, z = X + dr/(v dt) - h
//    (X = R/(v dt) - t0/dt - nb, split into an integer and a float32
//    fraction), then gives the first in-window sample (ceil z) and the
//    first tap's offset from the pulse centre.  This is the float32 window
//    filter.  Its error is bounded at set-up (block_lane) below half of
//    kGuard; a pair whose z lies within kGuard of a decision boundary (an
//    integer, or the last tap's threshold) is decided again from the
//    caller's float32 coordinates in float64, exactly as the float64
//    reference does, so window membership is the float64 decision.  Blocks
//    too close to a sensor for the bound use the float64 decision for every
//    pair.
//  * Tap stage, float32, offsets in samples: u_i = u_0 - i, and the
//    Gaussian factor by the exact recurrence e_{i+1} = e_i q_i,
//    q_{i+1} = q_i rq, so a pair costs two v_exp_f32 instead of one per tap
//    (windows longer than 18 taps re-evaluate e and q every 16 taps, since
//    the rounding of tap i grows like i^2).
//  * Forward: one workgroup = one tile of kernels x 64 sensors; lane = sensor,
//    the kernel loop is wave-uniform (kernel data in scalar registers) and the
//    workgroup's waves take the tile's reference blocks.  The waves share one
//    LDS trace segment per sensor over the tile's time shell, into which taps
//    go as 32-bit fixed-point integer adds (ds_add_u32 issues without
//    waiting, where a float add or a read-modify-write waits for LDS every
//    tap).  The fixed-point unit is per sensor: 2^-30 of a bound on any sum
//    the tile can put into one sample (sum_k |A_k| * sigma_max e^{-1/2} /
//    (2 r_low)), so no sum can overflow and each tap is rounded to 2^-31 of
//    that bound.  At the end the segment goes back to float32 and is added
//    to y with one coalesced float atomic per sample (tile-sensor partial
//    sums).
//  * Adjoint: one workgroup = one tile of kernels; lane = kernel, the sensor
//    loop is uniform.  For each stage of 64 sensors the residual over the
//    tile's time shell and the filter's per-sensor constants are staged in
//    LDS; every lane gathers its taps from it.  Per-lane sums go from float32
//    (within a stage) to float64 (across stages); no atomics.
//  * Blocks are remapped so that each of the 8 XCDs works on a contiguous
//    range of tiles (its L2 then holds that region's kernel records and the
//    matching residual rows).
#include <climits>

#include "filter.h"
#include "gpair_internal.h"

namespace gpair {
namespace {

constexpr double kLog2e = 1.4426950408889634074;

__device__ __forceinline__ int64_t xcd_logical_block(int64_t nlogical) {
  const int64_t per = (nlogical + kXcds - 1) / kXcds;
  const int64_t b = blockIdx.x;
  return (b % kXcds) * per + b / kXcds;
}

inline unsigned int xcd_grid(int64_t nlogical) {
  const int64_t per = (nlogical + kXcds - 1) / kXcds;
  return (unsigned int)(per * kXcds);
}

__device__ __forceinline__ int wave_min(int x) {
  for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off, kWave));
  return x;
}
__device__ __forceinline__ int wave_max(int x) {
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, kWave));
  return x;
}

// ---------------------------------------------------------------------------
// Per-call coefficient records (permuted order).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prep_kernel(
    const float *__restrict__ A, const float *__restrict__ sigma,
    const int32_t *__restrict__ perm, KernelRec *__restrict__ rec, int64_t M,
    double vdt, double nsig, double smax_eff, unsigned long long *viol) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int32_t k = perm[i];
  const float a = A ? A[k] : 0.0f;
  double s = (double)sigma[k];
  if (!(s > 0.0 && s <= smax_eff)) {
    atomicAdd(viol, 1ULL);
    s = (s > smax_eff) ? smax_eff : ((s > 0.0) ? s : smax_eff);
  }
  const double su = s / vdt;                // sigma in samples
  const double c = -kLog2e / (2.0 * su * su);
  const double h = nsig * su;
  const int32_t ntap = (int32_t)floor(2.0 * h) + 1;
  KernelRec &r = rec[i];  // the geometry fields were written at plan binding
  r.hf = (float)h;
  r.H = (float)((double)(ntap - 1) - 2.0 * h);
  r.amp = a;
  r.c = (float)c;
  r.k1 = (float)(-2.0 * c);
  r.rq = (float)exp2(2.0 * c);
  r.ntap = ntap;
  r.h = h;
}

// ---------------------------------------------------------------------------
// Pair stage shared by both operators.
// ---------------------------------------------------------------------------
// One pair's window: first tap's slot o (relative to the segment base nb),
// offset d0 of the first tap from the pulse centre (samples, in (h-1, h]),
// whether tap ntap-1 is in the window, and 1/r.
struct PairW {
  float d0;
  float rinv;
  int o;
  bool last_ok;
};

// The float32 filter in three parts: D = r^2 - R^2 from the record's offset
// dk = c - c_B and |dk|^2 (dx, dy, dz, dd); kit fixed-point steps of
// dr = (D - dr^2)/(2R) towards r - R; the window from dr.  The last returns
// true when a decision is within kGuard of its boundary (then the caller
// decides again with pair_exact).
__device__ __forceinline__ float filter_D(const BlockLane &bl, float dx, float dy, float dz,
                                          float dd) {
  return fmaf(bl.m2ux, dx, fmaf(bl.m2uy, dy, fmaf(bl.m2uz, dz, dd)));
}

__device__ __forceinline__ bool filter_window(const BlockLane &bl, float dr, float hf, float H,
                                              float inv_vdt_f, PairW &p) {
  const float zf = fmaf(dr, inv_vdt_f, bl.Xf - hf);
  const float cz = ceilf(zf);
  const float e = zf - cz;  // in (-1, 0]
  p.o = bl.Xi + (int)cz;
  p.d0 = e + hf;
  p.last_ok = e >= H;
  p.rinv = __builtin_amdgcn_rcpf(bl.Rf + dr);
  const float m = fminf(fminf(fabsf(e), fabsf(e + 1.0f)), fabsf(e - H));
  return m < kGuard;
}

__device__ __forceinline__ bool pair_filter(const BlockLane &bl, int kit, float dx, float dy,
                                            float dz, float dd, float hf, float H,
                                            float inv_vdt_f, PairW &p) {
  const float D = filter_D(bl, dx, dy, dz, dd);
  float dr = D * bl.inv2R;
  for (int it = 0; it < kit; ++it) dr = fmaf(-dr, dr, D) * bl.inv2R;
  return filter_window(bl, dr, hf, H, inv_vdt_f, p);
}

// The float64 decision: r from the caller's float32 coordinates, the first
// in-window sample lo = ceil((r - v t0)/(v dt) - h), as in the reference
// definition.  RINV: also set 1/r (otherwise the filter's value is kept).
template <bool RINV>
__device__ __forceinline__ void pair_exact(const double4 &s, float fcx, float fcy, float fcz,
                                           double h, int ntap, int nb, double inv_vdt,
                                           double t0_over_dt, PairW &p) {
  const double ex = s.x - (double)fcx, ey = s.y - (double)fcy, ez = s.z - (double)fcz;
  const double r = sqrt(fma(ez, ez, fma(ey, ey, ex * ex)));
  const double nc = fma(r, inv_vdt, -t0_over_dt);
  const double lo = ceil(nc - h);
  const double fr = nc - lo;
  p.o = (int)lo - nb;
  p.d0 = (float)fr;
  p.last_ok = fr >= (double)(ntap - 1) - h;
  if (RINV) p.rinv = (float)(1.0 / r);
}

// ---------------------------------------------------------------------------
// Forward.
// ---------------------------------------------------------------------------
// Everything the tap loop of one kernel-sensor pair needs.
struct Taps {
  float w;       // A / (2 r) Delta, in fixed-point units
  float f;       // w * exp2(c d0^2)
  float q;       // ratio of the second tap's Gaussian factor to the first's
  float d;       // d0 (samples)
  int o;         // first tap's slot in the lane's segment
  bool last_ok;  // tap ntap-1 is inside the window
};

struct FwdLoop {
  const KernelRec *krec;
  double4 s;
  BlockLane bl;
  int kit, nb;
  double inv_vdt, t0_over_dt;
  float inv_vdt_f;
  float iuw;  // fixed-point units per unit of A/r d/Delta: 2^30/B * Delta/2
};

// The tap setup of one pair from its window.
__device__ __forceinline__ Taps taps_of(const FwdLoop &c, const KernelRec &r, const PairW &p) {
  Taps t;
  t.d = p.d0;
  t.o = p.o;
  t.last_ok = p.last_ok;
  t.w = (p.rinv * r.amp) * c.iuw;
  t.f = t.w * __builtin_amdgcn_exp2f(r.c * t.d * t.d);
  t.q = __builtin_amdgcn_exp2f(fmaf(r.k1, t.d, r.c));
  return t;
}

template <bool EXACT>
__device__ __forceinline__ Taps pair_taps(const FwdLoop &c, const KernelRec &r) {
  PairW p;
  if (EXACT) {
    pair_exact<true>(c.s, r.fcx, r.fcy, r.fcz, r.h, r.ntap, c.nb, c.inv_vdt, c.t0_over_dt, p);
  } else if (pair_filter(c.bl, c.kit, r.dx, r.dy, r.dz, r.dd, r.hf, r.H, c.inv_vdt_f, p)) {
    pair_exact<false>(c.s, r.fcx, r.fcy, r.fcz, r.h, r.ntap, c.nb, c.inv_vdt, c.t0_over_dt, p);
  }
  return taps_of(c, r, p);
}

// Two pairs at once: the filter's steps of both run in one loop.
template <bool EXACT>
__device__ __forceinline__ void pair_taps2(const FwdLoop &c, const KernelRec &ra,
                                           const KernelRec &rb, Taps &ta, Taps &tb) {
  if (EXACT) {
    ta = pair_taps<true>(c, ra);
    tb = pair_taps<true>(c, rb);
    return;
  }
  const float Da = filter_D(c.bl, ra.dx, ra.dy, ra.dz, ra.dd);
  const float Db = filter_D(c.bl, rb.dx, rb.dy, rb.dz, rb.dd);
  float dra = Da * c.bl.inv2R, drb = Db * c.bl.inv2R;
  for (int it = 0; it < c.kit; ++it) {
    dra = fmaf(-dra, dra, Da) * c.bl.inv2R;
    drb = fmaf(-drb, drb, Db) * c.bl.inv2R;
  }
  PairW pa, pb;
  if (filter_window(c.bl, dra, ra.hf, ra.H, c.inv_vdt_f, pa))
    pair_exact<false>(c.s, ra.fcx, ra.fcy, ra.fcz, ra.h, ra.ntap, c.nb, c.inv_vdt, c.t0_over_dt,
                      pa);
  if (filter_window(c.bl, drb, rb.hf, rb.H, c.inv_vdt_f, pb))
    pair_exact<false>(c.s, rb.fcx, rb.fcy, rb.fcz, rb.h, rb.ntap, c.nb, c.inv_vdt, c.t0_over_dt,
                      pb);
  ta = taps_of(c, ra, pa);
  tb = taps_of(c, rb, pb);
}

// Add v (in fixed-point units) to an LDS word, rounded half up with one
// instruction (floor(v + 1/2) then convert; the compiler emits three).
__device__ __forceinline__ void lds_add(int *p, float v) {
  int n;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(n) : "v"(v));
  __hip_atomic_fetch_add(p, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Add the taps of one kernel-sensor pair into the lane's segment column p
// (stride 64 words), f already in fixed-point units: NT samples, of which the
// first ntap - 1 are inside the window and tap ntap - 1 is inside iff last_ok.
// The kernel's tap count ntap (wave-uniform) lies in NT - SPREAD .. NT, so
// only the last SPREAD + 1 samples can be outside: taps from ntap on by a
// uniform test, tap ntap - 1 by the lane's own.
template <int NT, int SPREAD>
__device__ __forceinline__ void taps_add(int *p, float f, float q, float d, float rq, int ntap,
                                         bool last_ok) {
  // t_i = f_i u_i with u_{i+1} = u_i - 1, f_{i+1} = f_i q_i: then
  // t_{i+1} = q_i t_i - f_{i+1}, one fused multiply-add per tap.
  float t[NT];
  t[0] = f * d;
#pragma unroll
  for (int i = 0; i + 1 < NT; ++i) {
    f *= q;
    t[i + 1] = fmaf(q, t[i], -f);
    q *= rq;
  }
  if (SPREAD == 0) {
    if (!last_ok) t[NT - 1] = 0.0f;
  } else {
#pragma unroll
    for (int i = (NT - 1 - SPREAD > 0 ? NT - 1 - SPREAD : 0); i < NT; ++i) {
      const bool inside = i < ntap - 1 || (i == ntap - 1 && last_ok);
      if (!inside) t[i] = 0.0f;
    }
  }
#pragma unroll
  for (int i = 0; i < NT; ++i) lds_add(p + i * kWave, t[i]);
}

// The recurrence of a tap loop runs at most this many taps from exactly
// evaluated factors: the relative error of tap i grows like i^2/2 float32
// roundings (about 1e-5 after 18 taps, 7e-5 after 48).
constexpr int kTapRun = 16;

// Taps of one pair whose tap count n is wave-uniform but not known at compile
// time: a scalar branch to the unrolled form; beyond 18 taps a loop that
// re-evaluates the Gaussian factors every kTapRun taps (rec: the pair's
// record, read again only there).
__device__ __forceinline__ void taps_add_n(int n, int *p, const Taps &t, float rq,
                                           const KernelRec *rec) {
  switch (n) {
#define GPAIR_TAPS_CASE(k) \
  case k: taps_add<k, 0>(p, t.f, t.q, t.d, rq, k, t.last_ok); return;
    GPAIR_TAPS_CASE(1) GPAIR_TAPS_CASE(2) GPAIR_TAPS_CASE(3) GPAIR_TAPS_CASE(4)
    GPAIR_TAPS_CASE(5) GPAIR_TAPS_CASE(6) GPAIR_TAPS_CASE(7) GPAIR_TAPS_CASE(8)
    GPAIR_TAPS_CASE(9) GPAIR_TAPS_CASE(10) GPAIR_TAPS_CASE(11) GPAIR_TAPS_CASE(12)
    GPAIR_TAPS_CASE(13) GPAIR_TAPS_CASE(14) GPAIR_TAPS_CASE(15) GPAIR_TAPS_CASE(16)
    GPAIR_TAPS_CASE(17) GPAIR_TAPS_CASE(18)
#undef GPAIR_TAPS_CASE
    default: break;
  }
  const float c = rec->c, k1 = rec->k1;
  const int nvalid = n - (t.last_ok ? 0 : 1);
  for (int i0 = 0; i0 < n; i0 += kTapRun) {
    float d = t.d - (float)i0;
    float f = t.w * __builtin_amdgcn_exp2f(c * d * d);
    float q = __builtin_amdgcn_exp2f(fmaf(k1, d, c));
    const int iend = min(i0 + kTapRun, n);
    for (int i = i0; i < iend; ++i) {
      lds_add(p + i * kWave, i < nvalid ? f * d : 0.0f);
      d -= 1.0f;
      f *= q;
      q *= rq;
    }
  }
}

// The kernel loop of one wave over records [k0, kend) of one reference
// block when every kernel of the tile has NT - SPREAD .. NT taps.  Kernels go
// in pairs: both pair stages sit in one straight-line block, so their chains
// interleave, and the records of the next pair are fetched meanwhile
// (clamped to the last record).
template <int NT, int SPREAD, bool EXACT>
__device__ __forceinline__ void kernel_loop(const FwdLoop &c, int *col, int k0, int kend) {
  if (k0 >= kend) return;
  const int last = kend - 1;
  const int pend = k0 + ((kend - k0) & ~1);
  KernelRec ra = c.krec[k0], rb = c.krec[min(k0 + 1, last)];
  for (int k = k0; k < pend; k += 2) {
    Taps ta, tb;
    pair_taps2<EXACT>(c, ra, rb, ta, tb);
    const float rqa = ra.rq, rqb = rb.rq;
    const int na = ra.ntap, nb = rb.ntap;
    ra = c.krec[min(k + 2, last)];
    rb = c.krec[min(k + 3, last)];
    taps_add<NT, SPREAD>(col + ta.o * kWave, ta.f, ta.q, ta.d, rqa, na, ta.last_ok);
    taps_add<NT, SPREAD>(col + tb.o * kWave, tb.f, tb.q, tb.d, rqb, nb, tb.last_ok);
  }
  if (pend < kend) {
    const Taps t = pair_taps<EXACT>(c, ra);
    taps_add<NT, SPREAD>(col + t.o * kWave, t.f, t.q, t.d, ra.rq, ra.ntap, t.last_ok);
  }
}

// The same loop for a tile whose kernels differ in width by more than two
// taps: each pair branches on its own tap count.
template <bool EXACT>
__device__ __forceinline__ void kernel_loop_mixed(const FwdLoop &c, int *col, int k0,
                                                  int kend) {
  if (k0 >= kend) return;
  const int last = kend - 1;
  const int pend = k0 + ((kend - k0) & ~1);
  KernelRec ra = c.krec[k0], rb = c.krec[min(k0 + 1, last)];
  for (int k = k0; k < pend; k += 2) {
    const Taps ta = pair_taps<EXACT>(c, ra);
    const Taps tb = pair_taps<EXACT>(c, rb);
    const float rqa = ra.rq, rqb = rb.rq;
    const int na = ra.ntap, nb = rb.ntap;
    ra = c.krec[min(k + 2, last)];
    rb = c.krec[min(k + 3, last)];
    taps_add_n(na, col + ta.o * kWave, ta, rqa, c.krec + k);
    taps_add_n(nb, col + tb.o * kWave, tb, rqb, c.krec + min(k + 1, last));
  }
  if (pend < kend) {
    const Taps t = pair_taps<EXACT>(c, ra);
    taps_add_n(ra.ntap, col + t.o * kWave, t, ra.rq, c.krec + pend);
  }
}

template <bool EXACT>
__device__ __forceinline__ void block_loops(const FwdLoop &c, int *col, int k0, int k1,
                                            int nt_unrolled, int spread) {
  switch (nt_unrolled) {
#define GPAIR_FWD_CASE(n)                                                      \
  case n:                                                                      \
    if (spread == 0) kernel_loop<n, 0, EXACT>(c, col, k0, k1);                 \
    else if (spread == 1) kernel_loop<n, 1, EXACT>(c, col, k0, k1);            \
    else kernel_loop<n, 2, EXACT>(c, col, k0, k1);                             \
    break;
    GPAIR_FWD_CASE(2) GPAIR_FWD_CASE(3) GPAIR_FWD_CASE(4) GPAIR_FWD_CASE(5)
    GPAIR_FWD_CASE(6) GPAIR_FWD_CASE(7) GPAIR_FWD_CASE(8) GPAIR_FWD_CASE(9)
    GPAIR_FWD_CASE(10) GPAIR_FWD_CASE(11) GPAIR_FWD_CASE(12) GPAIR_FWD_CASE(13)
    GPAIR_FWD_CASE(14) GPAIR_FWD_CASE(15) GPAIR_FWD_CASE(16) GPAIR_FWD_CASE(17)
    GPAIR_FWD_CASE(18)
#undef GPAIR_FWD_CASE
    default: kernel_loop_mixed<EXACT>(c, col, k0, k1); break;
  }
}

struct FwdArgs {
  const double4 *sens;
  const TileInfo *tiles;
  const TileInfo *blocks;  // adjoint tiles: the reference blocks
  float *y;
  int64_t nlogical;
  int32_t ntiles, nblocks;
  int32_t Nd, Nt, nsg, L;
  double inv_vdt, t0_over_dt, hmax, vdt;
  double peak;      // bound of |A/(2r) d e^{-d^2/2 sigma^2}| r / |A| over sigma <= sigma_max
  double min_dist;  // lower bound of every kernel-sensor distance (m)
  long long *y64;          // deterministic flush: int64 [Nd][Nt] in units of *det_unit
  const double *det_unit;  // the global unit (device), set before the launch
};

// The record array is a direct kernel argument (const, restrict) so that its
// uniform loads stay scalar loads next to the LDS adds of the tap loop.
// Compiled for 8 waves per SIMD (64 VGPRs, no spills; 75 unconstrained, at
// 6 waves, measured 1.3 % slower at the paper-scale shape).
template <int WAVES, bool DET>
__global__ __launch_bounds__(WAVES * kWave) __attribute__((amdgpu_waves_per_eu(8))) void forward_kernel(
    const KernelRec *__restrict__ krec, FwdArgs a) {
  extern __shared__ int seg[];  // [L][64]: sample-major, one column per sensor
  const int64_t logical = xcd_logical_block(a.nlogical);
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

  // Tap-count range and sum of |A_k| of the tile, read once per wave.  Every
  // wave adds the same values in the same order (the butterfly gives every
  // lane the same sum, as float addition commutes), so all waves of the
  // workgroup derive the same fixed-point unit.
  int nmin = 1 << 30, nmax = 0;
  float asum = 0.0f;
  for (int i = T.start + lane; i < T.start + T.count; i += kWave) {
    const int n = krec[i].ntap;
    nmin = min(nmin, n);
    nmax = max(nmax, n);
    asum += fabsf(krec[i].amp);
  }
  for (int off = 32; off > 0; off >>= 1) {
    nmin = min(nmin, __shfl_xor(nmin, off, kWave));
    nmax = max(nmax, __shfl_xor(nmax, off, kWave));
    asum += __shfl_xor(asum, off, kWave);
  }
  nmin = __builtin_amdgcn_readfirstlane(nmin);
  nmax = __builtin_amdgcn_readfirstlane(nmax);
  // Every member is at distance >= r_low, so every sample's sum over the tile
  // is at most `bound` = 2^30 units: with each tap rounded to half a unit the
  // integer stays below 2^31 for any tile size used here.  A non-finite asum
  // gives unit = inf or NaN and a non-finite output.
  const double r_low = fmax(R - T.rho, a.min_dist);
  const double bound = (double)asum * a.peak / r_low;
  const float unit = (float)(bound * 0x1p-30);
  __syncthreads();  // the segment is zero

  int *const col = seg + lane;
  FwdLoop c;
  c.krec = krec;
  c.s = s;
  c.nb = nb;
  c.inv_vdt = a.inv_vdt;
  c.t0_over_dt = a.t0_over_dt;
  c.inv_vdt_f = (float)a.inv_vdt;
  c.iuw = bound > 0.0 ? (float)(0x1p30 / bound * 0.5 * a.vdt) : 0.0f;
  const int nt_unrolled = (nmin >= nmax - 2 && nmax >= 2 && nmax <= 18) ? nmax : 0;
  const int spread = nmax - nmin;
  const int bend = tile + 1 < a.ntiles ? a.tiles[tile + 1].first_block : a.nblocks;
  for (int b = T.first_block + wave; b < bend; b += WAVES) {
    const TileInfo B = a.blocks[b];
    block_lane(s, B, nb, a.inv_vdt, a.t0_over_dt, c.bl);
    c.kit = B.filter_steps;
    if (c.kit < 0)
      block_loops<true>(c, col, B.start, B.start + B.count, nt_unrolled, spread);
    else
      block_loops<false>(c, col, B.start, B.start + B.count, nt_unrolled, spread);
  }
  __syncthreads();

  // Back to float32 (each lane's own unit; DET: kept as integers), row c
  // stored rotated by c columns so that the flush below reads a row of the
  // transpose without bank conflicts.  Each row is read and rewritten by one
  // wave.
  for (int cr = wave; cr < a.L; cr += WAVES) {
    const int v = col[cr * kWave];
    seg[cr * kWave + ((lane + cr) & (kWave - 1))] = DET ? v : __float_as_int((float)v * unit);
  }
  __syncthreads();

  if (DET) {
    // Deterministic flush: each sample's tile sum (integer, in units of
    // bound 2^-30) goes to the global unit G, rounded to the nearest integer,
    // and is added with a 64-bit integer atomic.  The rounding depends only
    // on the tile's own sum and integer addition is exact and commutative,
    // so y is the same bit for bit whatever the order of the tiles.  G is
    // 2^-62 of a bound on every sample of y, so no sum overflows.
    const double G = *a.det_unit;
    const double fac = bound * 0x1p-30 / G;
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

  // Flush: one sensor row per wave at a time, lanes walk its samples so that
  // consecutive lanes add to consecutive addresses of y (coalesced float
  // atomics; per-lane rows would scatter one atomic per cache line).
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
struct AdjArgs {
  const KernelRec *krec;
  const TileInfo *tiles;
  const int32_t *perm;
  const float *delta;
  float *gA;
  float *gS;   // null: not written
  float *gC;   // [M][3] centre gradient (MODE 2), caller order
  int64_t nlogical;
  int32_t Nd, Nt, L, ntap_max;
  int32_t rank;  // order the tile's kernels by tap count
  double inv_vdt, t0_over_dt, hmax, vdt, nsig;
};

// Sensors from which ranking a tile's kernels by tap count pays (measured:
// +13% adjoint time at 64 sensors, -2% at 1024 with sigma spread by 5%).
constexpr int kAdjRankMinSensors = 256;

// What the adjoint accumulates: MODE 0 the amplitude gradient; 1 also the
// sigma-gradient; 2 also the centre gradient.
constexpr int kAdjA = 0, kAdjSigma = 1, kAdjCentres = 2;
// Tap counts for which the A and sigma modes sum moments about the window's
// middle tap (shorter windows cancel in float32; longer ones keep the direct
// sums for their registers).
constexpr int kAdjMomentTaps[2] = {7, 12};

// Gather the taps of one kernel-sensor pair from a staged residual row (row
// points at the pair's first sample): NT samples, of which the first
// ntap - 1 are in the window and sample ntap - 1 is iff last_ok.  The wave's
// tap counts lie in NT - SPREAD .. NT, so only the last SPREAD + 1 samples
// can be outside (with SPREAD = 0 only the last, by last_ok alone).  All
// reads are issued first.  With t = delta f (f = e/r) and offsets u in
// samples: s1 += t u, and for MODE >= 1 s3 += t u^3, for MODE 2 s0 += t,
// s2 += t u^2.
template <int NT, int SPREAD, int MODE>
__device__ __forceinline__ void gather_taps(const float *row, float f, float q, float d,
                                            float rq, int ntap, bool last_ok, float &s0,
                                            float &s1, float &s2, float &s3) {
  float dl[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) dl[i] = row[i];
  if (SPREAD == 0) {
    if (!last_ok) dl[NT - 1] = 0.0f;
  } else {
#pragma unroll
    for (int i = (NT - 1 - SPREAD > 0 ? NT - 1 - SPREAD : 0); i < NT; ++i) {
      const bool inside = i < ntap - 1 || (i == ntap - 1 && last_ok);
      if (!inside) dl[i] = 0.0f;
    }
  }
  if (MODE != kAdjCentres && NT >= kAdjMomentTaps[0] && NT <= kAdjMomentTaps[1]) {
    // t_i = f_i u_i by the forward's recurrence t_{i+1} = q_i t_i - f_{i+1};
    // with C the middle tap and u_i = uc - (i - C), uc = d - C:
    //   sum w u^2 = uc (uc M0 + M1) + M2,
    // w = delta t, M0 = sum w, M1 = -2 sum w (i - C), M2 = sum w (i - C)^2.
    constexpr int C = (NT - 1) / 2;
    float t = f * d;
    float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const float w = dl[i] * t;
      m0 += w;
      if (MODE >= kAdjSigma && i != C) {
        m1 = fmaf(w, (float)(-2 * (i - C)), m1);
        m2 = fmaf(w, (float)((i - C) * (i - C)), m2);
      }
      if (i + 1 < NT) {
        f *= q;
        t = fmaf(q, t, -f);
        q *= rq;
      }
    }
    s1 += m0;
    if (MODE >= kAdjSigma) {
      const float uc = d - (float)C;
      s3 += fmaf(uc, fmaf(uc, m0, m1), m2);
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    if (MODE == kAdjCentres) {
      const float t = dl[i] * f;
      const float d2 = d * d;
      s0 += t;
      s2 = fmaf(t, d2, s2);
      const float pd = t * d;
      s1 += pd;
      s3 = fmaf(pd, d2, s3);
    } else {
      const float pd = dl[i] * f * d;
      s1 += pd;
      if (MODE >= kAdjSigma) s3 = fmaf(pd, d * d, s3);
    }
    d -= 1.0f;
    f *= q;
    q *= rq;
  }
}

// Per-lane sums of one stage (float32).
struct AdjSums {
  float a;           // sum delta u e/r                          (amplitude)
  float s;           // sum delta u^3 e/r                        (sigma)
  float cx, cy, cz;  // sum over pairs of (c - s)/r G, G = sum delta e/r
                     //   (1 - u^2/sigma_u^2) - (Delta/r) sum delta u e/r   (centres)
};

struct AdjPair {
  const double4 *sens;
  const KernelRec *r;
  const float *stage;
  const int *nbs;
  const float4 *su;  // per staged sensor: -2u (x, y, z), 1/(2R)
  const float4 *sv;  // per staged sensor: R, Xf, Xi (bits), unused
  int L, j0;
  int kit;           // the tile's filter steps, or -1 (every pair in float64)
  double inv_vdt, t0_over_dt;
  float inv_vdt_f;
  float vdt_f;       // Delta (m)
};

// The taps of one stage of sensors for one lane's kernel.  NT > 0: every
// kernel of the wave has NT - SPREAD .. NT taps (fully unrolled); NT = 0: any.
// isg2 = (Delta/sigma_k)^2 (MODE 2).
template <int NT, int SPREAD, int MODE>
__device__ __forceinline__ void adjoint_stage(const AdjPair &c, int nsb, float isg2,
                                              AdjSums &acc) {
  const KernelRec &r = *c.r;
  for (int js = 0; js < nsb; ++js) {
    // One sensor for the whole wave: U, V and the segment base are uniform;
    // the base is read only on the float64 path.
    const float4 U = c.su[js];
    const float4 V = c.sv[js];
    const int kit = c.kit;
    PairW p;
    if (kit >= 0) {
      BlockLane bl;
      bl.m2ux = U.x;
      bl.m2uy = U.y;
      bl.m2uz = U.z;
      bl.inv2R = U.w;
      bl.Rf = V.x;
      bl.Xf = V.y;
      bl.Xi = __float_as_int(V.z);
      if (pair_filter(bl, kit, r.dx, r.dy, r.dz, r.dd, r.hf, r.H, c.inv_vdt_f, p))
        pair_exact<false>(c.sens[c.j0 + js], r.fcx, r.fcy, r.fcz, r.h, r.ntap, c.nbs[js],
                          c.inv_vdt, c.t0_over_dt, p);
    } else {
      pair_exact<true>(c.sens[c.j0 + js], r.fcx, r.fcy, r.fcz, r.h, r.ntap, c.nbs[js], c.inv_vdt,
                       c.t0_over_dt, p);
    }
    const float d0 = p.d0;
    const float f = p.rinv * __builtin_amdgcn_exp2f(r.c * d0 * d0);
    const float q = __builtin_amdgcn_exp2f(fmaf(r.k1, d0, r.c));
    const float *row = c.stage + js * c.L + p.o;
    // MODE 2 needs the pair's own sums; otherwise taps add straight into the
    // stage's sums.
    float t0 = 0.0f, t1 = 0.0f, t2 = 0.0f, t3 = 0.0f;
    float &s1 = MODE == kAdjCentres ? t1 : acc.a;
    float &s3 = MODE == kAdjCentres ? t3 : acc.s;
    if (NT > 0) {
      gather_taps<(NT > 0 ? NT : 1), SPREAD, MODE>(row, f, q, d0, r.rq, r.ntap, p.last_ok, t0, s1,
                                                   t2, s3);
    } else {
      const int nvalid = p.last_ok ? r.ntap : r.ntap - 1;
      // Any tap count: the Gaussian factors are re-evaluated every kTapRun
      // taps, as in the forward.
      for (int i0 = 0; i0 < nvalid; i0 += kTapRun) {
        float d = d0 - (float)i0;
        float ff = p.rinv * __builtin_amdgcn_exp2f(r.c * d * d);
        float qq = __builtin_amdgcn_exp2f(fmaf(r.k1, d, r.c));
        const int iend = min(i0 + kTapRun, nvalid);
        for (int it = i0; it < iend; ++it) {
          const float t = row[it] * ff;
          const float pd = t * d;
          s1 += pd;
          if (MODE >= kAdjSigma) s3 = fmaf(pd, d * d, s3);
          if (MODE == kAdjCentres) {
            t0 += t;
            t2 = fmaf(t, d * d, t2);
          }
          d -= 1.0f;
          ff *= qq;
          qq *= r.rq;
        }
      }
    }
    if (MODE == kAdjCentres) {
      acc.a += t1;
      acc.s += t3;
      // c - s = dk + (-2u)/2; G/r along (c - s)/r.
      const float g = fmaf(-t2, isg2, t0) - (c.vdt_f * p.rinv) * t1;
      const float w = g * p.rinv;
      acc.cx = fmaf(w, fmaf(U.x, 0.5f, r.dx), acc.cx);
      acc.cy = fmaf(w, fmaf(U.y, 0.5f, r.dy), acc.cy);
      acc.cz = fmaf(w, fmaf(U.z, 0.5f, r.dz), acc.cz);
    }
  }
}

template <int BLOCK, int MODE>
__device__ __forceinline__ void adjoint_body(const double4 *__restrict__ sens, const AdjArgs &a) {
  extern __shared__ float stage[];  // [kAdjSensorsPerStage][L]
  __shared__ int nbs[kAdjSensorsPerStage];
  __shared__ float4 su[kAdjSensorsPerStage];
  __shared__ float4 sv[kAdjSensorsPerStage];
  __shared__ int4 tapn[BLOCK / 4];  // tap count of each of the tile's kernels
  __shared__ int order[BLOCK];      // tile kernels by tap count

  const int64_t logical = xcd_logical_block(a.nlogical);
  if (logical >= a.nlogical) return;
  const TileInfo T = a.tiles[logical];
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  const int wave = t >> 6;

  // Each wave runs the largest tap count of its kernels, so the tile's
  // kernels are assigned to threads in order of tap count (ties by index):
  // a wave then mostly holds kernels of one width.  Every kernel is still
  // summed by one thread with the same operations.  Positions past the
  // tile's end sort last, so thread t holds a kernel iff t < count.  The
  // ranking (BLOCK comparisons per thread) pays only when the sensor loop
  // is long (a.rank: N_d >= kAdjRankMinSensors).
  if (!a.rank) {
    order[t] = t;
  } else {
    const int mine = t < T.count ? a.krec[T.start + t].ntap : INT_MAX;
    reinterpret_cast<int *>(tapn)[t] = mine;
    __syncthreads();
    int rank = 0;
    for (int u4 = 0; u4 < BLOCK / 4; ++u4) {
      const int4 k = tapn[u4];
      const int u = 4 * u4;
      rank += (k.x < mine || (k.x == mine && u < t)) + (k.y < mine || (k.y == mine && u + 1 < t)) +
              (k.z < mine || (k.z == mine && u + 2 < t)) + (k.w < mine || (k.w == mine && u + 3 < t));
    }
    order[rank] = t;
  }
  __syncthreads();
  const bool live = t < T.count;
  const int64_t i = T.start + (live ? order[t] : 0);
  const KernelRec r = a.krec[i];

  // Tap-count range of the wave's kernels: selects the unrolled gather.
  const int nmax = __builtin_amdgcn_readfirstlane(wave_max(live ? r.ntap : 0));
  const int nmin = __builtin_amdgcn_readfirstlane(wave_min(live ? r.ntap : 1 << 30));
  const int NT = (nmax >= 2 && nmax <= 18 && nmin >= nmax - 2) ? nmax : 0;
  const int spread = nmax - nmin;

  AdjPair c;
  c.sens = sens;
  c.r = &r;
  c.stage = stage;
  c.nbs = nbs;
  c.su = su;
  c.sv = sv;
  c.L = a.L;
  c.inv_vdt = a.inv_vdt;
  c.t0_over_dt = a.t0_over_dt;
  c.inv_vdt_f = (float)a.inv_vdt;
  c.vdt_f = (float)a.vdt;
  c.kit = T.filter_steps;

  float isg2 = 0.0f;
  if (MODE == kAdjCentres) {
    const double ds = a.nsig / r.h;  // Delta / sigma_k
    isg2 = (float)(ds * ds);
  }
  double accA = 0.0, accS = 0.0, accC[3] = {0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < a.Nd; j0 += kAdjSensorsPerStage) {
    const int nsb = min(kAdjSensorsPerStage, a.Nd - j0);
    __syncthreads();  // the previous stage has been consumed
    if (t < nsb) {
      const double4 s = sens[j0 + t];
      const double dx = s.x - T.cx, dy = s.y - T.cy, dz = s.z - T.cz;
      const double R = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
      const int nb = (int)floor((R - T.rho) * a.inv_vdt - a.t0_over_dt - a.hmax) - 1;
      nbs[t] = nb;
      // The reference point's conversions are redone here every stage rather
      // than held in registers through the pair loops.
      TileInfo Tr = T;
      asm volatile("" : "+s"(Tr.cx), "+s"(Tr.cy), "+s"(Tr.cz));
      BlockLane bl;
      block_lane(s, Tr, nb, a.inv_vdt, a.t0_over_dt, bl);
      su[t] = make_float4(bl.m2ux, bl.m2uy, bl.m2uz, bl.inv2R);
      sv[t] = make_float4(bl.Rf, bl.Xf, __int_as_float(bl.Xi), 0.0f);
    }
    __syncthreads();
    // Stage the residual over the tile's time shell: one wave per row, lanes
    // along the row (coalesced), samples outside the trace read as zero.
    for (int js = wave; js < nsb; js += BLOCK / kWave) {
      const float *drow = a.delta + (int64_t)(j0 + js) * a.Nt;
      const int nb = nbs[js];
      for (int col = lane; col < a.L; col += kWave) {
        const int n = nb + col;
        stage[js * a.L + col] = (n >= 0 && n < a.Nt) ? drow[n] : 0.0f;
      }
    }
    __syncthreads();

    c.j0 = j0;
    AdjSums sums = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    switch (NT) {
#define GPAIR_ADJ_CASE(n)                                                       \
  case n:                                                                       \
    if (spread == 0) adjoint_stage<n, 0, MODE>(c, nsb, isg2, sums);             \
    else if (spread == 1) adjoint_stage<n, 1, MODE>(c, nsb, isg2, sums);        \
    else adjoint_stage<n, 2, MODE>(c, nsb, isg2, sums);                         \
    break;
      GPAIR_ADJ_CASE(2) GPAIR_ADJ_CASE(3) GPAIR_ADJ_CASE(4) GPAIR_ADJ_CASE(5)
      GPAIR_ADJ_CASE(6) GPAIR_ADJ_CASE(7) GPAIR_ADJ_CASE(8) GPAIR_ADJ_CASE(9)
      GPAIR_ADJ_CASE(10) GPAIR_ADJ_CASE(11) GPAIR_ADJ_CASE(12) GPAIR_ADJ_CASE(13)
      GPAIR_ADJ_CASE(14) GPAIR_ADJ_CASE(15) GPAIR_ADJ_CASE(16) GPAIR_ADJ_CASE(17)
      GPAIR_ADJ_CASE(18)
      default: adjoint_stage<0, 2, MODE>(c, nsb, isg2, sums); break;
#undef GPAIR_ADJ_CASE
    }
    accA += (double)sums.a;
    if (MODE >= kAdjSigma) accS += (double)sums.s;
    if (MODE == kAdjCentres) {
      accC[0] += (double)sums.cx;
      accC[1] += (double)sums.cy;
      accC[2] += (double)sums.cz;
    }
  }
  if (live) {
    // The sums ran over e/r with offsets in samples: gA = Delta/2 sum delta u e/r,
    // gsigma = A/2 (Delta/sigma)^3 sum delta u^3 e/r, Delta/sigma = n_sigma/h.
    // gc = A/2 sum over pairs of (c - s)/r G.
    // The kernel's index again from the ranking in LDS (nothing holds it
    // through the stages).
    const int32_t k = a.perm[T.start + order[t]];
    a.gA[k] = (float)(accA * 0.5 * a.vdt);
    if (MODE >= kAdjSigma && a.gS) {
      const double ds = a.nsig / r.h;
      a.gS[k] = (float)(accS * 0.5 * (double)r.amp * ds * ds * ds);
    }
    if (MODE == kAdjCentres) {
      const double h = 0.5 * (double)r.amp;
      a.gC[3 * (int64_t)k] = (float)(accC[0] * h);
      a.gC[3 * (int64_t)k + 1] = (float)(accC[1] * h);
      a.gC[3 * (int64_t)k + 2] = (float)(accC[2] * h);
    }
  }
}

// The amplitude and sigma modes are held to the register budget of 7 waves
// per SIMD (72 VGPRs, where they compile to 65-70); a variant that took 88
// VGPRs ran at 5 waves and 7 % slower.  The centre mode keeps its ~98 VGPRs
// (the cap would spill 19).
template <int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(7))) void adjoint_kernel(
    const double4 *__restrict__ sens, AdjArgs a) {
  adjoint_body<BLOCK, MODE>(sens, a);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void adjoint_centres_kernel(const double4 *__restrict__ sens,
                                                               AdjArgs a) {
  adjoint_body<BLOCK, kAdjCentres>(sens, a);
}

// Deterministic forward: sum of |A_k| in float64 in a fixed order (block
// partial sums, then one thread over the partials), and the global unit
// G = 2^-62 sum |A| peak / min_dist, a bound of every sample of y over 2^62.
__global__ __launch_bounds__(256) void det_abs_partial_kernel(const KernelRec *__restrict__ rec,
                                                             int64_t M, double *partials) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (int64_t)gridDim.x * 256)
    acc += fabs((double)rec[i].amp);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void det_unit_kernel(const double *partials, int nblocks, double scale, double *unit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double sum = 0.0;
  for (int b = 0; b < nblocks; ++b) sum += partials[b];
  *unit = sum * scale;
}

__global__ __launch_bounds__(256) void det_finish_kernel(const long long *__restrict__ y64,
                                                        const double *unit, float *y, int64_t n) {
  const double G = *unit;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    y[i] = (float)((double)y64[i] * G);
}

}  // namespace

hipError_t launch_prep(const gpair_plan_s *p, const float *A, const float *sigma,
                       hipStream_t s) {
  const int64_t M = p->M;
  const unsigned int grid = (unsigned int)((M + 255) / 256);
  prep_kernel<<<grid, 256, 0, s>>>(A, sigma, ws_perm(p), ws_krec(p), M, p->vdt, p->nsig,
                                   p->sigma_max * (1.0 + 1e-6), ws_counters(p));
  return hipGetLastError();
}

hipError_t launch_forward(const gpair_plan_s *p, float *y, hipStream_t s) {
  FwdArgs a;
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
  // max over d of |d| e^{-d^2/(2 sigma^2)} is sigma e^{-1/2}; the record
  // builder clamps sigma to sigma_max (1 + 1e-6), and the last factor covers
  // the float32 rounding of the taps.
  a.peak = 0.5 * p->sigma_max * (1.0 + 1e-6) * 0.60653065971263342 * (1.0 + 1e-5);
  a.min_dist = p->min_dist;
  a.y64 = nullptr;
  a.det_unit = nullptr;
  const int64_t n = (int64_t)p->Nd * p->Nt;
  if (p->deterministic) {
    a.y64 = ws_det(p);
    double *unit = (double *)(a.y64 + n);
    double *partials = ws_partials(p);
    det_abs_partial_kernel<<<kResidualBlocks, 256, 0, s>>>(ws_krec(p), p->M, partials);
    det_unit_kernel<<<1, 64, 0, s>>>(partials, kResidualBlocks, a.peak / a.min_dist * 0x1p-62,
                                     unit);
    a.det_unit = unit;
    hipError_t e = launch_fill((float *)a.y64, 2 * n, 0.0f, s);  // int64 zero = two float zeros
    if (e != hipSuccess) return e;
  }
  const size_t lds = (size_t)p->Lf * kWave * sizeof(int);
  const unsigned int grid = xcd_grid(a.nlogical);
#define GPAIR_FWD_LAUNCH(D)                                                                \
  switch (p->fwd_waves) {                                                                  \
    case 1: forward_kernel<1, D><<<grid, kWave, lds, s>>>(ws_krec(p), a); break;            \
    case 2: forward_kernel<2, D><<<grid, 2 * kWave, lds, s>>>(ws_krec(p), a); break;        \
    case 4: forward_kernel<4, D><<<grid, 4 * kWave, lds, s>>>(ws_krec(p), a); break;        \
    default: forward_kernel<8, D><<<grid, 8 * kWave, lds, s>>>(ws_krec(p), a); break;       \
  }
  if (p->deterministic) {
    GPAIR_FWD_LAUNCH(true)
    det_finish_kernel<<<(unsigned int)std::min<int64_t>((n + 255) / 256, 16384), 256, 0, s>>>(
        a.y64, a.det_unit, y, n);
  } else {
    GPAIR_FWD_LAUNCH(false)
  }
#undef GPAIR_FWD_LAUNCH
  return hipGetLastError();
}

hipError_t launch_adjoint(const gpair_plan_s *p, const float *delta, float *gA,
                          float *gsigma, float *gcentres, hipStream_t s) {
  AdjArgs a;
  a.krec = ws_krec(p);
  a.tiles = ws_atiles(p);
  a.perm = ws_perm(p);
  a.delta = delta;
  a.gA = gA;
  a.gS = gsigma;
  a.gC = gcentres;
  a.nlogical = (int64_t)p->host.atiles.size();
  a.Nd = p->Nd;
  a.Nt = p->Nt;
  a.L = p->La;
  a.ntap_max = p->ntap_max;
  a.inv_vdt = p->inv_vdt;
  a.t0_over_dt = p->t0_over_dt;
  a.hmax = p->hmax;
  a.vdt = p->vdt;
  a.nsig = p->nsig;
  a.rank = p->Nd >= kAdjRankMinSensors ? 1 : 0;
  const size_t lds = (size_t)p->La * kAdjSensorsPerStage * sizeof(float);
  const unsigned int grid = xcd_grid(a.nlogical);
  const double4 *sens = (const double4 *)ws_sens(p);
  const int mode = gcentres ? kAdjCentres : (gsigma ? kAdjSigma : kAdjA);
#define GPAIR_ADJ_LAUNCH(B)                                                          \
  switch (mode) {                                                                    \
    case kAdjA: adjoint_kernel<B, kAdjA><<<grid, B, lds, s>>>(sens, a); break;        \
    case kAdjSigma: adjoint_kernel<B, kAdjSigma><<<grid, B, lds, s>>>(sens, a); break; \
    default: adjoint_centres_kernel<B><<<grid, B, lds, s>>>(sens, a); break;          \
  }
  switch (p->adj_tile) {
    case 64: GPAIR_ADJ_LAUNCH(64) break;
    case 128: GPAIR_ADJ_LAUNCH(128) break;
    default: GPAIR_ADJ_LAUNCH(256) break;
  }
#undef GPAIR_ADJ_LAUNCH
  return hipGetLastError();
}

}  // namespace gpair
