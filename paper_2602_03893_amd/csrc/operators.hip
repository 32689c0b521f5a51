// operators.hip -- gfx950 kernels of the direct GPAIR operators.
//
// Forward (arXiv 2602.03893, Eq. (single_forward) summed over kernels, inside
// the n_sigma window that follows it):
//   y_j[n] = sum_k [|d| <= n_sigma sigma_k] A_k/(2 r_jk) d exp(-d^2/(2 sigma_k^2)),
//   d = r_jk - v (t0 + n dt).
// Adjoint: its transpose, plus the sigma-derivative of Eq. (single_forward).
//
// Work decomposition (VALU-bound; no MFMA: nothing here is a contraction).
//  * Pair stage, float64: r = |s - c| (float64 difference of float32
//    coordinates, float32 rsq seed + one float64 Newton step), pulse centre
//    in samples nc = (r - v t0)/(v dt), first in-window sample lo =
//    ceil(nc - h) with h = n_sigma sigma / (v dt).  Window membership is
//    therefore decided in float64, as in the float64 reference.
//  * Tap stage, float32: d_i = d_0 - i Delta, and the Gaussian factor by the
//    exact recurrence e_{i+1} = e_i q_i, q_{i+1} = q_i rq (two exp2 per pair
//    instead of one per tap; windows longer than 18 taps re-evaluate e and q
//    every 16 taps, since the rounding of tap i grows like i^2).
//  * Forward: one workgroup = one tile of kernels x 64 sensors; lane = sensor,
//    the kernel loop is wave-uniform (kernel data in scalar registers) and the
//    workgroup's waves split the tile's kernels.  The waves share one LDS
//    trace segment per sensor over the tile's time shell, into which taps go
//    as 32-bit fixed-point integer adds (ds_add_u32 issues without waiting,
//    where a float add or a read-modify-write waits for LDS every tap).  The
//    fixed-point unit is per sensor: 2^-30 of a bound on any sum the tile can
//    put into one sample (sum_k |A_k| * sigma_max e^{-1/2} / (2 r_low)), so no
//    sum can overflow and each tap is rounded to 2^-31 of that bound.  At the
//    end the segment goes back to float32 and is added to y with one
//    coalesced float atomic per sample (tile-sensor partial sums).
//  * Adjoint: one workgroup = one tile of kernels; lane = kernel, the sensor
//    loop is uniform.  For each stage of 64 sensors the residual over the
//    tile's time shell is staged in LDS; every lane gathers its taps from it.
//    Per-lane sums go from float32 (within a stage) to float64 (across
//    stages); no atomics.
//  * Blocks are remapped so that each of the 8 XCDs works on a contiguous
//    range of tiles (its L2 then holds that region's kernel records and the
//    matching residual rows).
#include <climits>

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
  const double c = -kLog2e / (2.0 * s * s);
  const double h = nsig * s / vdt;
  KernelRec &r = rec[i];  // the centre fields were written at plan binding
  r.h = h;
  r.amp = a;
  r.c = (float)c;
  r.k1 = (float)(-2.0 * c * vdt);
  r.k2 = (float)(c * vdt * vdt);
  r.rq = (float)exp2(2.0 * c * vdt * vdt);
  r.ntap = (int32_t)floor(2.0 * h) + 1;
  r.hlast = (double)(r.ntap - 1) - h;
}

// ---------------------------------------------------------------------------
// Pair stage shared by both operators (float64 distance and window).
// ---------------------------------------------------------------------------
struct PairTerms {
  double fr;    // nc - lo in (h - 1, h]: offset of the first tap, in samples
  int lo;       // first in-window sample index
  float rinv;   // 1/r (float32 rsq seed)
};

__device__ __forceinline__ PairTerms pair_terms(double sx, double sy, double sz,
                                                double cx, double cy, double cz,
                                                double h, double inv_vdt,
                                                double t0_over_dt) {
  const double ex = sx - cx, ey = sy - cy, ez = sz - cz;
  const double r2 = fma(ez, ez, fma(ey, ey, ex * ex));
  const float y0 = __builtin_amdgcn_rsqf((float)r2);
  const double y0d = (double)y0;
  const double r0 = r2 * y0d;                  // ~r to float32 accuracy
  const double res = fma(-r0, r0, r2);         // r2 - r0^2
  const double r = fma(res, 0.5 * y0d, r0);    // one Newton step: ~1e-15 rel
  const double nc = fma(r, inv_vdt, -t0_over_dt);
  const double lo = ceil(nc - h);
  PairTerms t;
  t.fr = nc - lo;
  t.lo = (int)lo;
  t.rinv = y0;
  return t;
}

// ---------------------------------------------------------------------------
// Forward.
// ---------------------------------------------------------------------------
// Everything the tap loop of one kernel-sensor pair needs.
struct Taps {
  float w;       // A / (2 r)
  float f;       // w * exp(-d0^2 / (2 sigma^2))
  float q;       // ratio of the second tap's Gaussian factor to the first's
  float d;       // d0 = r - v t of the first tap (m)
  int o;         // first tap's slot in the lane's segment
  bool last_ok;  // tap ntap-1 is inside the window
};

__device__ __forceinline__ Taps pair_taps(const double4 &s, const KernelRec &r, int nb, int omax,
                                          double inv_vdt, double t0_over_dt, double vdt) {
  const PairTerms pt = pair_terms(s.x, s.y, s.z, r.cx, r.cy, r.cz, r.h, inv_vdt, t0_over_dt);
  Taps t;
  t.d = (float)(pt.fr * vdt);
  t.last_ok = pt.fr >= r.hlast;
  // By construction of nb and L every tap slot o + i (i < ntap) is at most
  // L - 4; the clamp (omax = L - 1 - the samples the caller writes) only keeps
  // LDS accesses in range if that were ever violated.
  t.o = min(max(pt.lo - nb, 0), omax);
  t.w = (0.5f * r.amp) * pt.rinv;
  t.f = t.w * __builtin_amdgcn_exp2f(r.c * t.d * t.d);
  t.q = __builtin_amdgcn_exp2f(fmaf(r.k1, t.d, r.k2));
  return t;
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
// first nvalid are inside the window (nvalid = ntap - 1 or ntap, and ntap >=
// NT - 2, so only the last three can be outside).
template <int NT>
__device__ __forceinline__ void taps_add(int *p, float f, float q, float d, float rq,
                                         float vdt, int nvalid) {
  float t[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    t[i] = f * d;
    d -= vdt;
    f *= q;
    q *= rq;
  }
#pragma unroll
  for (int i = (NT - 3 > 0 ? NT - 3 : 0); i < NT; ++i)
    if (i >= nvalid) t[i] = 0.0f;
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
__device__ __forceinline__ void taps_add_n(int n, int *p, const Taps &t, float rq, float vdt,
                                           float iu, const KernelRec *rec) {
  const int nvalid = n - (t.last_ok ? 0 : 1);
  switch (n) {
#define GPAIR_TAPS_CASE(k) \
  case k: taps_add<k>(p, t.f * iu, t.q, t.d, rq, vdt, nvalid); return;
    GPAIR_TAPS_CASE(1) GPAIR_TAPS_CASE(2) GPAIR_TAPS_CASE(3) GPAIR_TAPS_CASE(4)
    GPAIR_TAPS_CASE(5) GPAIR_TAPS_CASE(6) GPAIR_TAPS_CASE(7) GPAIR_TAPS_CASE(8)
    GPAIR_TAPS_CASE(9) GPAIR_TAPS_CASE(10) GPAIR_TAPS_CASE(11) GPAIR_TAPS_CASE(12)
    GPAIR_TAPS_CASE(13) GPAIR_TAPS_CASE(14) GPAIR_TAPS_CASE(15) GPAIR_TAPS_CASE(16)
    GPAIR_TAPS_CASE(17) GPAIR_TAPS_CASE(18)
#undef GPAIR_TAPS_CASE
    default: break;
  }
  const float c = rec->c, k1 = rec->k1, k2 = rec->k2, w = t.w * iu;
  for (int i0 = 0; i0 < n; i0 += kTapRun) {
    float d = fmaf(-(float)i0, vdt, t.d);
    float f = w * __builtin_amdgcn_exp2f(c * d * d);
    float q = __builtin_amdgcn_exp2f(fmaf(k1, d, k2));
    const int iend = min(i0 + kTapRun, n);
    for (int i = i0; i < iend; ++i) {
      lds_add(p + i * kWave, i < nvalid ? f * d : 0.0f);
      d -= vdt;
      f *= q;
      q *= rq;
    }
  }
}

struct FwdLoop {
  const KernelRec *krec;
  double4 s;
  int nb, L, omax;
  double inv_vdt, t0_over_dt, vdt;
  float vdt_f, iu;
};

// The kernel loop of one wave over records [k0, kend) of its tile when every
// kernel of the tile has NT - 2 .. NT taps.  Kernels go in pairs: both pair
// stages sit in one straight-line block, so their float64 chains interleave,
// and the records of the next pair are fetched meanwhile (clamped to the last
// record).  (Four per iteration need 130 VGPRs and run slower.)
template <int NT>
__device__ __forceinline__ void kernel_loop(const FwdLoop &c, int *col, int k0, int kend) {
  if (k0 >= kend) return;
  const int last = kend - 1;
  const int pend = k0 + ((kend - k0) & ~1);
  KernelRec ra = c.krec[k0], rb = c.krec[min(k0 + 1, last)];
  for (int k = k0; k < pend; k += 2) {
    const Taps ta = pair_taps(c.s, ra, c.nb, c.omax, c.inv_vdt, c.t0_over_dt, c.vdt);
    const Taps tb = pair_taps(c.s, rb, c.nb, c.omax, c.inv_vdt, c.t0_over_dt, c.vdt);
    const float rqa = ra.rq, rqb = rb.rq;
    const int nva = ra.ntap - (ta.last_ok ? 0 : 1), nvb = rb.ntap - (tb.last_ok ? 0 : 1);
    ra = c.krec[min(k + 2, last)];
    rb = c.krec[min(k + 3, last)];
    taps_add<NT>(col + ta.o * kWave, ta.f * c.iu, ta.q, ta.d, rqa, c.vdt_f, nva);
    taps_add<NT>(col + tb.o * kWave, tb.f * c.iu, tb.q, tb.d, rqb, c.vdt_f, nvb);
  }
  if (pend < kend) {
    const Taps t = pair_taps(c.s, ra, c.nb, c.omax, c.inv_vdt, c.t0_over_dt, c.vdt);
    taps_add<NT>(col + t.o * kWave, t.f * c.iu, t.q, t.d, ra.rq, c.vdt_f,
                 ra.ntap - (t.last_ok ? 0 : 1));
  }
}

// The same loop for a tile whose kernels differ in width by more than two
// taps: each pair branches on its own tap count.
__device__ __forceinline__ void kernel_loop_mixed(const FwdLoop &c, int *col, int k0, int kend) {
  if (k0 >= kend) return;
  const int last = kend - 1;
  const int pend = k0 + ((kend - k0) & ~1);
  KernelRec ra = c.krec[k0], rb = c.krec[min(k0 + 1, last)];
  for (int k = k0; k < pend; k += 2) {
    const Taps ta = pair_taps(c.s, ra, c.nb, c.L - 1 - ra.ntap, c.inv_vdt, c.t0_over_dt, c.vdt);
    const Taps tb = pair_taps(c.s, rb, c.nb, c.L - 1 - rb.ntap, c.inv_vdt, c.t0_over_dt, c.vdt);
    const float rqa = ra.rq, rqb = rb.rq;
    const int na = ra.ntap, nb = rb.ntap;
    ra = c.krec[min(k + 2, last)];
    rb = c.krec[min(k + 3, last)];
    taps_add_n(na, col + ta.o * kWave, ta, rqa, c.vdt_f, c.iu, c.krec + k);
    taps_add_n(nb, col + tb.o * kWave, tb, rqb, c.vdt_f, c.iu, c.krec + min(k + 1, last));
  }
  if (pend < kend) {
    const Taps t = pair_taps(c.s, ra, c.nb, c.L - 1 - ra.ntap, c.inv_vdt, c.t0_over_dt, c.vdt);
    taps_add_n(ra.ntap, col + t.o * kWave, t, ra.rq, c.vdt_f, c.iu, c.krec + pend);
  }
}

struct FwdArgs {
  const double4 *sens;
  const TileInfo *tiles;
  float *y;
  int64_t nlogical;
  int32_t Nd, Nt, nsg, L;
  double inv_vdt, t0_over_dt, hmax, vdt;
  double peak;      // bound of |A/(2r) d e^{-d^2/2 sigma^2}| r / |A| over sigma <= sigma_max
  double min_dist;  // lower bound of every kernel-sensor distance (m)
};

// The record array is a direct kernel argument (const, restrict) so that its
// uniform loads stay scalar loads next to the LDS adds of the tap loop.
template <int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void forward_kernel(
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
  const float iu = bound > 0.0 ? (float)(0x1p30 / bound) : 0.0f;
  __syncthreads();  // the segment is zero

  int *const col = seg + lane;
  FwdLoop c;
  c.krec = krec;
  c.s = s;
  c.nb = nb;
  c.L = a.L;
  c.inv_vdt = a.inv_vdt;
  c.t0_over_dt = a.t0_over_dt;
  c.vdt = a.vdt;
  c.vdt_f = (float)a.vdt;
  c.iu = iu;
  const int per = (T.count + WAVES - 1) / WAVES;
  const int k0 = T.start + wave * per;
  const int k1 = min(T.start + T.count, k0 + per);
  if (nmin >= nmax - 2 && nmax >= 2 && nmax <= 18) {
    c.omax = a.L - 1 - nmax;
    switch (nmax) {
#define GPAIR_FWD_CASE(n) \
  case n: kernel_loop<n>(c, col, k0, k1); break;
      GPAIR_FWD_CASE(2) GPAIR_FWD_CASE(3) GPAIR_FWD_CASE(4) GPAIR_FWD_CASE(5)
      GPAIR_FWD_CASE(6) GPAIR_FWD_CASE(7) GPAIR_FWD_CASE(8) GPAIR_FWD_CASE(9)
      GPAIR_FWD_CASE(10) GPAIR_FWD_CASE(11) GPAIR_FWD_CASE(12) GPAIR_FWD_CASE(13)
      GPAIR_FWD_CASE(14) GPAIR_FWD_CASE(15) GPAIR_FWD_CASE(16) GPAIR_FWD_CASE(17)
      default: kernel_loop<18>(c, col, k0, k1); break;
#undef GPAIR_FWD_CASE
    }
  } else {
    kernel_loop_mixed(c, col, k0, k1);
  }
  __syncthreads();

  // Back to float32 (each lane's own unit), row c stored rotated by c columns
  // so that the flush below reads a row of the transpose without bank
  // conflicts.  Each row is read and rewritten by one wave.
  for (int cr = wave; cr < a.L; cr += WAVES) {
    const int v = col[cr * kWave];
    seg[cr * kWave + ((lane + cr) & (kWave - 1))] = __float_as_int((float)v * unit);
  }
  __syncthreads();

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
  float *gS;
  int64_t nlogical;
  int32_t Nd, Nt, L, ntap_max;
  int32_t rank;  // order the tile's kernels by tap count
  double inv_vdt, t0_over_dt, hmax, vdt, nsig;
};

// Sensors from which ranking a tile's kernels by tap count pays (measured:
// +13% adjoint time at 64 sensors, -2% at 1024 with sigma spread by 5%).
constexpr int kAdjRankMinSensors = 256;

__device__ __forceinline__ int wave_min(int x) {
  for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off, kWave));
  return x;
}
__device__ __forceinline__ int wave_max(int x) {
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, kWave));
  return x;
}

// Gather the taps of one kernel-sensor pair from a staged residual row (row
// points at the pair's first sample): NT samples of which the first nvalid
// are in the window (only the last three can be outside).  All reads are
// issued first.
template <int NT, bool SIG>
__device__ __forceinline__ void gather_taps(const float *row, float f, float q, float d,
                                            float rq, float vdt, int nvalid, float &pA,
                                            float &pS) {
  float dl[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) dl[i] = row[i];
#pragma unroll
  for (int i = (NT - 3 > 0 ? NT - 3 : 0); i < NT; ++i)
    if (i >= nvalid) dl[i] = 0.0f;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const float pd = dl[i] * f * d;
    pA += pd;
    if (SIG) pS = fmaf(pd, d * d, pS);
    d -= vdt;
    f *= q;
    q *= rq;
  }
}

struct AdjPair {
  const double4 *sens;
  const KernelRec *r;
  const float *stage;
  const int *nbs;
  int L, omax, j0;
  double inv_vdt, t0_over_dt, vdt;
  float vdt_f;
};

// The taps of one stage of sensors for one lane's kernel.  NT > 0: every
// kernel of the wave has NT - 2 .. NT taps (fully unrolled); NT = 0: any.
template <int NT, bool SIG>
__device__ __forceinline__ void adjoint_stage(const AdjPair &c, int nsb, float &pA, float &pS) {
  const KernelRec &r = *c.r;
  for (int js = 0; js < nsb; ++js) {
    const double4 s = c.sens[c.j0 + js];
    const int nb = c.nbs[js];
    const PairTerms pt = pair_terms(s.x, s.y, s.z, r.cx, r.cy, r.cz, r.h, c.inv_vdt,
                                    c.t0_over_dt);
    const float d0 = (float)(pt.fr * c.vdt);
    const int nvalid = (pt.fr >= r.hlast) ? r.ntap : r.ntap - 1;
    const int o = min(max(pt.lo - nb, 0), c.omax);
    const float f = 0.5f * pt.rinv * __builtin_amdgcn_exp2f(r.c * d0 * d0);
    const float q = __builtin_amdgcn_exp2f(fmaf(r.k1, d0, r.k2));
    const float *row = c.stage + js * c.L + o;
    if (NT > 0) {
      gather_taps<(NT > 0 ? NT : 1), SIG>(row, f, q, d0, r.rq, c.vdt_f, nvalid, pA, pS);
    } else {
      // Any tap count: the Gaussian factors are re-evaluated every kTapRun
      // taps, as in the forward.
      const float w = 0.5f * pt.rinv;
      for (int i0 = 0; i0 < nvalid; i0 += kTapRun) {
        float d = fmaf(-(float)i0, c.vdt_f, d0);
        float ff = w * __builtin_amdgcn_exp2f(r.c * d * d);
        float qq = __builtin_amdgcn_exp2f(fmaf(r.k1, d, r.k2));
        const int iend = min(i0 + kTapRun, nvalid);
        for (int it = i0; it < iend; ++it) {
          const float pd = row[it] * ff * d;
          pA += pd;
          if (SIG) pS = fmaf(pd, d * d, pS);
          d -= c.vdt_f;
          ff *= qq;
          qq *= r.rq;
        }
      }
    }
  }
}

template <int BLOCK, bool SIG>
__global__ __launch_bounds__(BLOCK) void adjoint_kernel(const double4 *__restrict__ sens,
                                                       AdjArgs a) {
  extern __shared__ float stage[];  // [kAdjSensorsPerStage][L]
  __shared__ int nbs[kAdjSensorsPerStage];
  __shared__ int4 tapn[BLOCK / 4];   // tap count of each of the tile's kernels
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

  AdjPair c;
  c.sens = sens;
  c.r = &r;
  c.stage = stage;
  c.nbs = nbs;
  c.L = a.L;
  // By construction every slot a lane reads (its window, plus up to three
  // padding samples in the unrolled gather) is at most L - 1.
  c.omax = a.L - (NT > 0 ? NT : r.ntap);
  c.inv_vdt = a.inv_vdt;
  c.t0_over_dt = a.t0_over_dt;
  c.vdt = a.vdt;
  c.vdt_f = (float)a.vdt;

  double accA = 0.0, accS = 0.0;
  for (int j0 = 0; j0 < a.Nd; j0 += kAdjSensorsPerStage) {
    const int nsb = min(kAdjSensorsPerStage, a.Nd - j0);
    __syncthreads();  // the previous stage has been consumed
    if (t < nsb) {
      const double4 s = sens[j0 + t];
      const double dx = s.x - T.cx, dy = s.y - T.cy, dz = s.z - T.cz;
      const double R = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
      nbs[t] = (int)floor((R - T.rho) * a.inv_vdt - a.t0_over_dt - a.hmax) - 1;
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
    float pA = 0.0f, pS = 0.0f;
    switch (NT) {
#define GPAIR_ADJ_CASE(n) \
  case n: adjoint_stage<n, SIG>(c, nsb, pA, pS); break;
      GPAIR_ADJ_CASE(2) GPAIR_ADJ_CASE(3) GPAIR_ADJ_CASE(4) GPAIR_ADJ_CASE(5)
      GPAIR_ADJ_CASE(6) GPAIR_ADJ_CASE(7) GPAIR_ADJ_CASE(8) GPAIR_ADJ_CASE(9)
      GPAIR_ADJ_CASE(10) GPAIR_ADJ_CASE(11) GPAIR_ADJ_CASE(12) GPAIR_ADJ_CASE(13)
      GPAIR_ADJ_CASE(14) GPAIR_ADJ_CASE(15) GPAIR_ADJ_CASE(16) GPAIR_ADJ_CASE(17)
      GPAIR_ADJ_CASE(18)
      default: adjoint_stage<0, SIG>(c, nsb, pA, pS); break;
#undef GPAIR_ADJ_CASE
    }
    accA += (double)pA;
    if (SIG) accS += (double)pS;
  }
  if (live) {
    const int32_t k = a.perm[i];
    a.gA[k] = (float)accA;
    if (SIG) {
      // sigma_k (as clamped by the record builder) from h = n_sigma sigma / Delta.
      const double sg = r.h * a.vdt / a.nsig;
      a.gS[k] = (float)(accS * (double)r.amp / (sg * sg * sg));
    }
  }
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
  a.y = y;
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
  const size_t lds = (size_t)p->Lf * kWave * sizeof(int);
  const unsigned int grid = xcd_grid(a.nlogical);
  switch (p->fwd_waves) {
    case 1: forward_kernel<1><<<grid, kWave, lds, s>>>(ws_krec(p), a); break;
    case 2: forward_kernel<2><<<grid, 2 * kWave, lds, s>>>(ws_krec(p), a); break;
    case 4: forward_kernel<4><<<grid, 4 * kWave, lds, s>>>(ws_krec(p), a); break;
    default: forward_kernel<8><<<grid, 8 * kWave, lds, s>>>(ws_krec(p), a); break;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(const gpair_plan_s *p, const float *delta, float *gA,
                          float *gsigma, hipStream_t s) {
  AdjArgs a;
  a.krec = ws_krec(p);
  a.tiles = ws_atiles(p);
  a.perm = ws_perm(p);
  a.delta = delta;
  a.gA = gA;
  a.gS = gsigma;
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
  const bool sig = gsigma != nullptr;
  switch (p->adj_tile) {
    case 64:
      if (sig) adjoint_kernel<64, true><<<grid, 64, lds, s>>>((const double4 *)ws_sens(p), a);
      else adjoint_kernel<64, false><<<grid, 64, lds, s>>>((const double4 *)ws_sens(p), a);
      break;
    case 128:
      if (sig) adjoint_kernel<128, true><<<grid, 128, lds, s>>>((const double4 *)ws_sens(p), a);
      else adjoint_kernel<128, false><<<grid, 128, lds, s>>>((const double4 *)ws_sens(p), a);
      break;
    default:
      if (sig) adjoint_kernel<256, true><<<grid, 256, lds, s>>>((const double4 *)ws_sens(p), a);
      else adjoint_kernel<256, false><<<grid, 256, lds, s>>>((const double4 *)ws_sens(p), a);
      break;
  }
  return hipGetLastError();
}

}  // namespace gpair
