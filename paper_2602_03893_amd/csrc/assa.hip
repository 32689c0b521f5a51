// assa.hip -- gfx950 kernels of the ASSA operators (adaptive supersampling
// alignment; arXiv 2602.03893, Methods, "Adaptive supersampling alignment for
// the differentiable model operator", and its Algorithm for the forward and
// adjoint operators with ASSA).
//
// One kernel width sigma shared by all kernels.  The fine-grid index of a
// kernel-sensor pair is k = floor(r ku + ku0), ku = alpha / (v dt),
// ku0 = 1/2 - alpha t0 / dt, evaluated in float64: r^2 = |s|^2 + |c|^2 - 2 s.c
// from the float64 copies of the float32 coordinates (|s|^2 and |c|^2 are
// precomputed, so a pair costs one add and three fused multiply-adds; the
// terms are at most a few times r^2, so the relative error stays ~1e-15),
// then r from a float32 rsq seed and one float64 Newton step.  The offset of
// the LDS segment is folded into the constant of the snap, so that one
// truncating conversion yields the row (the folded value is >= 0 wherever the
// row is used, where truncation and floor agree).
//
// Forward, fused per (tile, 64 sensors) in one workgroup of eight waves:
//  1. projection P_up: lane = sensor; the waves split the tile's kernels and
//     add x_i / r_ij into one fine-grid LDS segment per sensor.  The
//     waves share the segment, so the adds are LDS atomics; they are integer
//     adds of a fixed-point value (LDS float atomics measured about three times
//     slower).  The unit of a column is S / 2^30 with S = sum_tile |x| /
//     r_low, r_low a lower bound of the tile's distances to that sensor: no
//     partial sum can overflow, and every impulse is resolved to
//     2^-31 S (about 5e-7 of an impulse for a uniform tile of 1024 kernels).
//     Within a wave each lane owns its column, so the adds are free of bank
//     conflicts.  The sums are exact and independent of the order of the adds;
//     after the projection each column is converted to float in place;
//  2. transposed convolution with h and decimation, in LDS: coarse sample c
//     of a column is sum_{q<K} hq[q] (z[alpha c + q] - z[alpha c + 2K - q])
//     (h is odd and h[0] = 0), written back over the column's first rows;
//  3. flush: one coalesced float atomic per coarse sample into y, as in the
//     direct forward.  The write-back rotates row c by c columns so that both
//     the write-back (lanes along sensors) and the flush reads (lanes along
//     time) are free of bank conflicts.
// Adjoint:
//  1. delta_conv = correlation of the zero-filled residual with h, one
//     thread per (sensor, sample m) producing the fine samples alpha m + phi;
//  2. back-projection: one workgroup per tile, lane = kernel.  For each stage
//     of 64 sensors the tile's shell of delta_conv is staged in LDS; each lane
//     gathers one value per pair.  float32 within a stage, float64 across
//     stages, no atomics.
#include <algorithm>
#include <cmath>

#include "gpair_internal.h"

namespace gpair {
namespace {

// Waves per forward workgroup (one sensor group).  The projection is latency
// bound and the segment caps the workgroups per CU, so more waves per segment
// pay: 8 waves (83 VGPRs, 6 waves per SIMD) ran 12% faster than 4 at the
// paper shape.
constexpr int kAssaWaves = 8;
constexpr int kAssaOut = kWave / kAssaWaves;  // coarse samples per wave per convolution pass
constexpr int kAssaPass = kAssaWaves * kAssaOut;
constexpr int kAssaStageRegs = 16;    // floats per thread of an adjoint stage in flight
constexpr int kPairs = 4;             // kernel-sensor pairs per projection iteration
static_assert(kAssaPass == kWave, "one convolution pass covers 64 coarse samples");

__device__ __forceinline__ int64_t xcd_logical(int64_t nlogical) {
  const int64_t per = (nlogical + kXcds - 1) / kXcds;
  const int64_t b = blockIdx.x;
  return (b % kXcds) * per + b / kXcds;
}

inline unsigned int xcd_blocks(int64_t nlogical) {
  const int64_t per = (nlogical + kXcds - 1) / kXcds;
  return (unsigned int)(per * kXcds);
}

// floor(a / b) for b > 0.
__device__ __forceinline__ int floor_div(int a, int b) {
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

// Distance r (float64) and the float32 rsq seed 1/r of one pair.
struct Dist {
  double r;
  float rinv;
};

// r^2 = (|s|^2 + |c|^2) - 2 s.c with m2x = -2 s_x (or -2 c_x), ...
__device__ __forceinline__ Dist pair_dist(double m2x, double m2y, double m2z, double cx,
                                          double cy, double cz, double s2c2) {
  const double r2 = fma(m2x, cx, fma(m2y, cy, fma(m2z, cz, s2c2)));
  const float y0 = __builtin_amdgcn_rsqf((float)r2);
  const double y0d = (double)y0;
  const double r0 = r2 * y0d;
  const double res = fma(-r0, r0, r2);
  Dist d;
  d.r = fma(res, 0.5 * y0d, r0);
  d.rinv = y0;
  return d;
}

// Lower bound (minus one) of the fine index of any pair of a tile whose
// members lie within rho of the tile centre at distance R from the sensor.
__device__ __forceinline__ int shell_low(double R, double rho, double ku, double ku0) {
  return (int)floor(fma(R - rho, ku, ku0)) - 1;
}

// Bounding sphere of two consecutive tiles (their kernel ranges are adjacent
// in the permuted order): the smallest sphere enclosing both spheres, with
// the same relative margin as the planner's.  Used on the host and on the
// device, so that the host's segment bound holds for the device's sphere.
__host__ __device__ inline TileInfo merge_tiles(const TileInfo &a, const TileInfo &b) {
  TileInfo m = a;
  m.count = a.count + b.count;
  const double ex = b.cx - a.cx, ey = b.cy - a.cy, ez = b.cz - a.cz;
  const double d = sqrt(ex * ex + ey * ey + ez * ez);
  if (d + b.rho <= a.rho) return m;
  if (d + a.rho <= b.rho) {
    m.cx = b.cx;
    m.cy = b.cy;
    m.cz = b.cz;
    m.rho = b.rho;
    return m;
  }
  const double R = 0.5 * (d + a.rho + b.rho);
  const double f = (R - a.rho) / d;
  m.cx = a.cx + f * ex;
  m.cy = a.cy + f * ey;
  m.cz = a.cz + f * ez;
  m.rho = R * (1.0 + 1e-12) + 1e-15;
  return m;
}

// ---------------------------------------------------------------------------
// Amplitudes into the kernel records (permuted order).
// ---------------------------------------------------------------------------
// One workgroup per forward tile: the members' amplitudes into their records
// and the tile's sum of |x| into its TileInfo (the fixed-point scale).
__global__ __launch_bounds__(256) void assa_prep_kernel(const float *__restrict__ x,
                                                        const int32_t *__restrict__ perm,
                                                        AssaRec *__restrict__ rec,
                                                        TileInfo *__restrict__ tiles) {
  __shared__ float part[256 / kWave];
  TileInfo &T = tiles[blockIdx.x];
  const int start = T.start, count = T.count;
  float acc = 0.0f;
  for (int i = threadIdx.x; i < count; i += 256) {
    AssaRec &r = rec[start + i];
    const float v = x[perm[start + i]];
    const double cx = (double)r.fcx, cy = (double)r.fcy, cz = (double)r.fcz;
    r.cx = cx;
    r.cy = cy;
    r.cz = cz;
    r.amp = v;
    r.cc = fma(cz, cz, fma(cy, cy, cx * cx));  // |c|^2
    acc += fabsf(v);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) T.asum = (part[0] + part[1]) + (part[2] + part[3]);
}

// ---------------------------------------------------------------------------
// Forward.
// ---------------------------------------------------------------------------
struct AssaFwdArgs {
  const double4 *sens;
  const TileInfo *tiles;
  float *y;
  int64_t nlogical;
  int32_t Nd, Nt, nsg, nfine, alpha, K;
  int32_t Lc;   // coarse samples of a (tile, sensor) shell
  int32_t Lch;  // coarse samples per pass (Lc when the whole shell fits in LDS)
  int32_t F;    // fine rows of the LDS segment: alpha (Lch - 1) + 2K + 1
  double ku, ku0;
  double min_dist;      // lower bound of every kernel-sensor distance (m)
  float hq[kAssaMaxK];  // hq[q] = h(K - q), q = 0 .. K-1
};

// Per-lane constants of the projection in one pass.
struct Lane {
  double m2x, m2y, m2z;  // -2 s
  double s2;             // |s|^2
  double cst;            // ku0 - fbc + 1: u1 = r ku + cst = (fine index - fbc) + 1
  int plo, pspan;        // u1 truncates into [plo, plo + pspan) iff the fine point is in
                         // [0, nfine) and in the pass's rows [0, F)
  float inv_unit;        // fixed-point scale of the column
};

// The impulse of one pair: its row (clamped into [0, F)) and fixed-point
// value x / r * inv_unit (zero when outside the grid or the pass, so that the
// add is harmless).  u1 >= 1 wherever the row is used, so truncation = floor.
struct Impulse {
  int row;
  int val;
};

// floor(v + 1/2) as an integer in one instruction (the compiler emits three
// for the same expression).
__device__ __forceinline__ int round_half_up(float v) {
  int n;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(n) : "v"(v));
  return n;
}

__device__ __forceinline__ Impulse impulse(const Lane &l, const AssaRec &r, int F,
                                           double ku) {
  const Dist d = pair_dist(l.m2x, l.m2y, l.m2z, r.cx, r.cy, r.cz, l.s2 + r.cc);
  const int p1 = (int)fma(d.r, ku, l.cst);  // |value| < 1e9 (checked on the host)
  const bool in = (unsigned)(p1 - l.plo) < (unsigned)l.pspan;
  Impulse o;
  o.row = min(max(p1 - 1, 0), F - 1);
  o.val = round_half_up(in ? r.amp * d.rinv * l.inv_unit : 0.0f);  // a select, not a branch
  return o;
}

__device__ __forceinline__ void lds_add(int *p, int v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Convolution of kHalf coarse samples c0 .. c0 + kHalf - 1 of the lane's
// column (fixed point in icol, row stride 64), scaled by `unit`, into
// out[0 .. kHalf).  Sample c reads rows alpha c + [0, 2K]; the caller only
// asks for samples whose rows are in the segment.
constexpr int kHalf = kAssaOut / 2;

__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Grid known at compile time: the A (kHalf - 1) + 2 KK + 1 rows are loaded
// once into registers (immediate LDS offsets), the taps sit in scalar
// registers.
template <int A, int KK>
__device__ __forceinline__ void conv_window(const int *icol, int c0, const float *hqs,
                                            float unit, float *out) {
  constexpr int W = A * (kHalf - 1) + 2 * KK + 1;
  float hv[KK];
#pragma unroll
  for (int q = 0; q < KK; ++q) hv[q] = uniform_f(hqs[q]);
  const int *base = icol + (size_t)(A * c0) * kWave;
  float z[W];
#pragma unroll
  for (int i = 0; i < W; ++i) z[i] = (float)base[i * kWave];
#pragma unroll
  for (int u = 0; u < kHalf; ++u) {
    float v = 0.0f;
#pragma unroll
    for (int q = 0; q < KK; ++q) v = fmaf(hv[q], z[A * u + q] - z[A * u + 2 * KK - q], v);
    out[u] = v * unit;
  }
}

// Any grid, nu <= kHalf samples: rows read straight from LDS.
__device__ __forceinline__ void conv_any(const int *icol, int c0, int nu, int alpha, int K,
                                         const float *hqs, float unit, float *out) {
  float acc[kHalf];
#pragma unroll
  for (int u = 0; u < kHalf; ++u) acc[u] = 0.0f;
  const int *base = icol + (size_t)alpha * c0 * kWave;
  const int ustep = alpha * kWave;
  for (int q = 0; q < K; ++q) {
    const float hq = hqs[q];
    const int *lo = base + q * kWave;
    const int *hi = base + (2 * K - q) * kWave;
#pragma unroll
    for (int u = 0; u < kHalf; ++u)
      if (u < nu) acc[u] = fmaf(hq, (float)lo[u * ustep] - (float)hi[u * ustep], acc[u]);
  }
#pragma unroll
  for (int u = 0; u < kHalf; ++u) out[u] = acc[u] * unit;
}

// A, KK > 0: the grid (alpha, K) is fixed at compile time (register-window
// convolution); A = 0: any grid.  The register budget is that of 6 waves per
// SIMD (80 VGPRs; 2 spills for (3, 12), 9 for (2, 16)), which the segment
// already caps a CU at (3 workgroups): at the paper shape, (3, 12) measured
// 7.24 ms against 7.55 ms at the budget of 7 waves (72 VGPRs, 7 spills) and
// 9.5 ms unconstrained (83 VGPRs, no spills, 5 waves).
template <int A, int KK>
__global__ __launch_bounds__(kAssaWaves * kWave) __attribute__((amdgpu_waves_per_eu(6)))
void assa_forward_kernel(
    const AssaRec *__restrict__ krec, AssaFwdArgs a) {
  extern __shared__ float seg[];  // [F][64]: fine row p of sensor column l at p*64 + l
  __shared__ float hqs[kAssaMaxK];

  const int64_t logical = xcd_logical(a.nlogical);
  if (logical >= a.nlogical) return;
  const int64_t tile = logical / a.nsg;
  const int sg = (int)(logical - tile * a.nsg);
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int j = sg * kWave + lane;
  const double4 s = a.sens[j < a.Nd ? j : a.Nd - 1];
  const TileInfo T = a.tiles[tile];

  // Shell of the lane's sensor: coarse sample c is the sampling-grid point
  // nb + c and reads the fine points fb + [alpha c, alpha c + 2K], with
  // fb = alpha nb - K.  Every impulse of the tile has fine point >= fb + 2K,
  // and every coarse sample it reaches is < Lc (host bound on Lc).
  int nb, fb;
  float inv_unit, unit;  // fixed-point scale of the lane's column
  {
    const double dx = s.x - T.cx, dy = s.y - T.cy, dz = s.z - T.cz;
    const double R = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
    nb = floor_div(shell_low(R, T.rho, a.ku, a.ku0) - a.K, a.alpha);
    fb = nb * a.alpha - a.K;
    // Every pair distance of the tile is >= r_low, so |sum of the column's
    // impulses| <= asum / r_low = 2^30 units.
    const double r_low = fmax(R - T.rho, a.min_dist);
    const double bound = (double)T.asum / r_low;
    unit = (float)(bound * 0x1p-30);
    inv_unit = bound > 0.0 ? (float)(0x1p30 / bound) : 0.0f;
  }
  Lane L;
  L.m2x = -2.0 * s.x;
  L.m2y = -2.0 * s.y;
  L.m2z = -2.0 * s.z;
  L.s2 = s.w;
  L.inv_unit = inv_unit;
  float *const col = seg + lane;
  int *const icol = reinterpret_cast<int *>(seg) + lane;
  const int per = (T.count + kAssaWaves - 1) / kAssaWaves;
  const int k0 = T.start + wave * per;
  const int k1 = min(T.start + T.count, k0 + per);

  // Passes over the shell, Lch coarse samples each (one pass unless the
  // shell's fine rows exceed the LDS budget).  Pass cc needs the impulses of
  // fine rows [alpha cc, alpha (cc + Lch - 1) + 2K], i.e. rows [0, F) of its
  // segment; impulses in the overlap of two passes are added in both, each
  // time reaching only that pass's coarse samples.
  for (int cc = 0; cc < a.Lc; cc += a.Lch) {
    const int nc = min(a.Lch, a.Lc - cc);
    const int fbc = fb + a.alpha * cc;
    // fine point k = fbc + p1 - 1 is kept iff 0 <= k < nfine and 0 <= p1 - 1 < F
    L.cst = a.ku0 - (double)fbc + 1.0;
    L.plo = max(1, 1 - fbc);
    L.pspan = max(0, min(a.F + 1, a.nfine - fbc + 1) - L.plo);
    if (cc > 0) __syncthreads();  // the previous pass's flush has read the segment
    {
      float4 *s4 = reinterpret_cast<float4 *>(seg);
      const int n4 = a.F * (kWave / 4);
      for (int i = t; i < n4; i += kAssaWaves * kWave) s4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (cc == 0)
        for (int i = t; i < a.K; i += kAssaWaves * kWave) hqs[i] = a.hq[i];
    }
    __syncthreads();

    // 1. Projection: wave w takes a contiguous share of the tile's kernels,
    //    kPairs pairs per iteration in one straight-line block so that their
    //    float64 chains interleave (the chain is latency-bound: 4 pairs per
    //    iteration measured 19% faster than 2, 8 slower again), the next
    //    records fetched before the LDS adds are issued.
    if (k0 < k1) {
      static_assert(kPairs == 4, "the loop below is written out for 4 pairs");
      const int last = k1 - 1;
      AssaRec ra = krec[k0], rb = krec[min(k0 + 1, last)], rc = krec[min(k0 + 2, last)],
                rd = krec[min(k0 + 3, last)];
      int k = k0;
      for (; k + 3 < k1; k += 4) {
        const Impulse ia = impulse(L, ra, a.F, a.ku);
        const Impulse ib = impulse(L, rb, a.F, a.ku);
        const Impulse ic = impulse(L, rc, a.F, a.ku);
        const Impulse id = impulse(L, rd, a.F, a.ku);
        ra = krec[min(k + 4, last)];
        rb = krec[min(k + 5, last)];
        rc = krec[min(k + 6, last)];
        rd = krec[min(k + 7, last)];
        lds_add(icol + ia.row * kWave, ia.val);
        lds_add(icol + ib.row * kWave, ib.val);
        lds_add(icol + ic.row * kWave, ic.val);
        lds_add(icol + id.row * kWave, id.val);
      }
      for (; k < k1; ++k) {
        const Impulse im = impulse(L, krec[k], a.F, a.ku);
        lds_add(icol + im.row * kWave, im.val);
      }
    }
    __syncthreads();

    // 2. Convolution and decimation, 64 coarse samples per round (kAssaOut
    //    per wave), from the fixed-point rows (converted to float in registers),
    //    results in float.  Round r writes rows [64r, 64r + 64) once every
    //    wave has read its inputs; later rounds read rows >= alpha (64r + 64),
    //    so nothing they need is overwritten.
    for (int c0 = 0; c0 < nc; c0 += kAssaPass) {
      const int cw = c0 + wave * kAssaOut;
      const int nu = min(kAssaOut, nc - cw);  // may be <= 0
      float acc[kAssaOut];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int nh = min(kHalf, nu - h * kHalf);  // samples of this half (may be <= 0)
        if (A > 0 && nh == kHalf)
          conv_window<(A > 0 ? A : 1), (KK > 0 ? KK : 1)>(icol, cw + h * kHalf, hqs, unit,
                                                         acc + h * kHalf);
        else if (nh > 0)
          conv_any(icol, cw + h * kHalf, nh, a.alpha, a.K, hqs, unit, acc + h * kHalf);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kAssaOut; ++u)
        if (u < nu) {
          const int c = cw + u;
          seg[c * kWave + ((lane + c) & (kWave - 1))] = acc[u];
        }
      __syncthreads();
    }

    // 3. Flush: wave w adds the rows of sensors w, w + 8, ...; lanes walk the
    //    coarse samples of one sensor (consecutive addresses of y).
    for (int row = wave; row < kWave; row += kAssaWaves) {
      const int jr = sg * kWave + row;
      if (jr >= a.Nd) break;
      const int nbr = __builtin_amdgcn_readlane(nb, row) + cc;
      float *yrow = a.y + (int64_t)jr * a.Nt;
      for (int c = lane; c < nc; c += kWave) {
        const int n = nbr + c;
        const float v = seg[c * kWave + ((row + c) & (kWave - 1))];
        if (n >= 0 && n < a.Nt && v != 0.0f) unsafeAtomicAdd(yrow + n, v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint, step 1: delta_conv[j][alpha m + phi] =
//   sum_t h(alpha t - phi) delta[j][m + t],  |alpha t - phi| <= K.
// ---------------------------------------------------------------------------
struct AssaConvArgs {
  const float *delta;
  float *dconv;
  int64_t total;  // Nd * Nt
  int32_t Nt, nfine, alpha, K, n_half;
  float h[2 * kAssaMaxK + 1];  // h(m) at index m + K
};

__global__ __launch_bounds__(256) void assa_dconv_kernel(AssaConvArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= a.total) return;
  const int64_t j = idx / a.Nt;
  const int m = (int)(idx - j * a.Nt);
  const float *d = a.delta + j * a.Nt;
  float *out = a.dconv + j * a.nfine + (int64_t)a.alpha * m;
  for (int phi = 0; phi < a.alpha; ++phi) {
    float acc = 0.0f;
    const int tlo = phi > 0 ? 1 - a.n_half : -a.n_half;
    for (int tt = tlo; tt <= a.n_half; ++tt) {
      const int n = m + tt;
      if (n >= 0 && n < a.Nt) acc = fmaf(a.h[a.alpha * tt - phi + a.K], d[n], acc);
    }
    out[phi] = acc;
  }
}

// ---------------------------------------------------------------------------
// Adjoint, step 2: back-projection g_i = sum_j delta_conv_j[k_ij] / r_ij.
// ---------------------------------------------------------------------------
struct AssaAdjArgs {
  const AssaRec *krec;
  const TileInfo *tiles;
  const int32_t *perm;
  const float *dconv;
  float *out;
  int64_t nlogical;  // pairs of adjoint tiles
  int64_t ntiles;    // adjoint tiles
  int32_t Nd, nfine, Fa;
  int32_t S;  // sensors per stage (<= kAdjSensorsPerStage; fewer when Fa is long)
  uint32_t fdiv;  // ceil(2^32 / Fa)
  double ku, ku0;
};

// Shell constants of the stage's sensors (threads t < nsb): kb = first fine
// point of the staged row, cst = ku0 - kb (the snap with the row offset
// folded in).
__device__ __forceinline__ void stage_consts(const double4 *sens, const TileInfo &T, int j0,
                                             int nsb, double ku, double ku0, int *kbs,
                                             double *csts) {
  const int t = threadIdx.x;
  if (t < nsb) {
    const double4 s = sens[j0 + t];
    const double dx = s.x - T.cx, dy = s.y - T.cy, dz = s.z - T.cz;
    const double R = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
    const int kb = shell_low(R, T.rho, ku, ku0);
    kbs[t] = kb;
    csts[t] = ku0 - (double)kb;
  }
}

// Element e of a stage (row js = e / Fa of the staged sensors, column
// c = e - js Fa) is handled by thread e mod BLOCK, in slot e / BLOCK of its
// register buffer; fdiv = ceil(2^32 / Fa) makes the row a multiply-high
// (exact for e < 2^16).
template <int BLOCK>
__device__ __forceinline__ void stage_load(const float *dconv, int nfine, int Fa, unsigned fdiv,
                                           int j0, int nsb, const int *kbs,
                                           float (&buf)[kAssaStageRegs]) {
  // Branch-free so that all loads issue back to back: an element outside the
  // stage or the grid loads a valid address (offset 0) and is replaced by 0.
  // n_sensors * n_fine < 2^31 (checked on the host): 32-bit offsets.
  const int n = nsb * Fa;
#pragma unroll
  for (int k = 0; k < kAssaStageRegs; ++k) {
    const int e = (int)threadIdx.x + k * BLOCK;
    const int js = min((int)__umulhi((unsigned)e, fdiv), nsb - 1);
    const int kk = kbs[js] + (e - js * Fa);
    const bool ok = e < n && kk >= 0 && kk < nfine;
    const float v = dconv[ok ? (unsigned)((j0 + js) * nfine + kk) : 0u];
    buf[k] = ok ? v : 0.0f;
  }
}

template <int BLOCK>
__device__ __forceinline__ void stage_store(float *stage, int n,
                                            const float (&buf)[kAssaStageRegs]) {
#pragma unroll
  for (int k = 0; k < kAssaStageRegs; ++k) {
    const int e = (int)threadIdx.x + k * BLOCK;
    if (e < n) stage[e] = buf[k];
  }
}

// The stages are software-pipelined: the next stage's rows are loaded into
// registers before the current stage's pairs are evaluated and written to
// LDS after them, so their latency overlaps the pair loop; the shell
// constants are double-buffered.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void assa_adjoint_kernel(const double4 *__restrict__ sens,
                                                            AssaAdjArgs a) {
  extern __shared__ float stage[];  // [S][Fa]
  __shared__ int kbs[2][kAdjSensorsPerStage];
  __shared__ double csts[2][kAdjSensorsPerStage];

  const int64_t logical = xcd_logical(a.nlogical);
  if (logical >= a.nlogical) return;
  // Tiles 2b and 2b + 1 (one 8x8x8 block of a lattice for 256-kernel tiles):
  // thread t takes kernels start + t and start + t + BLOCK.
  TileInfo T = a.tiles[2 * logical];
  if (2 * logical + 1 < a.ntiles) T = merge_tiles(T, a.tiles[2 * logical + 1]);
  const int t = threadIdx.x;
  const bool live0 = t < T.count, live1 = t + BLOCK < T.count;
  const int64_t i0 = T.start + (live0 ? t : 0), i1 = T.start + (live1 ? t + BLOCK : 0);
  const AssaRec r0 = a.krec[i0], r1 = a.krec[i1];
  const int pmax = a.Fa - 1;
  const double ax = -2.0 * r0.cx, ay = -2.0 * r0.cy, az = -2.0 * r0.cz;
  const double ac2 = fma(r0.cz, r0.cz, fma(r0.cy, r0.cy, r0.cx * r0.cx));
  const double bx = -2.0 * r1.cx, by = -2.0 * r1.cy, bz = -2.0 * r1.cz;
  const double bc2 = fma(r1.cz, r1.cz, fma(r1.cy, r1.cy, r1.cx * r1.cx));
  float buf[kAssaStageRegs];

  // Prologue: stage 0 into LDS, constants of stages 0 and 1.
  int nsb = min(a.S, a.Nd);
  stage_consts(sens, T, 0, nsb, a.ku, a.ku0, kbs[0], csts[0]);
  if (a.S < a.Nd)
    stage_consts(sens, T, a.S, min(a.S, a.Nd - a.S), a.ku, a.ku0, kbs[1], csts[1]);
  __syncthreads();
  stage_load<BLOCK>(a.dconv, a.nfine, a.Fa, a.fdiv, 0, nsb, kbs[0], buf);
  stage_store<BLOCK>(stage, nsb * a.Fa, buf);
  __syncthreads();

  double acc0 = 0.0, acc1 = 0.0;
  int cur = 0;
  for (int j0 = 0; j0 < a.Nd; j0 += a.S) {
    const int j1 = j0 + a.S;
    const int nsn = j1 < a.Nd ? min(a.S, a.Nd - j1) : 0;  // sensors of the next stage
    if (nsn > 0)
      stage_load<BLOCK>(a.dconv, a.nfine, a.Fa, a.fdiv, j1, nsn, kbs[cur ^ 1], buf);

    const double *cst = csts[cur];
    float p0 = 0.0f, p1 = 0.0f;
    for (int js = 0; js < nsb; ++js) {
      const double4 s = sens[j0 + js];
      const double c = cst[js];
      const Dist d0 = pair_dist(ax, ay, az, s.x, s.y, s.z, s.w + ac2);
      const Dist d1 = pair_dist(bx, by, bz, s.x, s.y, s.z, s.w + bc2);
      // floor(r ku + ku0) - kb is in [1, Fa - 1] by construction of kb and
      // Fa, so the folded value is >= 1 and truncation is the floor; the
      // unsigned clamp only keeps the read in the stage were that ever
      // violated.
      const unsigned q0 = min((unsigned)(int)fma(d0.r, a.ku, c), (unsigned)pmax);
      const unsigned q1 = min((unsigned)(int)fma(d1.r, a.ku, c), (unsigned)pmax);
      const float *row = stage + js * a.Fa;
      p0 = fmaf(row[q0], d0.rinv, p0);
      p1 = fmaf(row[q1], d1.rinv, p1);
    }
    acc0 += (double)p0;
    acc1 += (double)p1;

    __syncthreads();  // stage j0 and its constants are consumed
    if (nsn > 0) {
      stage_store<BLOCK>(stage, nsn * a.Fa, buf);
      const int j2 = j1 + a.S;
      if (j2 < a.Nd)
        stage_consts(sens, T, j2, min(a.S, a.Nd - j2), a.ku, a.ku0, kbs[cur], csts[cur]);
    }
    __syncthreads();
    cur ^= 1;
    nsb = nsn;
  }
  if (live0) a.out[a.perm[i0]] = (float)acc0;
  if (live1) a.out[a.perm[i1]] = (float)acc1;
}

double max_tile_rho(const std::vector<TileInfo> &tiles) {
  double r = 0.0;
  for (const TileInfo &t : tiles) r = std::max(r, t.rho);
  return r;
}

// h(m) = (1/2) d exp(-d^2 / (2 sigma^2)), d = -v m dt / alpha, m = -K..K.
double assa_h(const gpair_plan_s *p, const AssaGrid &g, int m) {
  const double d = -p->v * (double)m * (p->dt / (double)g.alpha);
  return 0.5 * d * std::exp(-(d * d) / (2.0 * g.sigma * g.sigma));
}

}  // namespace

gpair_status assa_grid(const gpair_plan_s *p, double sigma, AssaGrid *g) {
  if (!std::isfinite(sigma) || !(sigma > 0.0) || sigma > p->sigma_max)
    return GPAIR_ERR_SIGMA_RANGE;
  const double x = p->nsig * sigma / p->vdt;
  const double nh = std::max(1.0, std::ceil(x - 1e-9 * std::max(1.0, x)));
  if (!(nh <= (double)kAssaMaxK)) return GPAIR_ERR_INVALID_ARG;
  AssaGrid o{};
  o.sigma = sigma;
  o.n_half = (int32_t)nh;
  o.alpha = std::max(1, (int32_t)std::ceil(12.0 / nh));
  o.K = o.alpha * o.n_half;
  if (o.K > kAssaMaxK) return GPAIR_ERR_INVALID_ARG;
  const int64_t nfine = (int64_t)o.alpha * p->Nt;
  if (nfine * p->Nd >= (int64_t(1) << 31)) return GPAIR_ERR_INVALID_ARG;
  o.n_fine = (int32_t)nfine;
  // Every fine index the kernels form must stay well inside int range.
  double smax = 0.0, cmax = 0.0;
  for (int32_t j = 0; j < p->Nd; ++j) {
    const double *s = &p->host.sens[4 * (size_t)j];
    smax = std::max(smax, std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]));
  }
  for (const TileInfo &t : p->host.ftiles)
    cmax = std::max(cmax, std::sqrt(t.cx * t.cx + t.cy * t.cy + t.cz * t.cz) + t.rho);
  const double ku = (double)o.alpha / p->vdt;
  const double ku0 = 0.5 - (double)o.alpha * p->t0 / p->dt;
  if (!((smax + cmax) * ku + std::fabs(ku0) + 8.0 * (o.K + 2) < 1e9))
    return GPAIR_ERR_INVALID_ARG;
  const double rf = max_tile_rho(p->host.ftiles);
  double ra = 0.0;  // the back-projection works on pairs of adjoint tiles
  {
    const std::vector<TileInfo> &at = p->host.atiles;
    for (size_t b = 0; b < at.size(); b += 2) {
      const TileInfo m = b + 1 < at.size() ? merge_tiles(at[b], at[b + 1]) : at[b];
      ra = std::max(ra, m.rho);
    }
    ra *= 1.0 + 1e-9;  // device rounding of the same formula
  }
  const double lc = std::ceil(2.0 * rf * p->inv_vdt + 2.0 * nh) + 4.0;
  const double fa = std::ceil(2.0 * o.alpha * ra * p->inv_vdt) + 4.0;
  if (!(lc < 1e6 && fa < 1e6)) return GPAIR_ERR_INVALID_ARG;
  o.Lc = (int32_t)lc;
  // Forward: the whole shell in one pass if its fine rows fit, else passes of
  // Lch coarse samples with alpha (Lch - 1) + 2K + 1 <= the LDS rows.
  const int rows = kMaxSegmentBytes / (kWave * 4);
  const int full = o.alpha * (o.Lc - 1) + 2 * o.K + 1;
  o.Lch = full <= rows ? o.Lc : (rows - 2 * o.K - 1) / o.alpha + 1;
  if (o.Lch < 1) return GPAIR_ERR_INVALID_ARG;
  o.F = o.alpha * (o.Lch - 1) + 2 * o.K + 1;
  // Adjoint: as many sensors per stage as fit, at most kAdjSensorsPerStage.
  o.Fa = (int32_t)fa;
  // (and whose elements fit the registers of the software pipeline)
  o.S = (int32_t)std::min<int64_t>({kAdjSensorsPerStage, kMaxSegmentBytes / (4 * (int64_t)o.Fa),
                                    (int64_t)kAssaStageRegs * p->adj_tile / o.Fa});
  if (o.S < 1) return GPAIR_ERR_INVALID_ARG;
  *g = o;
  return GPAIR_OK;
}

size_t assa_work_bytes(const gpair_plan_s *p, const AssaGrid &g) {
  return (size_t)p->Nd * (size_t)g.n_fine * sizeof(float);
}

hipError_t launch_assa_prep(const gpair_plan_s *p, const float *x, hipStream_t s) {
  const unsigned int grid = (unsigned int)p->host.ftiles.size();
  assa_prep_kernel<<<grid, 256, 0, s>>>(x, ws_perm(p), (AssaRec *)ws_krec(p), ws_ftiles(p));
  return hipGetLastError();
}

hipError_t launch_assa_forward(const gpair_plan_s *p, const AssaGrid &g, float *y,
                               hipStream_t s) {
  AssaFwdArgs a{};
  a.sens = (const double4 *)ws_sens(p);
  a.tiles = ws_ftiles(p);
  a.y = y;
  a.Nd = p->Nd;
  a.Nt = p->Nt;
  a.nsg = (p->Nd + kWave - 1) / kWave;
  a.nlogical = (int64_t)p->host.ftiles.size() * a.nsg;
  a.nfine = g.n_fine;
  a.alpha = g.alpha;
  a.K = g.K;
  a.Lc = g.Lc;
  a.Lch = g.Lch;
  a.F = g.F;
  a.ku = (double)g.alpha / p->vdt;
  a.ku0 = 0.5 - (double)g.alpha * p->t0 / p->dt;
  a.min_dist = p->min_dist;
  for (int q = 0; q < g.K; ++q) a.hq[q] = (float)assa_h(p, g, g.K - q);
  const size_t lds = (size_t)g.F * kWave * sizeof(float);
  const unsigned int grid = xcd_blocks(a.nlogical);
  const int block = kAssaWaves * kWave;
  if (g.alpha == 3 && g.K == 12)
    assa_forward_kernel<3, 12><<<grid, block, lds, s>>>((const AssaRec *)ws_krec(p), a);
  else if (g.alpha == 2 && g.K == 16)
    assa_forward_kernel<2, 16><<<grid, block, lds, s>>>((const AssaRec *)ws_krec(p), a);
  else if (g.alpha == 4 && g.K == 12)
    assa_forward_kernel<4, 12><<<grid, block, lds, s>>>((const AssaRec *)ws_krec(p), a);
  else
    assa_forward_kernel<0, 0><<<grid, block, lds, s>>>((const AssaRec *)ws_krec(p), a);
  return hipGetLastError();
}

hipError_t launch_assa_dconv(const gpair_plan_s *p, const AssaGrid &g, const float *delta,
                             float *dconv, hipStream_t s) {
  AssaConvArgs a{};
  a.delta = delta;
  a.dconv = dconv;
  a.total = (int64_t)p->Nd * p->Nt;
  a.Nt = p->Nt;
  a.nfine = g.n_fine;
  a.alpha = g.alpha;
  a.K = g.K;
  a.n_half = g.n_half;
  for (int m = -g.K; m <= g.K; ++m) a.h[m + g.K] = (float)assa_h(p, g, m);
  const unsigned int grid = (unsigned int)((a.total + 255) / 256);
  assa_dconv_kernel<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_assa_adjoint(const gpair_plan_s *p, const AssaGrid &g, const float *dconv,
                               float *out, hipStream_t s) {
  AssaAdjArgs a{};
  a.krec = (const AssaRec *)ws_krec(p);
  a.tiles = ws_atiles(p);
  a.perm = ws_perm(p);
  a.dconv = dconv;
  a.out = out;
  a.ntiles = (int64_t)p->host.atiles.size();
  a.nlogical = (a.ntiles + 1) / 2;
  a.Nd = p->Nd;
  a.nfine = g.n_fine;
  a.Fa = g.Fa;
  a.S = g.S;
  a.fdiv = (uint32_t)(((uint64_t(1) << 32) + (uint64_t)g.Fa - 1) / (uint64_t)g.Fa);
  a.ku = (double)g.alpha / p->vdt;
  a.ku0 = 0.5 - (double)g.alpha * p->t0 / p->dt;
  const size_t lds = (size_t)g.Fa * g.S * sizeof(float);
  const unsigned int grid = xcd_blocks(a.nlogical);
  const double4 *sens = (const double4 *)ws_sens(p);
  switch (p->adj_tile) {
    case 64: assa_adjoint_kernel<64><<<grid, 64, lds, s>>>(sens, a); break;
    case 128: assa_adjoint_kernel<128><<<grid, 128, lds, s>>>(sens, a); break;
    default: assa_adjoint_kernel<256><<<grid, 256, lds, s>>>(sens, a); break;
  }
  return hipGetLastError();
}

}  // namespace gpair
