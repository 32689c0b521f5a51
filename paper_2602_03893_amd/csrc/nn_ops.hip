// nn_ops.hip -- gfx950 kernels of the learned warm-start network: 3D
// convolutions as implicit GEMMs on v_mfma_f32_16x16x32_bf16, their weight
// gradients, 2x2x2 max pooling, stride-2 transposed convolution, the 1x1x1
// head, the MSE loss, weight packing and trilinear upsampling.
//
// Activations are bfloat16 channels-last with a channel stride, so one lane
// loads 8 consecutive channels of a voxel as 16 bytes: exactly the 8
// k-values a lane feeds to the matrix core.  The convolutions compute the
// transposed product D[cout][voxel] = W[cout][k] * X[k][voxel] so that each
// lane of the result holds 4 consecutive output channels of one voxel (one
// 8-byte store).
//
// Matrix-core lane layout of v_mfma_f32_16x16x32_bf16 used throughout
// (lane l, r = l % 16, g = l / 16):
//   A (16 x 32): lane holds A[r][8g .. 8g+7]
//   B (32 x 16): lane holds B[8g .. 8g+7][r]
//   D (16 x 16): lane holds D[4g .. 4g+3][r]
#include "nn_internal.h"

namespace gpair {
namespace nn {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
typedef __attribute__((ext_vector_type(2))) unsigned int u32x2;

__device__ __forceinline__ float bf2f(uint32_t b16) { return __uint_as_float(b16 << 16); }

// float -> bfloat16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint32_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ float lo16(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi16(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ uint32_t pack2(float a, float b) { return f2bf(a) | (f2bf(b) << 16); }

__device__ __forceinline__ f32x4 mfma16(const u32x4 &a, const u32x4 &b, const f32x4 &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ u32x4 ld16(const uint16_t *p) {
  return *reinterpret_cast<const u32x4 *>(p);
}

__device__ __forceinline__ u32x4 zero4() { return u32x4{0u, 0u, 0u, 0u}; }

// Block index -> logical index such that consecutive logical blocks run on the
// same XCD (blocks are dispatched round-robin over the 8 XCDs), so that
// neighbouring voxel tiles share that XCD's L2.
__device__ __forceinline__ int64_t xcd_logical(int64_t b, int64_t nb) {
  if (nb % 8) return b;
  const int64_t per = nb / 8;
  return (b % 8) * per + b / 8;
}

// ---------------------------------------------------------------------------
// 3x3x3 convolution (and the data gradient of the stride-2 transposed
// convolution) as an implicit GEMM.  Each wave computes 64 output voxels x
// COW output channels; K runs over (tap, input channel) in steps of 32.
// ---------------------------------------------------------------------------
template <int CIN, int COW, int MODE>
__global__ __launch_bounds__(kConvBlock) void conv_mfma_kernel(ConvArgs a) {
  constexpr int TAPS = MODE == kConv3 ? 27 : 8;
  constexpr int MB = COW / 16;
  constexpr int KPT = CIN == 16 ? 1 : CIN / 32;
  constexpr int KSTEPS = CIN == 16 ? (TAPS + 1) / 2 : TAPS * KPT;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t nblk = (int64_t)gridDim.x;
  const int64_t lb = xcd_logical(blockIdx.x, nblk);
  const int64_t tile = lb / a.ngroups;
  const int co0 = (int)(lb % a.ngroups) * COW;
  const int64_t vbase = tile * kVoxPerBlock + wave * kVoxPerWave;
  if (vbase >= a.g.nvox) return;  // wave-uniform; no block-wide barrier follows

  const int ld = a.g.ld, lh = a.g.lh, lw = a.g.lw;
  const int D = 1 << ld, H = 1 << lh, W = 1 << lw;
  int64_t base[4];
  int zz[4], yy[4], xx[4];
  bool live[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t v = vbase + 16 * j + r;
    live[j] = v < a.g.nvox;
    xx[j] = (int)(v & (W - 1));
    yy[j] = (int)((v >> lw) & (H - 1));
    zz[j] = (int)((v >> (lw + lh)) & (D - 1));
    if (MODE == kConv3) {
      base[j] = v * a.in_cs;
    } else {
      const int64_t n = v >> (lw + lh + ld);
      const int64_t fine =
          ((((n << (ld + 1)) + 2 * zz[j]) << (lh + 1)) + 2 * yy[j]) * ((int64_t)2 << lw) +
          2 * xx[j];
      base[j] = fine * a.in_cs;
    }
  }

  f32x4 acc[MB][4];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const uint16_t *__restrict__ wp = a.w;
  const uint16_t *__restrict__ ip = a.in;
#pragma unroll 2
  for (int s = 0; s < KSTEPS; ++s) {
    int t, ci;
    if (CIN == 16) {
      t = 2 * s + (g >> 1);
      ci = 8 * (g & 1);
    } else {
      t = s / KPT;
      ci = (s % KPT) * 32 + 8 * g;
    }
    const bool tap_ok = t < TAPS;
    int dz = 0, dy = 0, dx = 0;
    int64_t toff;
    if (MODE == kConv3) {
      dz = t / 9 - 1;
      dy = (t / 3) % 3 - 1;
      dx = t % 3 - 1;
      toff = (int64_t)((dz << (lh + lw)) + (dy << lw) + dx) * a.in_cs;
    } else {
      const int tz = t >> 2, ty = (t >> 1) & 1, tx = t & 1;
      toff = ((int64_t)((tz << (lh + lw + 2)) + (ty << (lw + 1)) + tx)) * a.in_cs;
    }
    u32x4 af[MB], bfr[4];
#pragma unroll
    for (int m = 0; m < MB; ++m)
      af[m] = tap_ok ? ld16(wp + ((int64_t)t * a.cout + co0 + 16 * m + r) * CIN + ci) : zero4();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bool ok = tap_ok && live[j];
      if (MODE == kConv3)
        ok = ok && (unsigned)(zz[j] + dz) < (unsigned)D && (unsigned)(yy[j] + dy) < (unsigned)H &&
             (unsigned)(xx[j] + dx) < (unsigned)W;
      bfr[j] = ok ? ld16(ip + base[j] + toff + ci) : zero4();
    }
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[m][j] = mfma16(af[m], bfr[j], acc[m][j]);
  }

  // Epilogue: lane holds channels co .. co+3 of voxel vbase + 16 j + r.
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int co = co0 + 16 * m + 4 * g;
    float bias[4] = {0.f, 0.f, 0.f, 0.f};
    if (a.epi == GPAIR_NN_EPI_BIAS_RELU || a.epi == GPAIR_NN_EPI_BIAS) {
#pragma unroll
      for (int i = 0; i < 4; ++i) bias[i] = a.bias[co + i];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!live[j]) continue;
      const int64_t v = vbase + 16 * j + r;
      float o[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = acc[m][j][i] + bias[i];
      if (a.epi == GPAIR_NN_EPI_BIAS_RELU) {
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = fmaxf(o[i], 0.f);
      } else if (a.epi == GPAIR_NN_EPI_MASK) {
        const u32x2 m2 = *reinterpret_cast<const u32x2 *>(a.aux + v * a.aux_cs + co);
        if (!(lo16(m2[0]) > 0.f)) o[0] = 0.f;
        if (!(hi16(m2[0]) > 0.f)) o[1] = 0.f;
        if (!(lo16(m2[1]) > 0.f)) o[2] = 0.f;
        if (!(hi16(m2[1]) > 0.f)) o[3] = 0.f;
      }
      *reinterpret_cast<u32x2 *>(a.out + v * a.out_cs + co) =
          u32x2{pack2(o[0], o[1]), pack2(o[2], o[3])};
    }
  }
}

// 3x3x3 convolution of a single-channel input (the network's first layer):
// 27 x cout multiply-adds per voxel on the vector ALU, weights in LDS.
template <int COUT>
__global__ __launch_bounds__(256) void conv_c1_kernel(const uint16_t *__restrict__ in,
                                                      int64_t in_cs, Grid g,
                                                      const uint16_t *__restrict__ w,
                                                      const float *__restrict__ bias,
                                                      uint16_t *__restrict__ out,
                                                      int64_t out_cs, int epi) {
  __shared__ float ws[27][COUT];
  for (int i = threadIdx.x; i < 27 * COUT; i += 256) ws[i / COUT][i % COUT] = bf2f(w[i]);
  __syncthreads();
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= g.nvox) return;
  const int D = 1 << g.ld, H = 1 << g.lh, W = 1 << g.lw;
  const int x = (int)(v & (W - 1)), y = (int)((v >> g.lw) & (H - 1)),
            z = (int)((v >> (g.lw + g.lh)) & (D - 1));
  float acc[COUT];
#pragma unroll
  for (int c = 0; c < COUT; ++c) acc[c] = 0.f;
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    if ((unsigned)(z + dz) >= (unsigned)D || (unsigned)(y + dy) >= (unsigned)H ||
        (unsigned)(x + dx) >= (unsigned)W)
      continue;
    const int64_t u = v + ((int64_t)dz << (g.lw + g.lh)) + ((int64_t)dy << g.lw) + dx;
    const float xin = bf2f(in[u * in_cs]);
#pragma unroll
    for (int c = 0; c < COUT; ++c) acc[c] = fmaf(xin, ws[t][c], acc[c]);
  }
  uint16_t *o = out + v * out_cs;
#pragma unroll
  for (int c = 0; c < COUT; c += 4) {
    float q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      q[i] = acc[c + i];
      if (epi == GPAIR_NN_EPI_BIAS_RELU || epi == GPAIR_NN_EPI_BIAS) q[i] += bias[c + i];
      if (epi == GPAIR_NN_EPI_BIAS_RELU) q[i] = fmaxf(q[i], 0.f);
    }
    *reinterpret_cast<u32x2 *>(o + c) = u32x2{pack2(q[0], q[1]), pack2(q[2], q[3])};
  }
}

// ---------------------------------------------------------------------------
// Stride-2 2x2x2 transposed convolution: every coarse voxel writes its 8
// children, one tap (8 x a GEMM over the input channels) at a time.
// ---------------------------------------------------------------------------
template <int CIN, int COW>
__global__ __launch_bounds__(kConvBlock) void upconv_kernel(UpArgs a) {
  constexpr int MB = COW / 16;
  constexpr int KS = CIN / 32;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t lb = xcd_logical(blockIdx.x, (int64_t)gridDim.x);
  const int64_t tile = lb / a.ngroups;
  const int co0 = (int)(lb % a.ngroups) * COW;
  const int64_t vbase = tile * kVoxPerBlock + wave * kVoxPerWave;
  if (vbase >= a.g.nvox) return;
  const int ld = a.g.ld, lh = a.g.lh, lw = a.g.lw;
  const int D = 1 << ld, H = 1 << lh, W = 1 << lw;
  bool live[4];
  int64_t fine0[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t v = vbase + 16 * j + r;
    live[j] = v < a.g.nvox;
    const int x = (int)(v & (W - 1)), y = (int)((v >> lw) & (H - 1)),
              z = (int)((v >> (lw + lh)) & (D - 1));
    const int64_t n = v >> (lw + lh + ld);
    fine0[j] = ((((n << (ld + 1)) + 2 * z) << (lh + 1)) + 2 * y) * ((int64_t)2 << lw) + 2 * x;
  }
  u32x4 bfr[KS][4];
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      bfr[s][j] = live[j] ? ld16(a.in + (vbase + 16 * j + r) * a.in_cs + 32 * s + 8 * g)
                          : zero4();
  for (int t = 0; t < 8; ++t) {
    f32x4 acc[MB][4];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      u32x4 af[MB];
#pragma unroll
      for (int m = 0; m < MB; ++m)
        af[m] = ld16(a.w + ((int64_t)t * a.cout + co0 + 16 * m + r) * CIN + 32 * s + 8 * g);
#pragma unroll
      for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[m][j] = mfma16(af[m], bfr[s][j], acc[m][j]);
    }
    const int tz = t >> 2, ty = (t >> 1) & 1, tx = t & 1;
    const int64_t toff = ((int64_t)tz << (lh + lw + 2)) + ((int64_t)ty << (lw + 1)) + tx;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int co = co0 + 16 * m + 4 * g;
      float bias[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) bias[i] = a.bias[co + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!live[j]) continue;
        float o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = acc[m][j][i] + bias[i];
        *reinterpret_cast<u32x2 *>(a.out + (fine0[j] + toff) * a.out_cs + co) =
            u32x2{pack2(o[0], o[1]), pack2(o[2], o[3])};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradients.  dw[t][ci][co] = sum over base voxels of
//   conv3:            in[v + o(t)][ci] * gout[v][co]
//   transposed conv:  in[v][ci] * gout[child(v, t)][co]
// A block owns a group of taps and a fixed subset of 64-voxel chunks; for
// each chunk it stages both operands in LDS transposed to [channel][voxel]
// (so a lane's 8 k-values, 8 consecutive voxels, are one 16-byte read) and
// runs the (ci x co) tiles of every tap of its group on the matrix cores.
// Sums over chunks stay in registers; the block writes its partial sums and a
// second kernel adds the partials in a fixed order.
// ---------------------------------------------------------------------------
template <int CI, int CO, int MODE>
struct WgradShape {
  static constexpr int TAPS = MODE == kConv3 ? 27 : 8;
  static constexpr int CT = MODE == kConv3 ? CI : CO;  // channels of the tap operand
  static constexpr int CF = MODE == kConv3 ? CO : CI;  // channels of the fixed operand
  static constexpr int TPT = (CI / 16) * (CO / 16);    // 16x16 tiles per tap
  static constexpr int TPG0 = TAPS < 64 / TPT ? TAPS : (64 / TPT < 1 ? 1 : 64 / TPT);
  static constexpr int LDSCAP = (65536 / (2 * kLdsRow) - CF) / CT;  // 64 KiB per block
  static constexpr int TPG = TPG0 < LDSCAP ? TPG0 : (LDSCAP < 1 ? 1 : LDSCAP);
  static constexpr int GROUPS = (TAPS + TPG - 1) / TPG;
  static constexpr int R = (TPG * TPT + 3) / 4;  // tiles per wave
  static constexpr size_t LDS = (size_t)(TPG * CT + CF) * kLdsRow * 2;
};

// Stage 64 voxels x C channels of one operand into lds[c][voxel] (row stride
// kLdsRow), 4 voxels x 8 channels per task.  src(i) returns the element
// pointer of voxel i of the chunk or nullptr for a zero row.
template <int C, typename Src>
__device__ __forceinline__ void stage_T(uint16_t *lds, Src src) {
  constexpr int OCT = C / 8;
  for (int task = threadIdx.x; task < 16 * OCT; task += kConvBlock) {
    const int q = task / OCT, oc = task % OCT;
    u32x4 vals[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint16_t *p = src(4 * q + e);
      vals[e] = p ? ld16(p + 8 * oc) : zero4();
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      // channels 8 oc + 2 jj (low halves) and 8 oc + 2 jj + 1 (high halves)
      const uint32_t w0 = vals[0][jj], w1 = vals[1][jj], w2 = vals[2][jj], w3 = vals[3][jj];
      const u32x2 even = u32x2{(w0 & 0xffffu) | (w1 << 16), (w2 & 0xffffu) | (w3 << 16)};
      const u32x2 odd = u32x2{(w0 >> 16) | (w1 & 0xffff0000u), (w2 >> 16) | (w3 & 0xffff0000u)};
      *reinterpret_cast<u32x2 *>(lds + (8 * oc + 2 * jj) * kLdsRow + 4 * q) = even;
      *reinterpret_cast<u32x2 *>(lds + (8 * oc + 2 * jj + 1) * kLdsRow + 4 * q) = odd;
    }
  }
}

template <int CI, int CO, int MODE>
__global__ __launch_bounds__(kConvBlock) void wgrad_kernel(WgradArgs a) {
  using S = WgradShape<CI, CO, MODE>;
  extern __shared__ __align__(16) uint16_t lds[];
  uint16_t *ldsT = lds;                                // [TPG][CT][kLdsRow]
  uint16_t *ldsF = lds + S::TPG * S::CT * kLdsRow;     // [CF][kLdsRow]
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int split = blockIdx.x;
  const int grp = blockIdx.y;
  const int t0 = grp * S::TPG;
  const int ntap = (S::TAPS - t0) < S::TPG ? (S::TAPS - t0) : S::TPG;
  const int ld = a.g.ld, lh = a.g.lh, lw = a.g.lw;
  const int D = 1 << ld, H = 1 << lh, W = 1 << lw;

  f32x4 acc[S::R];
#pragma unroll
  for (int i = 0; i < S::R; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int64_t chunk = split; chunk < a.nchunks; chunk += a.nsplit) {
    const int64_t c0 = chunk * kChunk;
    __syncthreads();  // previous chunk's reads are done
    // fixed operand: voxel c0 + i of the base grid
    stage_T<S::CF>(ldsF, [&](int i) -> const uint16_t * {
      const int64_t v = c0 + i;
      return v < a.g.nvox ? a.f_src + v * a.f_cs : nullptr;
    });
    for (int tl = 0; tl < ntap; ++tl) {
      const int t = t0 + tl;
      stage_T<S::CT>(ldsT + tl * S::CT * kLdsRow, [&](int i) -> const uint16_t * {
        const int64_t v = c0 + i;
        if (v >= a.g.nvox) return nullptr;
        const int x = (int)(v & (W - 1)), y = (int)((v >> lw) & (H - 1)),
                  z = (int)((v >> (lw + lh)) & (D - 1));
        if (MODE == kConv3) {
          const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
          if ((unsigned)(z + dz) >= (unsigned)D || (unsigned)(y + dy) >= (unsigned)H ||
              (unsigned)(x + dx) >= (unsigned)W)
            return nullptr;
          const int64_t u = v + ((int64_t)dz << (lw + lh)) + ((int64_t)dy << lw) + dx;
          return a.t_src + u * a.t_cs;
        } else {
          const int tz = t >> 2, ty = (t >> 1) & 1, tx = t & 1;
          const int64_t n = v >> (lw + lh + ld);
          const int64_t fine =
              ((((n << (ld + 1)) + 2 * z + tz) << (lh + 1)) + 2 * y + ty) * ((int64_t)2 << lw) +
              2 * x + tx;
          return a.t_src + fine * a.t_cs;
        }
      });
    }
    __syncthreads();
#pragma unroll
    for (int ri = 0; ri < S::R; ++ri) {
      const int i = wave + 4 * ri;
      if (i >= ntap * S::TPT) break;
      const int tl = i / S::TPT, rem = i % S::TPT;
      const int mb = rem / (CO / 16), nb = rem % (CO / 16);  // ci tile, co tile
      const uint16_t *arow, *brow;
      if (MODE == kConv3) {
        arow = ldsT + (tl * S::CT + 16 * mb + r) * kLdsRow;  // input channels
        brow = ldsF + (16 * nb + r) * kLdsRow;               // output channels
      } else {
        arow = ldsF + (16 * mb + r) * kLdsRow;
        brow = ldsT + (tl * S::CT + 16 * nb + r) * kLdsRow;
      }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const u32x4 av = ld16(arow + 32 * ks + 8 * g);
        const u32x4 bv = ld16(brow + 32 * ks + 8 * g);
        acc[ri] = mfma16(av, bv, acc[ri]);
      }
    }
  }
  // partial[split][t][ci][co]; lane holds ci = 16 mb + 4 g + i, co = 16 nb + r
#pragma unroll
  for (int ri = 0; ri < S::R; ++ri) {
    const int i = wave + 4 * ri;
    if (i >= ntap * S::TPT) break;
    const int tl = i / S::TPT, rem = i % S::TPT;
    const int mb = rem / (CO / 16), nb = rem % (CO / 16);
    float *dst = a.partial + (((int64_t)split * S::TAPS + t0 + tl) * CI) * CO;
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[(int64_t)(16 * mb + 4 * g + k) * CO + 16 * nb + r] = acc[ri][k];
  }
}

// dw[t][0][co] of the single-channel first layer on the matrix cores:
// D[tap][co] = sum_v T[tap][v] F[co][v] with T[tap][v] = in[v + o(tap)] (rows
// 27..31 zero) and F = gout transposed, both staged per 64-voxel chunk.
template <int CO>
__global__ __launch_bounds__(kConvBlock) void wgrad_c1_kernel(const uint16_t *__restrict__ in,
                                                              int64_t in_cs,
                                                              const uint16_t *__restrict__ gout,
                                                              int64_t gout_cs, Grid g,
                                                              int nsplit,
                                                              float *__restrict__ partial) {
  constexpr int NB = CO / 16;
  constexpr int TILES = 2 * NB;  // two 16-row blocks of taps
  __shared__ __align__(16) uint16_t ldsT[32 * kLdsRow];
  __shared__ __align__(16) uint16_t ldsF[CO * kLdsRow];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int D = 1 << g.ld, H = 1 << g.lh, W = 1 << g.lw;
  const int64_t nchunks = (g.nvox + kChunk - 1) / kChunk;
  for (int i = threadIdx.x; i < 5 * kLdsRow; i += kConvBlock) ldsT[27 * kLdsRow + i] = 0;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += nsplit) {
    const int64_t c0 = chunk * kChunk;
    __syncthreads();
    stage_T<CO>(ldsF, [&](int i) -> const uint16_t * {
      const int64_t v = c0 + i;
      return v < g.nvox ? gout + v * gout_cs : nullptr;
    });
    for (int idx = threadIdx.x; idx < 27 * kChunk; idx += kConvBlock) {
      const int t = idx / kChunk, i = idx % kChunk;
      const int64_t v = c0 + i;
      uint16_t val = 0;
      if (v < g.nvox) {
        const int x = (int)(v & (W - 1)), y = (int)((v >> g.lw) & (H - 1)),
                  z = (int)((v >> (g.lw + g.lh)) & (D - 1));
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        if ((unsigned)(z + dz) < (unsigned)D && (unsigned)(y + dy) < (unsigned)H &&
            (unsigned)(x + dx) < (unsigned)W)
          val = in[(v + ((int64_t)dz << (g.lw + g.lh)) + ((int64_t)dy << g.lw) + dx) * in_cs];
      }
      ldsT[t * kLdsRow + i] = val;
    }
    __syncthreads();
    if (wave < TILES) {
      const int mb = wave / NB, nb = wave % NB;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const u32x4 av = ld16(ldsT + (16 * mb + r) * kLdsRow + 32 * ks + 8 * q);
        const u32x4 bv = ld16(ldsF + (16 * nb + r) * kLdsRow + 32 * ks + 8 * q);
        acc = mfma16(av, bv, acc);
      }
    }
  }
  if (wave < TILES) {
    const int mb = wave / NB, nb = wave % NB;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = 16 * mb + 4 * q + k;
      if (t < 27) partial[((int64_t)blockIdx.x * 27 + t) * CO + 16 * nb + r] = acc[k];
    }
  }
}

// ---------------------------------------------------------------------------
// Streamed weight gradients (grid rows of at least 8 voxels).  The operands
// are first rewritten in 8-voxel blocks, [voxel / 8][channel][8] (bfloat16),
// the conv input as three copies shifted by dx = -1, 0, +1 inside each row
// (zero outside), the transposed conv's output gradient split by child tap
// ([tap][coarse voxel / 8][channel][8]).  Every A / B fragment of the
// weight-gradient GEMM (K = voxels) is then one aligned 16-byte load of 8
// consecutive voxels of one channel, and the 64 lanes of a fragment read one
// contiguous 1 KiB block (16 channels x 32 voxels): a (dz, dy) shift moves
// whole 8-voxel blocks, a dx shift picks the copy.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t half_of(const u32x4 &q, int c) {
  const uint32_t w = q[c >> 1];
  return (c & 1) ? (w >> 16) : (w & 0xffffu);
}

// One 8-voxel group x 8 channels: out[c][j] = vox[j][c] for j < 8.
__device__ __forceinline__ u32x4 column(const u32x4 *vox, int c) {
  u32x4 o;
#pragma unroll
  for (int k = 0; k < 4; ++k) o[k] = half_of(vox[2 * k], c) | (half_of(vox[2 * k + 1], c) << 16);
  return o;
}

// xt[s][v / 8][c][v % 8] = x[v + s - 1][c] (0 where x + s - 1 leaves the row).
__global__ __launch_bounds__(256) void xt_shift3_kernel(const uint16_t *__restrict__ x,
                                                        int64_t cs, int C, Grid g,
                                                        uint16_t *__restrict__ xt) {
  const int oct = C / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (g.nvox / 8) * oct) return;
  const int64_t v0 = (idx / oct) * 8;
  const int oc = (int)(idx % oct);
  const int x0 = (int)(v0 & ((1 << g.lw) - 1));
  u32x4 q[10];
  q[0] = x0 > 0 ? ld16(x + (v0 - 1) * cs + 8 * oc) : zero4();
#pragma unroll
  for (int j = 0; j < 8; ++j) q[j + 1] = ld16(x + (v0 + j) * cs + 8 * oc);
  q[9] = x0 + 8 < (1 << g.lw) ? ld16(x + (v0 + 8) * cs + 8 * oc) : zero4();
#pragma unroll
  for (int sh = 0; sh < 3; ++sh)
#pragma unroll
    for (int c = 0; c < 8; ++c)
      *reinterpret_cast<u32x4 *>(xt + (int64_t)sh * C * g.nvox + (v0 / 8 * C + 8 * oc + c) * 8) =
          column(q + sh, c);
}

// Block-level channel sums of an 8 x 8 tile per thread: partial[block][C].
__device__ __forceinline__ void block_chan_sums(const u32x4 *vox, bool live, int C,
                                                float *__restrict__ partial) {
  __shared__ float sh[256][8];
  const int oct = C / 8;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    float t = 0.f;
    if (live)
#pragma unroll
      for (int j = 0; j < 8; ++j) t += bf2f(half_of(vox[j], c));
    sh[threadIdx.x][c] = t;
  }
  __syncthreads();
  if (threadIdx.x < C) {
    const int oc = threadIdx.x / 8, c = threadIdx.x % 8;
    float t = 0.f;
    for (int k = oc; k < 256; k += oct) t += sh[k][c];
    partial[(int64_t)blockIdx.x * C + threadIdx.x] = t;
  }
}

// xt[v / 8][c][v % 8] = x[v][c]; optional per-block channel sums.
__global__ __launch_bounds__(256) void xt_plain_kernel(const uint16_t *__restrict__ x,
                                                       int64_t cs, int C, int64_t V,
                                                       uint16_t *__restrict__ xt,
                                                       float *__restrict__ sums) {
  const int oct = C / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = idx < (V / 8) * oct;
  const int64_t v0 = (idx / oct) * 8;
  const int oc = (int)(idx % oct);
  u32x4 q[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) q[j] = live ? ld16(x + (v0 + j) * cs + 8 * oc) : zero4();
  if (live)
#pragma unroll
    for (int c = 0; c < 8; ++c)
      *reinterpret_cast<u32x4 *>(xt + (v0 / 8 * C + 8 * oc + c) * 8) = column(q, c);
  if (sums) block_chan_sums(q, live, C, sums);
}

// gt[t][v / 8][c][v % 8] = g[child(v, t)][c] for coarse voxel v; optional sums.
__global__ __launch_bounds__(256) void gt_s2d_kernel(const uint16_t *__restrict__ gf,
                                                     int64_t cs, int C, Grid cg,
                                                     uint16_t *__restrict__ gt,
                                                     float *__restrict__ sums) {
  const int oct = C / 8;
  const int64_t per_tap = (cg.nvox / 8) * oct;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = idx < 8 * per_tap;
  const int t = (int)(idx / per_tap);
  const int64_t rem = idx % per_tap;
  const int64_t v0 = (rem / oct) * 8;
  const int oc = (int)(rem % oct);
  const int ld = cg.ld, lh = cg.lh, lw = cg.lw;
  u32x4 q[8];
  if (live) {
    const int x0 = (int)(v0 & ((1 << lw) - 1)), y = (int)((v0 >> lw) & ((1 << lh) - 1)),
              z = (int)((v0 >> (lw + lh)) & ((1 << ld) - 1));
    const int64_t n = v0 >> (lw + lh + ld);
    const int tz = t >> 2, ty = (t >> 1) & 1, tx = t & 1;
    const int64_t f0 =
        ((((n << (ld + 1)) + 2 * z + tz) << (lh + 1)) + 2 * y + ty) * ((int64_t)2 << lw) +
        2 * x0 + tx;
#pragma unroll
    for (int j = 0; j < 8; ++j) q[j] = ld16(gf + (f0 + 2 * j) * cs + 8 * oc);
#pragma unroll
    for (int c = 0; c < 8; ++c)
      *reinterpret_cast<u32x4 *>(gt + (int64_t)t * C * cg.nvox + (v0 / 8 * C + 8 * oc + c) * 8) =
          column(q, c);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) q[j] = zero4();
  }
  if (sums) block_chan_sums(q, live, C, sums);
}

struct StreamArgs {
  const uint16_t *xt;  // conv3: [3][V/8][CI][8]; transposed conv: [V/8][CI][8]
  const uint16_t *gt;  // conv3: [V/8][CO][8];    transposed conv: [8][V/8][CO][8]
  Grid g;              // base grid (coarse for the transposed conv)
  int CI, CO, taps, nt, mgroups;
  int64_t kvox;        // voxels per split, multiple of 32
  float *partial;      // [nsplit][taps][CI][CO]
};

// One wave: taps [t0, t0 + nt) x NM input-channel blocks x NN output-channel
// blocks, summed over the split's voxels.  D[ci][co] += A[ci][v] B[v][co].
template <int NTM, int NM, int NN, int MODE>
__global__ __launch_bounds__(64) void wgrad_stream_kernel(StreamArgs a) {
  const int lane = threadIdx.x;
  const int r = lane & 15, q = lane >> 4;
  const int split = blockIdx.x;
  const int tg = blockIdx.y / a.mgroups, mg = blockIdx.y % a.mgroups;
  const int t0 = tg * a.nt;
  const int ntap = min(a.nt, a.taps - t0);
  const int ci0 = mg * NM * 16;
  const int64_t V = a.g.nvox;
  const int64_t vb = (int64_t)split * a.kvox;
  const int64_t ve = min(V, vb + a.kvox);
  const int ld = a.g.ld, lh = a.g.lh, lw = a.g.lw;
  const int D = 1 << ld, H = 1 << lh;
  f32x4 acc[NTM][NM][NN];
#pragma unroll
  for (int i = 0; i < NTM; ++i)
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
      for (int n = 0; n < NN; ++n) acc[i][m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  // per-tap element offsets: conv3, the dx copy plus the (dz, dy) shift in
  // whole 8-voxel blocks; transposed conv, the plane of child tap t
  int64_t aoff[NTM];
  int dzs[NTM], dys[NTM];
#pragma unroll
  for (int i = 0; i < NTM; ++i) {
    const int t = t0 + (i < ntap ? i : 0);
    if (MODE == kConv3) {
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      dzs[i] = dz;
      dys[i] = dy;
      const int64_t shift = ((int64_t)dz << (lh + lw)) + ((int64_t)dy << lw);  // multiple of 8
      aoff[i] = (int64_t)(dx + 1) * a.CI * V + shift * a.CI;
    } else {
      dzs[i] = dys[i] = 0;
      aoff[i] = (int64_t)t * a.CO * V;
    }
  }
  for (int64_t v0 = vb; v0 < ve; v0 += 32) {
    const int64_t v = v0 + 8 * q;  // this lane group's 8 voxels (one row segment)
    const bool vok = v < ve;
    const int y = (int)((v >> lw) & (H - 1)), z = (int)((v >> (lw + lh)) & (D - 1));
    if (MODE == kConv3) {
      const int64_t bo = (v >> 3) * a.CO * 8;
      const int64_t ao = (v >> 3) * a.CI * 8;
      u32x4 bf[NN];
#pragma unroll
      for (int n = 0; n < NN; ++n) bf[n] = vok ? ld16(a.gt + bo + (16 * n + r) * 8) : zero4();
#pragma unroll
      for (int i = 0; i < NTM; ++i) {
        if (i < ntap) {
          const bool ok = vok && (unsigned)(z + dzs[i]) < (unsigned)D &&
                          (unsigned)(y + dys[i]) < (unsigned)H;
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            const u32x4 af = ok ? ld16(a.xt + aoff[i] + ao + (ci0 + 16 * m + r) * 8) : zero4();
#pragma unroll
            for (int n = 0; n < NN; ++n) acc[i][m][n] = mfma16(af, bf[n], acc[i][m][n]);
          }
        }
      }
    } else {
      const int64_t ao = (v >> 3) * a.CI * 8;
      const int64_t bo = (v >> 3) * a.CO * 8;
      u32x4 af[NM];
#pragma unroll
      for (int m = 0; m < NM; ++m) af[m] = vok ? ld16(a.xt + ao + (ci0 + 16 * m + r) * 8) : zero4();
#pragma unroll
      for (int i = 0; i < NTM; ++i) {
        if (i < ntap) {
#pragma unroll
          for (int n = 0; n < NN; ++n) {
            const u32x4 bf = vok ? ld16(a.gt + aoff[i] + bo + (16 * n + r) * 8) : zero4();
#pragma unroll
            for (int m = 0; m < NM; ++m) acc[i][m][n] = mfma16(af[m], bf, acc[i][m][n]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NTM; ++i) {
    if (i < ntap) {
      float *dst = a.partial + ((int64_t)split * a.taps + t0 + i) * a.CI * a.CO;
#pragma unroll
      for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int n = 0; n < NN; ++n)
#pragma unroll
          for (int k = 0; k < 4; ++k)
            dst[(int64_t)(ci0 + 16 * m + 4 * q + k) * a.CO + 16 * n + r] = acc[i][m][n][k];
    }
  }
}

// red[gi][e] = sum over splits s in [64 gi, 64 gi + 64) of partial[s][e].
__global__ __launch_bounds__(256) void reduce_stage1_kernel(const float *__restrict__ partial,
                                                            int nsplit, int64_t n,
                                                            float *__restrict__ red) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int s0 = blockIdx.y * 64;
  const int s1 = min(nsplit, s0 + 64);
  float s = 0.f;
  for (int k = s0; k < s1; ++k) s += partial[(int64_t)k * n + e];
  red[(int64_t)blockIdx.y * n + e] = s;
}

// out[e] = sum_s partial[s][e], s ascending.
__global__ __launch_bounds__(256) void reduce_splits_kernel(const float *__restrict__ partial,
                                                            int nsplit, int64_t n,
                                                            float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int k = 0; k < nsplit; ++k) s += partial[(int64_t)k * n + e];
  out[e] = s;
}

// partial[b][c] = sum over block b's voxel range of x[v][c]; thread (row, c)
// adds a strided subset, rows are then added in order.
__global__ __launch_bounds__(256) void chansum_kernel(const uint16_t *__restrict__ x,
                                                      int64_t cs, int c, int64_t nvox,
                                                      float *__restrict__ partial) {
  __shared__ float sh[256];
  const int rows = 256 / c;
  const int row = threadIdx.x / c, ch = threadIdx.x % c;
  const int64_t per = (nvox + gridDim.x - 1) / gridDim.x;
  const int64_t v0 = (int64_t)blockIdx.x * per;
  const int64_t v1 = v0 + per < nvox ? v0 + per : nvox;
  float s = 0.f;
  if (row < rows)
    for (int64_t v = v0 + row; v < v1; v += rows) s += bf2f(x[v * cs + ch]);
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < c) {
    float tot = 0.f;
    for (int k = 0; k < rows; ++k) tot += sh[k * c + threadIdx.x];
    partial[(int64_t)blockIdx.x * c + threadIdx.x] = tot;
  }
}

// ---------------------------------------------------------------------------
// 2x2x2 max pooling; argmax code = child tap (z%2)*4 + (y%2)*2 + (x%2).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void maxpool_kernel(const uint16_t *__restrict__ in,
                                                      int64_t in_cs, Grid cg, int c,
                                                      uint16_t *__restrict__ out,
                                                      int64_t out_cs,
                                                      uint8_t *__restrict__ argmax) {
  const int oct = c / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= cg.nvox * oct) return;
  const int64_t v = idx / oct;
  const int oc = (int)(idx % oct);
  const int ld = cg.ld, lh = cg.lh, lw = cg.lw;
  const int x = (int)(v & ((1 << lw) - 1)), y = (int)((v >> lw) & ((1 << lh) - 1)),
            z = (int)((v >> (lw + lh)) & ((1 << ld) - 1));
  const int64_t n = v >> (lw + lh + ld);
  const int64_t fine0 =
      ((((n << (ld + 1)) + 2 * z) << (lh + 1)) + 2 * y) * ((int64_t)2 << lw) + 2 * x;
  float best[8];
  uint32_t arg[8];
  for (int t = 0; t < 8; ++t) {
    const int tz = t >> 2, ty = (t >> 1) & 1, tx = t & 1;
    const int64_t u = fine0 + ((int64_t)tz << (lh + lw + 2)) + ((int64_t)ty << (lw + 1)) + tx;
    const u32x4 q = ld16(in + u * in_cs + 8 * oc);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float val = (k & 1) ? hi16(q[k >> 1]) : lo16(q[k >> 1]);
      if (t == 0 || val > best[k]) {
        best[k] = val;
        arg[k] = t;
      }
    }
  }
  u32x4 o;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    o[k] = (__float_as_uint(best[2 * k]) >> 16) | (__float_as_uint(best[2 * k + 1]) & 0xffff0000u);
  *reinterpret_cast<u32x4 *>(out + v * out_cs + 8 * oc) = o;
  const u32x2 am = u32x2{arg[0] | (arg[1] << 8) | (arg[2] << 16) | (arg[3] << 24),
                         arg[4] | (arg[5] << 8) | (arg[6] << 16) | (arg[7] << 24)};
  *reinterpret_cast<u32x2 *>(argmax + v * c + 8 * oc) = am;
}

// gin[u] = (gskip[u] + [argmax(parent) == tap(u)] gout[parent]) * (act[u] > 0)
__global__ __launch_bounds__(256) void maxpool_bwd_kernel(
    const uint16_t *__restrict__ gout, int64_t gout_cs, const uint8_t *__restrict__ argmax,
    const uint16_t *gskip, int64_t gskip_cs, const uint16_t *__restrict__ act,
    int64_t act_cs, uint16_t *gin, int64_t gin_cs, Grid fg, int c) {
  const int oct = c / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= fg.nvox * oct) return;
  const int64_t u = idx / oct;
  const int oc = (int)(idx % oct);
  const int ld = fg.ld, lh = fg.lh, lw = fg.lw;
  const int x = (int)(u & ((1 << lw) - 1)), y = (int)((u >> lw) & ((1 << lh) - 1)),
            z = (int)((u >> (lw + lh)) & ((1 << ld) - 1));
  const int64_t n = u >> (lw + lh + ld);
  const int tap = ((z & 1) << 2) | ((y & 1) << 1) | (x & 1);
  const int64_t parent =
      ((((n << (ld - 1)) + (z >> 1)) << (lh - 1)) + (y >> 1)) * ((int64_t)1 << (lw - 1)) +
      (x >> 1);
  const u32x4 go = ld16(gout + parent * gout_cs + 8 * oc);
  const u32x2 am = *reinterpret_cast<const u32x2 *>(argmax + parent * c + 8 * oc);
  const u32x4 ac = ld16(act + u * act_cs + 8 * oc);
  u32x4 sk = zero4();
  if (gskip) sk = ld16(gskip + u * gskip_cs + 8 * oc);
  u32x4 o;
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    float r2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = 2 * k2 + h;
      const uint32_t code = (am[k >> 2] >> (8 * (k & 3))) & 0xffu;
      const float gv = h ? hi16(go[k2]) : lo16(go[k2]);
      const float sv = h ? hi16(sk[k2]) : lo16(sk[k2]);
      const float av = h ? hi16(ac[k2]) : lo16(ac[k2]);
      float s = sv + ((int)code == tap ? gv : 0.f);
      r2[h] = av > 0.f ? s : 0.f;
    }
    o[k2] = pack2(r2[0], r2[1]);
  }
  *reinterpret_cast<u32x4 *>(gin + u * gin_cs + 8 * oc) = o;
}

// ---------------------------------------------------------------------------
// 1x1x1 head with ReLU, and its backward (fixed-order partial sums).
// ---------------------------------------------------------------------------
template <int C>
__global__ __launch_bounds__(256) void head_kernel(const uint16_t *__restrict__ in, int64_t cs,
                                                   int64_t nvox, const float *__restrict__ w,
                                                   const float *__restrict__ b,
                                                   float *__restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= nvox) return;
  float s = 0.f;
#pragma unroll
  for (int oc = 0; oc < C / 8; ++oc) {
    const u32x4 q = ld16(in + v * cs + 8 * oc);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      s = fmaf((k & 1) ? hi16(q[k >> 1]) : lo16(q[k >> 1]), w[8 * oc + k], s);
  }
  out[v] = fmaxf(s + b[0], 0.f);
}

template <int C>
__global__ __launch_bounds__(256) void head_bwd_kernel(
    const uint16_t *__restrict__ in, int64_t cs, int64_t nvox, const float *__restrict__ w,
    const float *__restrict__ out, const float *__restrict__ gout, uint16_t *__restrict__ gin,
    int64_t gin_cs, float *__restrict__ partial) {
  __shared__ float sh[256][C + 1];
  float acc[C + 1];
#pragma unroll
  for (int k = 0; k <= C; ++k) acc[k] = 0.f;
  const int64_t per = (nvox + gridDim.x - 1) / gridDim.x;
  const int64_t v0 = (int64_t)blockIdx.x * per;
  const int64_t v1 = v0 + per < nvox ? v0 + per : nvox;
  for (int64_t v = v0 + threadIdx.x; v < v1; v += 256) {
    const float gp = out[v] > 0.f ? gout[v] : 0.f;
#pragma unroll
    for (int oc = 0; oc < C / 8; ++oc) {
      const u32x4 q = ld16(in + v * cs + 8 * oc);
      u32x4 o;
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) {
        const float x0 = lo16(q[k2]), x1 = hi16(q[k2]);
        const int c0 = 8 * oc + 2 * k2;
        acc[c0] = fmaf(gp, x0, acc[c0]);
        acc[c0 + 1] = fmaf(gp, x1, acc[c0 + 1]);
        o[k2] = pack2(x0 > 0.f ? gp * w[c0] : 0.f, x1 > 0.f ? gp * w[c0 + 1] : 0.f);
      }
      *reinterpret_cast<u32x4 *>(gin + v * gin_cs + 8 * oc) = o;
    }
    acc[C] += gp;
  }
#pragma unroll
  for (int k = 0; k <= C; ++k) sh[threadIdx.x][k] = acc[k];
  __syncthreads();
  if (threadIdx.x <= C) {
    float tot = 0.f;
    for (int i = 0; i < 256; ++i) tot += sh[i][threadIdx.x];
    partial[(int64_t)blockIdx.x * (C + 1) + threadIdx.x] = tot;
  }
}

// dw[k] = sum_b partial[b][k] (k < c), db = sum_b partial[b][c], b ascending.
__global__ __launch_bounds__(256) void head_reduce_kernel(const float *__restrict__ partial,
                                                          int nb, int c, float *__restrict__ dw,
                                                          float *__restrict__ db) {
  const int k = threadIdx.x;
  if (k > c) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * (c + 1) + k];
  if (k < c)
    dw[k] = s;
  else
    db[0] = s;
}

// ---------------------------------------------------------------------------
// MSE loss (float64 fixed-order sum) and its gradient.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mse_partial_kernel(int64_t n,
                                                          const float *__restrict__ pred,
                                                          const float *__restrict__ target,
                                                          float *__restrict__ gpred, float gscale,
                                                          double *__restrict__ partial) {
  __shared__ double sh[256];
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const float p = pred[i], t = target[i];
    const double d = (double)p - (double)t;
    s += d * d;
    if (gpred) gpred[i] = gscale * (p - t);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void mse_final_kernel(const double *__restrict__ partial,
                                                        int nparts, double inv_n,
                                                        double *__restrict__ loss) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += partial[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = sh[0] * inv_n;
}

// ---------------------------------------------------------------------------
// Weight packing, input conversion, trilinear upsampling.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_kernel(const float *__restrict__ master, int taps,
                                                   int cin, int cout, uint16_t *__restrict__ fwd,
                                                   uint16_t *__restrict__ dgrad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;  // master index [t][ci][co]
  const int64_t n = (int64_t)taps * cin * cout;
  if (e >= n) return;
  const int t = (int)(e / ((int64_t)cin * cout));
  const int ci = (int)((e / cout) % cin), co = (int)(e % cout);
  const uint16_t b = (uint16_t)f2bf(master[e]);
  fwd[((int64_t)t * cout + co) * cin + ci] = b;
  if (dgrad) {
    const int tf = taps == 27 ? 26 - t : t;
    dgrad[((int64_t)tf * cin + ci) * cout + co] = b;
  }
}

__global__ __launch_bounds__(256) void from_float_kernel(const float *__restrict__ x, float scale,
                                                         uint16_t *__restrict__ out, int64_t cs,
                                                         int64_t nvox) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v < nvox) out[v * cs] = (uint16_t)f2bf(scale * x[v]);
}

__device__ __forceinline__ void lin_src(int i, int n, int &i0, int &i1, float &f) {
  float s = 0.5f * (float)i - 0.25f;  // (i + 0.5) / 2 - 0.5
  if (s < 0.f) s = 0.f;
  i0 = (int)s;
  if (i0 > n - 1) i0 = n - 1;
  i1 = i0 + 1 < n ? i0 + 1 : n - 1;
  f = s - (float)i0;
}

__global__ __launch_bounds__(256) void upsample2_kernel(const float *__restrict__ x, int n, int d,
                                                        int h, int w, float *__restrict__ out) {
  const int64_t W2 = 2 * (int64_t)w, H2 = 2 * (int64_t)h, D2 = 2 * (int64_t)d;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * D2 * H2 * W2) return;
  const int X = (int)(e % W2), Y = (int)((e / W2) % H2), Z = (int)((e / (W2 * H2)) % D2);
  const int64_t b = e / (W2 * H2 * D2);
  int z0, z1, y0, y1, x0, x1;
  float fz, fy, fx;
  lin_src(Z, d, z0, z1, fz);
  lin_src(Y, h, y0, y1, fy);
  lin_src(X, w, x0, x1, fx);
  const float *p = x + b * d * h * w;
  auto at = [&](int z, int y, int xx) { return p[((int64_t)z * h + y) * w + xx]; };
  const float c00 = (1.f - fx) * at(z0, y0, x0) + fx * at(z0, y0, x1);
  const float c01 = (1.f - fx) * at(z0, y1, x0) + fx * at(z0, y1, x1);
  const float c10 = (1.f - fx) * at(z1, y0, x0) + fx * at(z1, y0, x1);
  const float c11 = (1.f - fx) * at(z1, y1, x0) + fx * at(z1, y1, x1);
  const float c0 = (1.f - fy) * c00 + fy * c01;
  const float c1 = (1.f - fy) * c10 + fy * c11;
  out[e] = (1.f - fz) * c0 + fz * c1;
}

unsigned int blocks_for(int64_t n, int per) { return (unsigned int)((n + per - 1) / per); }

template <int CIN, int COW, int MODE>
hipError_t conv_go(const ConvArgs &a0, hipStream_t s) {
  ConvArgs a = a0;
  a.ngroups = a.cout / COW;
  a.ntiles = (a.g.nvox + kVoxPerBlock - 1) / kVoxPerBlock;
  const int64_t nb = a.ntiles * a.ngroups;
  conv_mfma_kernel<CIN, COW, MODE><<<dim3((unsigned)nb), dim3(kConvBlock), 0, s>>>(a);
  return hipGetLastError();
}

template <int CIN, int MODE>
hipError_t conv_cow(const ConvArgs &a, hipStream_t s) {
  switch (a.cout) {
    case 16: return conv_go<CIN, 16, MODE>(a, s);
    case 32: return conv_go<CIN, 32, MODE>(a, s);
    default: return conv_go<CIN, 64, MODE>(a, s);  // 64 and 128 (two groups)
  }
}

template <int CIN, int COW>
hipError_t up_go(const UpArgs &a0, hipStream_t s) {
  UpArgs a = a0;
  a.ngroups = a.cout / COW;
  a.ntiles = (a.g.nvox + kVoxPerBlock - 1) / kVoxPerBlock;
  const int64_t nb = a.ntiles * a.ngroups;
  upconv_kernel<CIN, COW><<<dim3((unsigned)nb), dim3(kConvBlock), 0, s>>>(a);
  return hipGetLastError();
}

template <int CIN>
hipError_t up_cow(const UpArgs &a, hipStream_t s) {
  switch (a.cout) {
    case 16: return up_go<CIN, 16>(a, s);
    case 32: return up_go<CIN, 32>(a, s);
    default: return up_go<CIN, 64>(a, s);
  }
}

template <int CI, int CO, int MODE>
hipError_t wgrad_go(const WgradArgs &a0, float *dw, hipStream_t s) {
  using S = WgradShape<CI, CO, MODE>;
  WgradArgs a = a0;
  const size_t lds = S::LDS;
  wgrad_kernel<CI, CO, MODE>
      <<<dim3((unsigned)a.nsplit, (unsigned)S::GROUPS), dim3(kConvBlock), lds, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)S::TAPS * CI * CO;
  reduce_splits_kernel<<<blocks_for(n, 256), 256, 0, s>>>(a.partial, a.nsplit, n, dw);
  return hipGetLastError();
}

template <int CI, int MODE>
hipError_t wgrad_co(const WgradArgs &a, int cout, float *dw, hipStream_t s) {
  switch (cout) {
    case 16: return wgrad_go<CI, 16, MODE>(a, dw, s);
    case 32: return wgrad_go<CI, 32, MODE>(a, dw, s);
    case 64: return wgrad_go<CI, 64, MODE>(a, dw, s);
    default: return wgrad_go<CI, 128, MODE>(a, dw, s);
  }
}

template <int MODE>
hipError_t wgrad_ci(const WgradArgs &a, int cin, int cout, float *dw, hipStream_t s) {
  switch (cin) {
    case 16: return wgrad_co<16, MODE>(a, cout, dw, s);
    case 32: return wgrad_co<32, MODE>(a, cout, dw, s);
    case 64: return wgrad_co<64, MODE>(a, cout, dw, s);
    default: return wgrad_co<128, MODE>(a, cout, dw, s);
  }
}

template <int CI, int CO, int MODE>
size_t wgrad_lds() { return WgradShape<CI, CO, MODE>::LDS; }

}  // namespace

int wgrad_splits(int64_t nvox, int taps, int cin, int cout) {
  const int64_t chunks = (nvox + kChunk - 1) / kChunk;
  if (cin == 1) {
    int64_t ns = nvox / 4096;
    if (ns < 1) ns = 1;
    if (ns > kWgradBlocks) ns = kWgradBlocks;
    return (int)ns;
  }
  const int tpt = (cin / 16) * (cout / 16);
  int tpg = 64 / tpt < 1 ? 1 : 64 / tpt;
  if (tpg > taps) tpg = taps;
  const int ct = taps == 27 ? cin : cout;
  const int cf = taps == 27 ? cout : cin;
  const int cap = (65536 / (2 * kLdsRow) - cf) / ct;
  if (tpg > cap) tpg = cap < 1 ? 1 : cap;
  const int groups = (taps + tpg - 1) / tpg;
  int64_t ns = (kWgradBlocks + groups - 1) / groups;
  const int64_t budget = (int64_t)(kWgradPartialCap / ((size_t)taps * cin * cout * 4));
  if (ns > budget) ns = budget;
  if (ns > chunks) ns = chunks;
  if (ns < 1) ns = 1;
  return (int)ns;
}

hipError_t launch_conv3(const ConvArgs &a, int cin, int mode, hipStream_t s) {
  if (mode == kConv3) {
    switch (cin) {
      case 16: return conv_cow<16, kConv3>(a, s);
      case 32: return conv_cow<32, kConv3>(a, s);
      case 64: return conv_cow<64, kConv3>(a, s);
      default: return conv_cow<128, kConv3>(a, s);
    }
  }
  switch (cin) {
    case 16: return conv_cow<16, kUpDgrad>(a, s);
    case 32: return conv_cow<32, kUpDgrad>(a, s);
    default: return conv_cow<64, kUpDgrad>(a, s);
  }
}

hipError_t launch_conv_c1(const uint16_t *in, int64_t in_cs, const Grid &g, const uint16_t *w,
                          const float *bias, uint16_t *out, int64_t out_cs, int cout, int epi,
                          hipStream_t s) {
  const unsigned nb = blocks_for(g.nvox, 256);
  switch (cout) {
    case 16: conv_c1_kernel<16><<<nb, 256, 0, s>>>(in, in_cs, g, w, bias, out, out_cs, epi); break;
    case 32: conv_c1_kernel<32><<<nb, 256, 0, s>>>(in, in_cs, g, w, bias, out, out_cs, epi); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_upconv(const UpArgs &a, int cin, hipStream_t s) {
  switch (cin) {
    case 32: return up_cow<32>(a, s);
    case 64: return up_cow<64>(a, s);
    default: return up_cow<128>(a, s);
  }
}

hipError_t launch_wgrad(const WgradArgs &a, int mode, int cin, int cout, float *dw,
                        hipStream_t s) {
  return mode == kConv3 ? wgrad_ci<kConv3>(a, cin, cout, dw, s)
                        : wgrad_ci<kUpDgrad>(a, cin, cout, dw, s);
}

hipError_t launch_wgrad_c1(const uint16_t *in, int64_t in_cs, const uint16_t *gout,
                           int64_t gout_cs, const Grid &g, int cout, float *partial,
                           int nsplit, float *dw, hipStream_t s) {
  if (cout == 16)
    wgrad_c1_kernel<16><<<nsplit, kConvBlock, 0, s>>>(in, in_cs, gout, gout_cs, g, nsplit, partial);
  else
    wgrad_c1_kernel<32><<<nsplit, kConvBlock, 0, s>>>(in, in_cs, gout, gout_cs, g, nsplit, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = 27 * (int64_t)cout;
  reduce_splits_kernel<<<blocks_for(n, 256), 256, 0, s>>>(partial, nsplit, n, dw);
  return hipGetLastError();
}

hipError_t launch_chansum(const uint16_t *x, int64_t cs, int c, int64_t nvox, float *partial,
                          float *out, hipStream_t s) {
  int nb = (int)((nvox + 255) / 256);
  if (nb > kSumBlocks) nb = kSumBlocks;
  chansum_kernel<<<nb, 256, 0, s>>>(x, cs, c, nvox, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  reduce_splits_kernel<<<blocks_for(c, 256), 256, 0, s>>>(partial, nb, c, out);
  return hipGetLastError();
}

hipError_t launch_maxpool(const uint16_t *in, int64_t in_cs, const Grid &coarse, int c,
                          uint16_t *out, int64_t out_cs, uint8_t *argmax, hipStream_t s) {
  maxpool_kernel<<<blocks_for(coarse.nvox * (c / 8), 256), 256, 0, s>>>(in, in_cs, coarse, c,
                                                                        out, out_cs, argmax);
  return hipGetLastError();
}

hipError_t launch_maxpool_bwd(const uint16_t *gout, int64_t gout_cs, const uint8_t *argmax,
                              const uint16_t *gskip, int64_t gskip_cs, const uint16_t *act,
                              int64_t act_cs, uint16_t *gin, int64_t gin_cs,
                              const Grid &fine, int c, hipStream_t s) {
  maxpool_bwd_kernel<<<blocks_for(fine.nvox * (c / 8), 256), 256, 0, s>>>(
      gout, gout_cs, argmax, gskip, gskip_cs, act, act_cs, gin, gin_cs, fine, c);
  return hipGetLastError();
}

hipError_t launch_head(const uint16_t *in, int64_t cs, int c, int64_t nvox, const float *w,
                       const float *b, float *out, hipStream_t s) {
  const unsigned nb = blocks_for(nvox, 256);
  if (c == 16)
    head_kernel<16><<<nb, 256, 0, s>>>(in, cs, nvox, w, b, out);
  else
    head_kernel<32><<<nb, 256, 0, s>>>(in, cs, nvox, w, b, out);
  return hipGetLastError();
}

hipError_t launch_head_bwd(const uint16_t *in, int64_t cs, int c, int64_t nvox,
                           const float *w, const float *out, const float *gout,
                           uint16_t *gin, int64_t gin_cs, float *partial, float *dw,
                           float *db, hipStream_t s) {
  int nb = (int)((nvox + 255) / 256);
  if (nb > kSumBlocks) nb = kSumBlocks;
  if (c == 16)
    head_bwd_kernel<16><<<nb, 256, 0, s>>>(in, cs, nvox, w, out, gout, gin, gin_cs, partial);
  else
    head_bwd_kernel<32><<<nb, 256, 0, s>>>(in, cs, nvox, w, out, gout, gin, gin_cs, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  head_reduce_kernel<<<1, 256, 0, s>>>(partial, nb, c, dw, db);
  return hipGetLastError();
}

hipError_t launch_mse(int64_t n, const float *pred, const float *target, float *gpred,
                      double *loss, double *partial, hipStream_t s) {
  mse_partial_kernel<<<GPAIR_NN_MSE_PARTIALS, 256, 0, s>>>(n, pred, target, gpred,
                                                           (float)(2.0 / (double)n), partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mse_final_kernel<<<1, 256, 0, s>>>(partial, GPAIR_NN_MSE_PARTIALS, 1.0 / (double)n, loss);
  return hipGetLastError();
}

hipError_t launch_pack(const float *master, int taps, int cin, int cout, uint16_t *fwd,
                       uint16_t *dgrad, hipStream_t s) {
  const int64_t n = (int64_t)taps * cin * cout;
  pack_kernel<<<blocks_for(n, 256), 256, 0, s>>>(master, taps, cin, cout, fwd, dgrad);
  return hipGetLastError();
}

hipError_t launch_from_float(const float *x, float scale, uint16_t *out, int64_t cs,
                             int64_t nvox, hipStream_t s) {
  from_float_kernel<<<blocks_for(nvox, 256), 256, 0, s>>>(x, scale, out, cs, nvox);
  return hipGetLastError();
}

hipError_t launch_upsample2(const float *x, int n, int d, int h, int w, float *out,
                            hipStream_t s) {
  const int64_t tot = (int64_t)n * 8 * d * h * w;
  upsample2_kernel<<<blocks_for(tot, 256), 256, 0, s>>>(x, n, d, h, w, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weight-gradient jobs: path choice, scratch layout, launches.
// ---------------------------------------------------------------------------
namespace {

struct StreamCfg {
  int ntm, nm, nn;  // template shape
  int nt, mgroups, tgroups;
};

// Tiles per wave (taps x input-channel blocks x output-channel blocks) are
// kept to at most 16 (64 accumulator registers) so that several waves per SIMD
// hide the load latency of the streamed operands.
StreamCfg stream_cfg(int taps, int cin, int cout) {
  StreamCfg c;
  const int tpt = (cin / 16) * (cout / 16);
  c.nn = cout / 16;
  c.nm = cin / 16;
  c.mgroups = 1;
  if (tpt <= 16) {
    if (taps == 27)
      c.ntm = tpt == 1 ? 9 : tpt == 2 ? 7 : tpt == 4 ? 4 : tpt == 8 ? 2 : 1;
    else
      c.ntm = tpt <= 2 ? 8 : tpt == 4 ? 4 : tpt == 8 ? 2 : 1;
  } else {
    c.ntm = 1;
    c.nm = 16 / c.nn;
    c.mgroups = (cin / 16) / c.nm;
  }
  c.nt = c.ntm < taps ? c.ntm : taps;
  c.tgroups = (taps + c.nt - 1) / c.nt;
  return c;
}

enum WgradPath { kPathC1, kPathStaged, kPathStream };

struct WgradLayout {
  int path, nsplit, g2, nblk_sum, g2sum;
  int64_t kvox;
  size_t partial, red2, xt, gt, sums, sums2, total;
};

// base: the conv grid (conv3) or the coarse grid (transposed conv).
WgradLayout wgrad_layout(int mode, const Grid &base, int cin, int cout) {
  WgradLayout L{};
  const int taps = mode == kConv3 ? 27 : 8;
  const int64_t V = base.nvox;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) & ~size_t(255);
    return o;
  };
  if (mode == kConv3 && cin == 1) {
    L.path = kPathC1;
  } else if (base.lw >= 3) {
    L.path = kPathStream;
  } else {
    L.path = kPathStaged;
  }
  const int64_t n = (int64_t)taps * (cin == 1 ? 1 : cin) * cout;
  if (L.path == kPathStream) {
    const StreamCfg c = stream_cfg(taps, cin, cout);
    const int groups = c.tgroups * c.mgroups;
    int64_t ns = (4096 + groups - 1) / groups;
    const int64_t budget = (int64_t)(kWgradPartialCap / ((size_t)n * 4));
    if (ns > budget) ns = budget;
    int64_t kv = (V + ns - 1) / ns;
    if (kv < 256) kv = 256;
    kv = (kv + 31) / 32 * 32;
    L.kvox = kv;
    L.nsplit = (int)((V + kv - 1) / kv);
    L.g2 = (L.nsplit + 63) / 64;
    L.partial = take((size_t)L.nsplit * n * 4);
    L.red2 = take((size_t)L.g2 * n * 4);
    const int64_t vfine_or_same = mode == kConv3 ? V : 8 * V;
    L.xt = take((size_t)(mode == kConv3 ? 3 : 1) * cin * V * 2);
    L.gt = take((size_t)cout * vfine_or_same * 2);
    const int64_t threads = (vfine_or_same / 8) * (cout / 8);
    L.nblk_sum = (int)((threads + 255) / 256);
  } else {
    L.nsplit = wgrad_splits(V, taps, cin, cout);
    L.partial = take((size_t)L.nsplit * n * 4);
    L.g2 = 0;
    L.nblk_sum = kSumBlocks;
  }
  L.g2sum = (L.nblk_sum + 63) / 64;
  L.sums = take((size_t)L.nblk_sum * cout * 4);
  L.sums2 = take((size_t)L.g2sum * cout * 4);
  L.total = off;
  return L;
}

// out[e] = sum over s < ns of partial[s][e], in a fixed order (two stages when
// there are many splits).
hipError_t reduce_fixed(const float *partial, int ns, int64_t n, float *red2, float *out,
                        hipStream_t s) {
  if (ns <= 64 || !red2) {
    reduce_splits_kernel<<<blocks_for(n, 256), 256, 0, s>>>(partial, ns, n, out);
    return hipGetLastError();
  }
  const int g2 = (ns + 63) / 64;
  reduce_stage1_kernel<<<dim3(blocks_for(n, 256), g2), 256, 0, s>>>(partial, ns, n, red2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  reduce_splits_kernel<<<blocks_for(n, 256), 256, 0, s>>>(red2, g2, n, out);
  return hipGetLastError();
}

template <int NTM, int NM, int NN, int MODE>
hipError_t stream_go(const StreamArgs &a, int nsplit, int groups, hipStream_t s) {
  wgrad_stream_kernel<NTM, NM, NN, MODE><<<dim3((unsigned)nsplit, (unsigned)groups), 64, 0, s>>>(a);
  return hipGetLastError();
}

template <int MODE>
hipError_t stream_dispatch(const StreamCfg &c, const StreamArgs &a, int nsplit, hipStream_t s) {
  const int groups = c.tgroups * c.mgroups;
#define GPAIR_SW(T, M, N) \
  if (c.ntm == T && c.nm == M && c.nn == N) return stream_go<T, M, N, MODE>(a, nsplit, groups, s);
  GPAIR_SW(9, 1, 1) GPAIR_SW(7, 2, 1) GPAIR_SW(7, 1, 2) GPAIR_SW(4, 2, 2) GPAIR_SW(4, 4, 1)
  GPAIR_SW(4, 1, 4) GPAIR_SW(2, 4, 2) GPAIR_SW(2, 2, 4) GPAIR_SW(2, 8, 1) GPAIR_SW(2, 1, 8)
  GPAIR_SW(1, 4, 4) GPAIR_SW(1, 8, 2) GPAIR_SW(1, 2, 8) GPAIR_SW(8, 2, 1)
#undef GPAIR_SW
  return hipErrorInvalidValue;
}

}  // namespace

size_t wgrad_scratch_bytes(int mode, const Grid &base, int cin, int cout) {
  return wgrad_layout(mode, base, cin, cout).total;
}

hipError_t launch_wgrad_job(const WgradJob &j, void *scratch, float *dw, float *db,
                            hipStream_t s) {
  const WgradLayout L = wgrad_layout(j.mode, j.base, j.cin, j.cout);
  char *base = static_cast<char *>(scratch);
  float *partial = reinterpret_cast<float *>(base + L.partial);
  const int taps = j.mode == kConv3 ? 27 : 8;
  const int64_t n = (int64_t)taps * (j.cin == 1 ? 1 : j.cin) * j.cout;
  hipError_t e;
  if (L.path == kPathC1) {
    e = launch_wgrad_c1(j.x, j.x_cs, j.g, j.g_cs, j.base, j.cout, partial, L.nsplit, dw, s);
    if (e != hipSuccess) return e;
  } else if (L.path == kPathStaged) {
    WgradArgs a{};
    if (j.mode == kConv3) {
      a.t_src = j.x;
      a.t_cs = j.x_cs;
      a.f_src = j.g;
      a.f_cs = j.g_cs;
    } else {
      a.t_src = j.g;
      a.t_cs = j.g_cs;
      a.f_src = j.x;
      a.f_cs = j.x_cs;
    }
    a.g = j.base;
    a.partial = partial;
    a.nsplit = L.nsplit;
    a.nchunks = (j.base.nvox + kChunk - 1) / kChunk;
    e = launch_wgrad(a, j.mode, j.cin, j.cout, dw, s);
    if (e != hipSuccess) return e;
  } else {
    uint16_t *xt = reinterpret_cast<uint16_t *>(base + L.xt);
    uint16_t *gt = reinterpret_cast<uint16_t *>(base + L.gt);
    float *sums = db ? reinterpret_cast<float *>(base + L.sums) : nullptr;
    const int64_t V = j.base.nvox;
    if (j.mode == kConv3) {
      xt_shift3_kernel<<<blocks_for((V / 8) * (j.cin / 8), 256), 256, 0, s>>>(j.x, j.x_cs, j.cin,
                                                                              j.base, xt);
      xt_plain_kernel<<<L.nblk_sum, 256, 0, s>>>(j.g, j.g_cs, j.cout, V, gt, sums);
    } else {
      xt_plain_kernel<<<blocks_for((V / 8) * (j.cin / 8), 256), 256, 0, s>>>(j.x, j.x_cs, j.cin,
                                                                             V, xt, nullptr);
      gt_s2d_kernel<<<L.nblk_sum, 256, 0, s>>>(j.g, j.g_cs, j.cout, j.base, gt, sums);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const StreamCfg c = stream_cfg(taps, j.cin, j.cout);
    StreamArgs a;
    a.xt = xt;
    a.gt = gt;
    a.g = j.base;
    a.CI = j.cin;
    a.CO = j.cout;
    a.taps = taps;
    a.nt = c.nt;
    a.mgroups = c.mgroups;
    a.kvox = L.kvox;
    a.partial = partial;
    e = j.mode == kConv3 ? stream_dispatch<kConv3>(c, a, L.nsplit, s)
                         : stream_dispatch<kUpDgrad>(c, a, L.nsplit, s);
    if (e != hipSuccess) return e;
    e = reduce_fixed(partial, L.nsplit, n, reinterpret_cast<float *>(base + L.red2), dw, s);
    if (e != hipSuccess) return e;
    if (db)
      return reduce_fixed(sums, L.nblk_sum, j.cout, reinterpret_cast<float *>(base + L.sums2),
                          db, s);
    return hipSuccess;
  }
  if (!db) return hipSuccess;
  // bias gradient of the other paths: channel sums of the output gradient
  const int64_t nv = j.mode == kConv3 ? j.base.nvox : 8 * j.base.nvox;
  return launch_chansum(j.g, j.g_cs, j.cout, nv, reinterpret_cast<float *>(base + L.sums), db, s);
}

}  // namespace nn
}  // namespace gpair
