// peaks.hip -- issue-rate probes of the vector ALU instructions the operators
// are made of (gpair_peak_probe): float32 FMA, float64 FMA, the float32 exp2
// and reciprocal square root, the float64 reciprocal square root and the
// float64 <-> float32 conversions.
//
// Each thread runs kChains independent dependency chains of one instruction
// (so latency is hidden by the chains and the waves), kUnroll steps per loop
// iteration; the probe reports how many of the probed instructions one wave
// issues, and the caller divides by the measured time.  The chains converge to
// finite fixed points, so no step sees an infinity or a denormal.
#include "gpair_internal.h"

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 8;

template <int KIND>
__global__ __launch_bounds__(256) void peak_kernel(int32_t iters, float *out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  float xf[kChains];
  double xd[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    xf[c] = 0.5f + 0.01f * (float)(c + (t & 7));
    xd[c] = 0.5 + 0.01 * (double)(c + (t & 7));
  }
  const float af = 0.999f, bf = 1e-4f;
  const double ad = 0.999, bd = 1e-4;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        if (KIND == 0) xf[c] = fmaf(xf[c], af, bf);                        // v_fma_f32
        if (KIND == 1) xd[c] = fma(xd[c], ad, bd);                         // v_fma_f64
        if (KIND == 2) xf[c] = __builtin_amdgcn_exp2f(-xf[c]);             // v_exp_f32
        if (KIND == 3) xf[c] = __builtin_amdgcn_rsqf(xf[c]);               // v_rsq_f32
        if (KIND == 4) xd[c] = __builtin_amdgcn_rsq(xd[c]);                // v_rsq_f64
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += xf[c] + (float)xd[c];
  out[t] = s;
}

}  // namespace

extern "C" gpair_status gpair_peak_probe(int32_t kind, int32_t blocks, int32_t iters, float *out,
                                         int64_t *per_wave, gpair_stream stream) {
  if (kind < 0 || kind > 4 || blocks <= 0 || iters <= 0 || !out || !per_wave)
    return GPAIR_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int64_t steps = (int64_t)iters * kUnroll * kChains;
  *per_wave = steps;
  switch (kind) {
    case 0: peak_kernel<0><<<blocks, 256, 0, s>>>(iters, out); break;
    case 1: peak_kernel<1><<<blocks, 256, 0, s>>>(iters, out); break;
    case 2: peak_kernel<2><<<blocks, 256, 0, s>>>(iters, out); break;
    case 3: peak_kernel<3><<<blocks, 256, 0, s>>>(iters, out); break;
    default: peak_kernel<4><<<blocks, 256, 0, s>>>(iters, out); break;
  }
  return hipGetLastError() == hipSuccess ? GPAIR_OK : GPAIR_ERR_HIP;
}
