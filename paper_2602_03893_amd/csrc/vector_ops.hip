// vector_ops.hip -- element-wise and reduction kernels of the reconstruction
// loop (arXiv 2602.03893, Algorithm 2: loss, trace gradient y - b, parameter
// update).  All HBM-bound: coalesced grid-stride loops, float64 partial sums
// reduced in a fixed order so the norms are bitwise reproducible.
#include "gpair_internal.h"

namespace gpair {
namespace {

constexpr int kVecBlock = 256;

unsigned int vec_grid(int64_t n) {
  int64_t g = (n + kVecBlock - 1) / kVecBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned int)g;
}

__global__ __launch_bounds__(kVecBlock) void fill_kernel(float *__restrict__ x, int64_t n,
                                                         float value) {
  const int64_t stride = (int64_t)gridDim.x * kVecBlock;
  for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += stride)
    x[i] = value;
}

// Block-wide float64 sum of two values in a fixed tree order.
__device__ __forceinline__ void block_sum2(double &a, double &b, double *sh) {
  const int t = threadIdx.x;
  sh[t] = a;
  sh[kVecBlock + t] = b;
  __syncthreads();
  for (int w = kVecBlock / 2; w > 0; w >>= 1) {
    if (t < w) {
      sh[t] += sh[t + w];
      sh[kVecBlock + t] += sh[kVecBlock + t + w];
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[kVecBlock];
}

__global__ __launch_bounds__(kVecBlock) void residual_partial_kernel(
    const float *y, const float *__restrict__ b, float scale, float *delta, int64_t n,
    double *__restrict__ partials) {
  __shared__ double sh[2 * kVecBlock];
  double s_rr = 0.0, s_bb = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kVecBlock;
  for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += stride) {
    const float yi = y[i], bi = b[i];
    const double rd = (double)yi - (double)bi;  // exact difference for the norm
    s_rr += rd * rd;
    s_bb += (double)bi * (double)bi;
    if (delta) delta[i] = scale * (yi - bi);
  }
  block_sum2(s_rr, s_bb, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s_rr;
    partials[2 * blockIdx.x + 1] = s_bb;
  }
}

__global__ __launch_bounds__(kVecBlock) void residual_final_kernel(
    const double *__restrict__ partials, int nparts, double *__restrict__ norms) {
  __shared__ double sh[2 * kVecBlock];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kVecBlock) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  block_sum2(a, b, sh);
  if (threadIdx.x == 0) {
    norms[0] = a;
    norms[1] = b;
  }
}

__global__ __launch_bounds__(kVecBlock) void scale_kernel(float *__restrict__ x, int64_t n,
                                                          float alpha) {
  const int64_t stride = (int64_t)gridDim.x * kVecBlock;
  for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += stride)
    x[i] = alpha * x[i];
}

// Block-wide float64 sum of three values in a fixed tree order.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *sh) {
  const int t = threadIdx.x;
  sh[t] = a;
  sh[kVecBlock + t] = b;
  sh[2 * kVecBlock + t] = c;
  __syncthreads();
  for (int w = kVecBlock / 2; w > 0; w >>= 1) {
    if (t < w) {
      sh[t] += sh[t + w];
      sh[kVecBlock + t] += sh[kVecBlock + t + w];
      sh[2 * kVecBlock + t] += sh[2 * kVecBlock + t + w];
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[kVecBlock];
  c = sh[2 * kVecBlock];
}

__global__ __launch_bounds__(kVecBlock) void dot3_partial_kernel(const float *__restrict__ y,
                                                                 const float *__restrict__ b,
                                                                 int64_t n,
                                                                 double *__restrict__ partials) {
  __shared__ double sh[3 * kVecBlock];
  double yb = 0.0, yy = 0.0, bb = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kVecBlock;
  for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += stride) {
    const double yi = y[i], bi = b[i];
    yb += yi * bi;
    yy += yi * yi;
    bb += bi * bi;
  }
  block_sum3(yb, yy, bb, sh);
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x] = yb;
    partials[3 * blockIdx.x + 1] = yy;
    partials[3 * blockIdx.x + 2] = bb;
  }
}

__global__ __launch_bounds__(kVecBlock) void dot3_final_kernel(const double *__restrict__ partials,
                                                               int nparts,
                                                               double *__restrict__ out) {
  __shared__ double sh[3 * kVecBlock];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kVecBlock) {
    a += partials[3 * i];
    b += partials[3 * i + 1];
    c += partials[3 * i + 2];
  }
  block_sum3(a, b, c, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
    out[2] = c;
  }
}

__global__ __launch_bounds__(kVecBlock) void pgd_kernel(float *__restrict__ x,
                                                        const float *__restrict__ g,
                                                        int64_t n, float step, float lo,
                                                        float hi) {
  const int64_t stride = (int64_t)gridDim.x * kVecBlock;
  for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += stride) {
    const float v = fmaf(-step, g[i], x[i]);
    x[i] = fminf(hi, fmaxf(lo, v));
  }
}

__global__ __launch_bounds__(kVecBlock) void adam_kernel(
    float *__restrict__ x, const float *__restrict__ g, float *__restrict__ m,
    float *__restrict__ v, int64_t n, float grad_scale, float lr, float beta1, float beta2,
    float eps, float inv_bc1, float inv_sqrt_bc2, float lo, float hi) {
  const int64_t stride = (int64_t)gridDim.x * kVecBlock;
  for (int64_t i = (int64_t)blockIdx.x * kVecBlock + threadIdx.x; i < n; i += stride) {
    const float gi = grad_scale * g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = (mi * inv_bc1) / (sqrtf(vi) * inv_sqrt_bc2 + eps);
    const float xi = x[i] - lr * upd;
    x[i] = fminf(hi, fmaxf(lo, xi));
  }
}

}  // namespace

hipError_t launch_fill(float *x, int64_t n, float value, hipStream_t s) {
  fill_kernel<<<vec_grid(n), kVecBlock, 0, s>>>(x, n, value);
  return hipGetLastError();
}

hipError_t launch_residual(const gpair_plan_s *p, const float *y, const float *b,
                           float scale, float *delta, double *norms, hipStream_t s) {
  const int64_t n = (int64_t)p->Nd * p->Nt;
  double *partials = ws_partials(p);
  residual_partial_kernel<<<kResidualBlocks, kVecBlock, 0, s>>>(y, b, scale, delta, n,
                                                               partials);
  residual_final_kernel<<<1, kVecBlock, 0, s>>>(partials, kResidualBlocks, norms);
  return hipGetLastError();
}

hipError_t launch_scale(float *x, int64_t n, float alpha, hipStream_t s) {
  scale_kernel<<<vec_grid(n), kVecBlock, 0, s>>>(x, n, alpha);
  return hipGetLastError();
}

hipError_t launch_dot3(const gpair_plan_s *p, const float *y, const float *b, double *out,
                       hipStream_t s) {
  const int64_t n = (int64_t)p->Nd * p->Nt;
  double *partials = ws_partials(p);
  dot3_partial_kernel<<<kResidualBlocks, kVecBlock, 0, s>>>(y, b, n, partials);
  dot3_final_kernel<<<1, kVecBlock, 0, s>>>(partials, kResidualBlocks, out);
  return hipGetLastError();
}

hipError_t launch_pgd(int64_t n, float *x, const float *g, float step, float lo, float hi,
                      hipStream_t s) {
  pgd_kernel<<<vec_grid(n), kVecBlock, 0, s>>>(x, g, n, step, lo, hi);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float *x, const float *g, float *m, float *v,
                       float grad_scale, float lr, float beta1, float beta2, float eps,
                       int32_t t, float lo, float hi, hipStream_t s) {
  const double bc1 = 1.0 - std::pow((double)beta1, (double)t);
  const double bc2 = 1.0 - std::pow((double)beta2, (double)t);
  adam_kernel<<<vec_grid(n), kVecBlock, 0, s>>>(x, g, m, v, n, grad_scale, lr, beta1, beta2,
                                                eps, (float)(1.0 / bc1),
                                                (float)(1.0 / std::sqrt(bc2)), lo, hi);
  return hipGetLastError();
}

}  // namespace gpair
