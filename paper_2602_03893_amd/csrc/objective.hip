// objective.hip -- gfx950 kernels of the paper's full objective around the
// operators (arXiv 2602.03893, Methods): the non-negativity parameterisation
// x = (z + eps)^2 and its chain rule ("Nonnegative parameterization
// constraint"), and the vessel continuity regulariser R_VCR = R_H + beta R_TV
// with its gradient ("Vessel continuity regularization").
//
// Discretisation (the paper gives none): a volume [nz][ny][nx], x fastest,
// unit spacing; D_d x_i = x[i+e_d] - x[i]; D_pp x_i = x[i+e_p] - 2 x[i] +
// x[i-e_p]; D_pq x_i = x[i+e_p+e_q] - x[i+e_p] - x[i+e_q] + x[i] (p != q, each
// mixed term twice in the Frobenius sum); a difference whose stencil leaves
// the volume is 0.
//
// The regulariser is two HBM-bound passes, one thread per voxel along x
// (coalesced; the neighbour reads hit L1/L2):
//  1. terms: the nine differences in float64 (from the float32 volume), the
//     norms n_T = sqrt(sum D_d^2 + eps) and n_H = sqrt(sum D_pp^2 + 2 sum D_pq^2
//     + eps), and the normalised terms dn/dD -- D_d / n_T, D_pp / n_H,
//     2 D_pq / n_H -- stored as nine float32 arrays; per-block float64 sums of
//     n_H + beta n_T (added in a fixed order by a second small kernel);
//  2. gradient: the transpose of every difference operator applied to its
//     normalised term, gathered per voxel; grad += lambda * (that sum).
#include <cmath>

#include "gpair_internal.h"

namespace gpair {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void npc_map_kernel(int64_t n, const float *__restrict__ z,
                                                         float eps, float *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    const float t = z[i] + eps;
    x[i] = t * t;
  }
}

// gz may alias gx.
__global__ __launch_bounds__(kBlock) void npc_grad_kernel(int64_t n, const float *__restrict__ z,
                                                          const float *gx, float eps, float *gz) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) gz[i] = gx[i] * 2.0f * (z[i] + eps);
}

struct VcrDims {
  int32_t nx, ny, nz;
  int64_t sy, sz, n;  // strides of y and z, voxel count
};

// The nine normalised terms, structure of arrays: tx ty tz (first), pxx pyy pzz
// (pure second), mxy mxz myz (mixed).
enum { kTx = 0, kTy, kTz, kPxx, kPyy, kPzz, kMxy, kMxz, kMyz, kTerms };

__global__ __launch_bounds__(kBlock) void vcr_terms_kernel(VcrDims g, const float *__restrict__ x,
                                                           double eps, double beta,
                                                           float *__restrict__ terms,
                                                           double *__restrict__ partial) {
  __shared__ double part[kBlock / kWave];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double v = 0.0;
  if (i < g.n) {
    const int ix = (int)(i % g.nx);
    const int iy = (int)((i / g.nx) % g.ny);
    const int iz = (int)(i / g.sz);
    const bool px = ix + 1 < g.nx, mx = ix > 0;
    const bool py = iy + 1 < g.ny, my = iy > 0;
    const bool pz = iz + 1 < g.nz, mz = iz > 0;
    const double c = x[i];
    const double xp = px ? (double)x[i + 1] : 0.0, xm = mx ? (double)x[i - 1] : 0.0;
    const double yp = py ? (double)x[i + g.sy] : 0.0, ym = my ? (double)x[i - g.sy] : 0.0;
    const double zp = pz ? (double)x[i + g.sz] : 0.0, zm = mz ? (double)x[i - g.sz] : 0.0;
    const double dx = px ? xp - c : 0.0, dy = py ? yp - c : 0.0, dz = pz ? zp - c : 0.0;
    const double dxx = (px && mx) ? xp - 2.0 * c + xm : 0.0;
    const double dyy = (py && my) ? yp - 2.0 * c + ym : 0.0;
    const double dzz = (pz && mz) ? zp - 2.0 * c + zm : 0.0;
    const double dxy = (px && py) ? (double)x[i + 1 + g.sy] - xp - yp + c : 0.0;
    const double dxz = (px && pz) ? (double)x[i + 1 + g.sz] - xp - zp + c : 0.0;
    const double dyz = (py && pz) ? (double)x[i + g.sy + g.sz] - yp - zp + c : 0.0;
    const double nt = sqrt(dx * dx + dy * dy + dz * dz + eps);
    const double nh = sqrt(dxx * dxx + dyy * dyy + dzz * dzz +
                           2.0 * (dxy * dxy + dxz * dxz + dyz * dyz) + eps);
    const double it = 1.0 / nt, ih = 1.0 / nh;
    float *t = terms + i;
    t[kTx * g.n] = (float)(dx * it);
    t[kTy * g.n] = (float)(dy * it);
    t[kTz * g.n] = (float)(dz * it);
    t[kPxx * g.n] = (float)(dxx * ih);
    t[kPyy * g.n] = (float)(dyy * ih);
    t[kPzz * g.n] = (float)(dzz * ih);
    t[kMxy * g.n] = (float)(2.0 * dxy * ih);
    t[kMxz * g.n] = (float)(2.0 * dxz * ih);
    t[kMyz * g.n] = (float)(2.0 * dyz * ih);
    v = nh + beta * nt;
  }
  if (partial) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
  }
}

// Fixed-order sum of the per-block partial sums (one workgroup).
__global__ __launch_bounds__(kBlock) void vcr_sum_kernel(const double *__restrict__ partial,
                                                         int64_t nb, double *__restrict__ out) {
  __shared__ double part[kBlock];
  double v = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kBlock) v += partial[b];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

__global__ __launch_bounds__(kBlock) void vcr_grad_kernel(VcrDims g,
                                                          const float *__restrict__ terms,
                                                          float beta, float lambda,
                                                          float *__restrict__ grad) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= g.n) return;
  const int ix = (int)(j % g.nx);
  const int iy = (int)((j / g.nx) % g.ny);
  const int iz = (int)(j / g.sz);
  const bool mx = ix > 0, my = iy > 0, mz = iz > 0;
  const bool px = ix + 1 < g.nx, py = iy + 1 < g.ny, pz = iz + 1 < g.nz;
  const int64_t n = g.n;
  auto T = [&](int k, int64_t idx) { return terms[k * n + idx]; };
  // first differences: transpose of x[i + e_d] - x[i]
  float gt = -(T(kTx, j) + T(kTy, j) + T(kTz, j));
  if (mx) gt += T(kTx, j - 1);
  if (my) gt += T(kTy, j - g.sy);
  if (mz) gt += T(kTz, j - g.sz);
  // pure second differences: the stencil is symmetric
  float gh = -2.0f * (T(kPxx, j) + T(kPyy, j) + T(kPzz, j));
  if (mx) gh += T(kPxx, j - 1);
  if (px) gh += T(kPxx, j + 1);
  if (my) gh += T(kPyy, j - g.sy);
  if (py) gh += T(kPyy, j + g.sy);
  if (mz) gh += T(kPzz, j - g.sz);
  if (pz) gh += T(kPzz, j + g.sz);
  // mixed: transpose of x[i+p+q] - x[i+p] - x[i+q] + x[i]
  gh += T(kMxy, j) + T(kMxz, j) + T(kMyz, j);
  if (mx) gh -= T(kMxy, j - 1) + T(kMxz, j - 1);
  if (my) gh -= T(kMxy, j - g.sy) + T(kMyz, j - g.sy);
  if (mz) gh -= T(kMxz, j - g.sz) + T(kMyz, j - g.sz);
  if (mx && my) gh += T(kMxy, j - 1 - g.sy);
  if (mx && mz) gh += T(kMxz, j - 1 - g.sz);
  if (my && mz) gh += T(kMyz, j - g.sy - g.sz);
  grad[j] += lambda * (gh + beta * gt);
}

inline unsigned int blocks_for(int64_t n) { return (unsigned int)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_npc_map(int64_t n, const float *z, float eps, float *x, hipStream_t s) {
  npc_map_kernel<<<blocks_for(n), kBlock, 0, s>>>(n, z, eps, x);
  return hipGetLastError();
}

hipError_t launch_npc_grad(int64_t n, const float *z, const float *gx, float eps, float *gz,
                           hipStream_t s) {
  npc_grad_kernel<<<blocks_for(n), kBlock, 0, s>>>(n, z, gx, eps, gz);
  return hipGetLastError();
}

size_t vcr_work_bytes(int32_t nx, int32_t ny, int32_t nz) {
  const int64_t n = (int64_t)nx * ny * nz;
  const size_t terms = ((size_t)kTerms * n * sizeof(float) + 255) & ~size_t(255);
  return terms + (size_t)blocks_for(n) * sizeof(double);
}

hipError_t launch_vcr(int32_t nx, int32_t ny, int32_t nz, const float *x, double beta,
                      double eps, double lambda, float *grad, double *value, void *work,
                      hipStream_t s) {
  VcrDims g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.sy = nx;
  g.sz = (int64_t)nx * ny;
  g.n = g.sz * nz;
  const size_t tb = ((size_t)kTerms * g.n * sizeof(float) + 255) & ~size_t(255);
  float *terms = (float *)work;
  double *partial = value ? (double *)((char *)work + tb) : nullptr;
  const unsigned int nb = blocks_for(g.n);
  vcr_terms_kernel<<<nb, kBlock, 0, s>>>(g, x, eps, beta, terms, partial);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && value) {
    vcr_sum_kernel<<<1, kBlock, 0, s>>>(partial, nb, value);
    e = hipGetLastError();
  }
  if (e == hipSuccess && grad) {
    vcr_grad_kernel<<<nb, kBlock, 0, s>>>(g, terms, (float)beta, (float)lambda, grad);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace gpair
