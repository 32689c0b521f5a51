// assa_static.hip -- the ASSA back-projection for callers that cannot
// allocate device memory (code under graph capture, serving loops, hosts that
// forbid hipMalloc): gpair_assa_adjoint_static.
//
// gpair_assa_adjoint takes a caller buffer for the convolved residual
// (float32 [n_sensors][alpha n_samples]).  This variant keeps that buffer in
// a file-scope device array of fixed size instead, and launches the same two
// kernels.  Each GPU the library runs on holds its own copy of the array
// (kScratchBytes) from the first call on that GPU until the process ends.
//
// In host code `scratch` names a host-side stand-in, not a device address:
// the device address is looked up once per device with hipGetSymbolAddress
// (that device current) and only that pointer is handed to kernels.
#include <mutex>

#include "gpair_internal.h"

using namespace gpair;

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB: 16,777,216 floats

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, or null

// The device address of `scratch` on the current device (looked up on the
// first call on that device).
gpair_status scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GPAIR_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return GPAIR_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GPAIR_OK;
}

}  // namespace

extern "C" {

size_t gpair_assa_static_scratch_bytes(void) { return kScratchBytes; }

gpair_status gpair_assa_adjoint_static(gpair_plan p, double sigma, const float *delta, float *g,
                                       gpair_stream stream) {
  if (!p || !p->ws || !delta || !g) return GPAIR_ERR_INVALID_ARG;
  AssaGrid grid;
  const gpair_status st = assa_grid(p, sigma, &grid);
  if (st != GPAIR_OK) return st;
  if (assa_work_bytes(p, grid) > kScratchBytes) return GPAIR_ERR_WORKSPACE;
  void *work = nullptr;
  const gpair_status sa = scratch_address(&work);
  if (sa != GPAIR_OK) return sa;
  hipStream_t s = (hipStream_t)stream;
  // The correlation writes every element of [n_sensors][alpha n_samples]
  // before the back-projection reads it: nothing needs clearing.
  hipError_t e = launch_assa_dconv(p, grid, delta, (float *)work, s);
  if (e == hipSuccess) e = launch_assa_adjoint(p, grid, (const float *)work, g, s);
  return e == hipSuccess ? GPAIR_OK : GPAIR_ERR_HIP;
}

}  // extern "C"
