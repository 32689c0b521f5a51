// nn_internal.h -- kernel argument blocks and launchers of the learned
// warm-start network (3D U-Net on bfloat16 channels-last volumes).  The C
// entry points in nn_api.cpp validate shapes and call the launchers here.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gpair_nn.h"

namespace gpair {
namespace nn {

// Conv kernels: 4 waves per block, each wave 64 output voxels.
constexpr int kConvBlock = 256;
constexpr int kVoxPerWave = 64;
constexpr int kVoxPerBlock = 256;
// Weight-gradient kernels: chunk of 64 base-grid voxels staged in LDS.
constexpr int kChunk = 64;
constexpr int kLdsRow = kChunk + 8;  // padded row (bank spread), elements
constexpr int kWgradBlocks = 1024;   // target blocks per launch
constexpr size_t kWgradPartialCap = size_t(64) << 20;  // bytes of split partials
constexpr int kSumBlocks = 512;      // blocks of the channel-sum / head reductions

enum Mode { kConv3 = 0, kUpDgrad = 1 };

// log2 of a power of two, or -1.
inline int ilog2(int64_t x) {
  if (x <= 0 || (x & (x - 1))) return -1;
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

struct Grid {
  int ld, lh, lw;   // log2 of D, H, W
  int64_t nvox;     // N * D * H * W
};

struct ConvArgs {
  const uint16_t *in;
  int64_t in_cs;
  Grid g;               // output grid (coarse grid in kUpDgrad mode)
  const uint16_t *w;    // [taps][cout][cin]
  const float *bias;
  uint16_t *out;
  int64_t out_cs;
  const uint16_t *aux;
  int64_t aux_cs;
  int cout, epi, ngroups;
  int64_t ntiles;
};

struct UpArgs {
  const uint16_t *in;
  int64_t in_cs;
  Grid g;               // coarse (input) grid
  const uint16_t *w;    // [8][cout][cin]
  const float *bias;
  uint16_t *out;        // fine grid
  int64_t out_cs;
  int cout, ngroups;
  int64_t ntiles;
};

struct WgradArgs {
  const uint16_t *t_src;  // tap-indexed operand (conv3: input; transposed conv: gout)
  int64_t t_cs;
  const uint16_t *f_src;  // fixed operand (conv3: gout; transposed conv: input)
  int64_t f_cs;
  Grid g;                 // base grid (transposed conv: the coarse grid)
  float *partial;         // [nsplit][taps][cin][cout]
  int nsplit;
  int64_t nchunks;
};

// Split count of a weight-gradient launch (shared by the size query and the launch).
int wgrad_splits(int64_t nvox, int taps, int cin, int cout);

// A weight gradient (and optional bias gradient) of a 3x3x3 conv (mode kConv3:
// x is the conv input, g the output gradient, both on `base`) or of the
// stride-2 transposed conv (mode kUpDgrad: x on the coarse grid `base`, g on
// the fine grid).
struct WgradJob {
  int mode;
  const uint16_t *x;
  int64_t x_cs;
  const uint16_t *g;
  int64_t g_cs;
  Grid base;
  int cin, cout;
};
size_t wgrad_scratch_bytes(int mode, const Grid &base, int cin, int cout);
hipError_t launch_wgrad_job(const WgradJob &j, void *scratch, float *dw, float *db,
                            hipStream_t s);

hipError_t launch_conv3(const ConvArgs &a, int cin, int mode, hipStream_t s);
hipError_t launch_conv_c1(const uint16_t *in, int64_t in_cs, const Grid &g, const uint16_t *w,
                          const float *bias, uint16_t *out, int64_t out_cs, int cout, int epi,
                          hipStream_t s);
hipError_t launch_upconv(const UpArgs &a, int cin, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs &a, int mode, int cin, int cout, float *dw,
                        hipStream_t s);
hipError_t launch_wgrad_c1(const uint16_t *in, int64_t in_cs, const uint16_t *gout,
                           int64_t gout_cs, const Grid &g, int cout, float *partial,
                           int nsplit, float *dw, hipStream_t s);
hipError_t launch_chansum(const uint16_t *x, int64_t cs, int c, int64_t nvox, float *partial,
                          float *out, hipStream_t s);
hipError_t launch_maxpool(const uint16_t *in, int64_t in_cs, const Grid &coarse, int c,
                          uint16_t *out, int64_t out_cs, uint8_t *argmax, hipStream_t s);
hipError_t launch_maxpool_bwd(const uint16_t *gout, int64_t gout_cs, const uint8_t *argmax,
                              const uint16_t *gskip, int64_t gskip_cs, const uint16_t *act,
                              int64_t act_cs, uint16_t *gin, int64_t gin_cs,
                              const Grid &fine, int c, hipStream_t s);
hipError_t launch_head(const uint16_t *in, int64_t cs, int c, int64_t nvox, const float *w,
                       const float *b, float *out, hipStream_t s);
hipError_t launch_head_bwd(const uint16_t *in, int64_t cs, int c, int64_t nvox,
                           const float *w, const float *out, const float *gout,
                           uint16_t *gin, int64_t gin_cs, float *partial, float *dw,
                           float *db, hipStream_t s);
hipError_t launch_mse(int64_t n, const float *pred, const float *target, float *gpred,
                      double *loss, double *partial, hipStream_t s);
hipError_t launch_pack(const float *master, int taps, int cin, int cout, uint16_t *fwd,
                       uint16_t *dgrad, hipStream_t s);
hipError_t launch_from_float(const float *x, float scale, uint16_t *out, int64_t cs,
                             int64_t nvox, hipStream_t s);
hipError_t launch_upsample2(const float *x, int n, int d, int h, int w, float *out,
                            hipStream_t s);

}  // namespace nn
}  // namespace gpair
