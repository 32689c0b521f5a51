/*
 * gpair_nn.h -- C ABI of the 3D convolution kernels of the learned warm start.
 *
 * The warm start maps the back-projected (adjoint) image of a reconstruction
 * problem to non-negative amplitudes with a small 3D encoder-decoder
 * (U-Net): 3x3x3 convolutions with ReLU, 2x2x2 max pooling, stride-2 2x2x2
 * transposed convolutions and skip concatenation, and a 1x1x1 head with ReLU.
 * It is this build's addition, not part of arXiv 2602.03893 (the paper's
 * Discussion names learned priors inside reconstruction pipelines as future
 * work); the adjoint image it consumes is the paper's adjoint operator
 * (Methods, "Adjoint Operator" subsection).
 *
 * Conventions
 *  - Activations are bfloat16, channels-last (N, D, H, W, C), with a channel
 *    stride cs >= C between consecutive voxels, so a tensor can be a channel
 *    slice of a wider one (this is how skip concatenation is zero-copy).
 *    D, H and W must be powers of two.  Accumulation is float32 (MFMA).
 *  - 3x3x3 weights (forward layout) are bfloat16 [27][C_out][C_in], tap
 *    t = (dz+1)*9 + (dy+1)*3 + (dx+1); transposed-convolution weights are
 *    bfloat16 [8][C_out][C_in], tap t = (z%2)*4 + (y%2)*2 + (x%2) of the
 *    output voxel.  Master weights are float32 [taps][C_in][C_out] (the
 *    layout gpair_nn_pack_weights reads).
 *  - Supported channel counts: 3x3x3 convolution C_in in {1, 16, 32, 64,
 *    128} and C_out in {16, 32, 64, 128} (C_in = 1: C_out in {16, 32}, no
 *    MASK epilogue); transposed convolution C_in in {32, 64, 128}, C_out in
 *    {16, 32, 64}; max pooling C in {16, 32, 64, 128}; head C in {16, 32}.
 *  - Views with C > 1 need a 16-byte aligned data pointer and a channel
 *    stride that is a multiple of 8 (8 channels are one 16-byte access).
 *  - An output must not overlap an input of the same call, except where a
 *    call says so.
 *  - All pointers are device memory owned by the caller; work goes on
 *    `stream`; shapes are validated on the host (GPAIR_ERR_INVALID_ARG,
 *    nothing launched).  Launch failures return GPAIR_ERR_HIP.
 */
#ifndef GPAIR_NN_H
#define GPAIR_NN_H

#include <stddef.h>
#include <stdint.h>

#include "gpair.h"

#ifdef __cplusplus
extern "C" {
#endif

/* A channels-last bfloat16 (or float32 where stated) tensor view. */
typedef struct gpair_nn_tensor {
  void *data;   /* first element of channel 0 of voxel 0             */
  int32_t n, d, h, w;
  int32_t c;    /* channels of this view                             */
  int32_t cs;   /* elements between consecutive voxels (>= c)        */
} gpair_nn_tensor;

#define GPAIR_NN_EPI_BIAS_RELU 0  /* out = max(0, acc + bias)                 */
#define GPAIR_NN_EPI_BIAS 1       /* out = acc + bias                         */
#define GPAIR_NN_EPI_MASK 2       /* out = acc * (aux > 0)   (ReLU backward)  */
#define GPAIR_NN_EPI_NONE 3       /* out = acc                                */

/*
 * 3x3x3 convolution, stride 1, zero padding 1, as an implicit GEMM on
 * v_mfma_f32_16x16x32_bf16:  out[v][co] = epi( sum_{t,ci} in[v + o(t)][ci]
 * * w[t][co][ci] ).  With the weights of gpair_nn_pack_weights' data-gradient
 * layout (taps flipped, C_in and C_out exchanged) and GPAIR_NN_EPI_MASK this
 * is the convolution's input gradient fused with the ReLU backward of the
 * layer that produced the input.  bias: float32 [C_out] (read for the BIAS
 * epilogues, else may be NULL); aux: bfloat16 view of out's shape (MASK).
 */
gpair_status gpair_nn_conv3(const gpair_nn_tensor *in, const void *w, const float *bias,
                            const gpair_nn_tensor *out, int epilogue,
                            const gpair_nn_tensor *aux, gpair_stream stream);

/*
 * Weight gradient of the 3x3x3 convolution: dw[t][ci][co] (float32, master
 * layout, overwritten) = sum_v gout[v][co] * in[v + o(t)][ci]; db[co] =
 * sum_v gout[v][co] (float32, overwritten; NULL to skip).  Sums run over
 * voxel chunks into `partial` (float32, gpair_nn_wgrad_partial_size bytes)
 * and are then reduced in a fixed order.
 */
size_t gpair_nn_wgrad_partial_size(const gpair_nn_tensor *in, const gpair_nn_tensor *gout,
                                   int taps);
gpair_status gpair_nn_conv3_wgrad(const gpair_nn_tensor *in, const gpair_nn_tensor *gout,
                                  float *partial, float *dw, float *db,
                                  gpair_stream stream);

/* 2x2x2 max pooling, stride 2: out (half size) and the argmax code (uint8,
 * [voxels_out][C], the tap of the maximum; ties take the first). */
gpair_status gpair_nn_maxpool2(const gpair_nn_tensor *in, const gpair_nn_tensor *out,
                               uint8_t *argmax, gpair_stream stream);

/*
 * Backward of max pooling merged with a skip-connection gradient and the
 * ReLU backward of the pooled activation:
 *   gin[u][c] = ( gskip[u][c] + [argmax of u's window is u] gout[u/2][c] )
 *               * (act[u][c] > 0)
 * gskip may be NULL (no skip branch).  gin may alias gskip.
 */
gpair_status gpair_nn_maxpool2_backward(const gpair_nn_tensor *gout, const uint8_t *argmax,
                                        const gpair_nn_tensor *gskip,
                                        const gpair_nn_tensor *act,
                                        const gpair_nn_tensor *gin, gpair_stream stream);

/*
 * 2x2x2 transposed convolution, stride 2 (upsampling):
 *   out[2v + t][co] = sum_ci in[v][ci] * w[t][co][ci] + bias[co].
 * Data gradient (with the transposed weights [8][C_in][C_out] of
 * gpair_nn_pack_weights): gin[v][ci] = mask * sum_{t,co} gout[2v+t][co] w[t][co][ci],
 * mask = (aux[v][ci] > 0) when aux is given (ReLU backward), else 1.
 */
gpair_status gpair_nn_upconv2(const gpair_nn_tensor *in, const void *w, const float *bias,
                              const gpair_nn_tensor *out, gpair_stream stream);
gpair_status gpair_nn_upconv2_dgrad(const gpair_nn_tensor *gout, const void *wt,
                                    const gpair_nn_tensor *gin, const gpair_nn_tensor *aux,
                                    gpair_stream stream);
/* dw[t][ci][co] = sum_v gout[2v+t][co] in[v][ci]; db as for conv3_wgrad. */
gpair_status gpair_nn_upconv2_wgrad(const gpair_nn_tensor *in, const gpair_nn_tensor *gout,
                                    float *partial, float *dw, float *db,
                                    gpair_stream stream);

/*
 * 1x1x1 head with ReLU: out[v] = max(0, sum_c in[v][c] w[c] + b) (float32
 * [voxels]).  Backward: gpre = gout * (out > 0); gin[v][c] = gpre w[c] *
 * (in[v][c] > 0); dw[c] = sum_v gpre in[v][c]; db = sum_v gpre (dw, db
 * float32 [C] and [1], summed in a fixed order through `partial`, float32
 * [gpair_nn_head_partial_size bytes]).
 */
gpair_status gpair_nn_head(const gpair_nn_tensor *in, const float *w, const float *b,
                           float *out, gpair_stream stream);
size_t gpair_nn_head_partial_size(const gpair_nn_tensor *in);
gpair_status gpair_nn_head_backward(const gpair_nn_tensor *in, const float *w,
                                    const float *out, const float *gout,
                                    const gpair_nn_tensor *gin, float *partial, float *dw,
                                    float *db, gpair_stream stream);

/*
 * Mean squared error L = mean((pred - target)^2) over n values: loss (float64
 * [1], device) and, when gpred is not NULL, gpred = 2 (pred - target) / n
 * (float32).  partial: float64 [GPAIR_NN_MSE_PARTIALS] scratch; the sum is
 * taken in a fixed order (bitwise reproducible).
 */
#define GPAIR_NN_MSE_PARTIALS 1024
gpair_status gpair_nn_mse(int64_t n, const float *pred, const float *target, float *gpred,
                          double *loss, double *partial, gpair_stream stream);

/*
 * Convert master weights (float32 [taps][C_in][C_out]) to the compute copies:
 * fwd (bfloat16 [taps][C_out][C_in]) and, when dgrad is not NULL, the
 * data-gradient copy (bfloat16 [taps][C_in][C_out], taps flipped for 3x3x3,
 * taps kept for the 2x2x2 transposed convolution).  taps is 27 or 8.
 */
gpair_status gpair_nn_pack_weights(const float *master, int taps, int c_in, int c_out,
                                   void *fwd, void *dgrad, gpair_stream stream);

/* out (bfloat16 view, C = 1) = scale * x (float32 [voxels]). */
gpair_status gpair_nn_from_float(const float *x, float scale, const gpair_nn_tensor *out,
                                 gpair_stream stream);

/* Trilinear x2 upsampling of a float32 volume [n][d][h][w] to [n][2d][2h][2w]
 * (half-voxel aligned, edge clamped). */
gpair_status gpair_nn_upsample2(const float *x, int32_t n, int32_t d, int32_t h, int32_t w,
                                float *out, gpair_stream stream);

/* ------------------------------------------------------------------------ */
/* The warm-start U-Net executor                                              */
/* ------------------------------------------------------------------------ */
/*
 * A U-Net with `levels` in 1..4 and base width 16 (level l has 16 * 2^l
 * channels).  Encoder level l < levels-1: two 3x3x3 conv + ReLU layers, then
 * 2x2x2 max pooling; bottom level: two conv + ReLU layers; decoder level l:
 * a stride-2 2x2x2 transposed conv (bias, no activation) whose output is
 * concatenated with the encoder output of level l as [upsampled, skip], then
 * two conv + ReLU layers; a 1x1x1 head with ReLU gives one output channel.
 *
 * Parameters are one float32 vector.  Layers are stored in the order
 * enc0a, enc0b, ..., enc{L-2}b, bot_a, bot_b, up{L-2}, dec{L-2}a, dec{L-2}b,
 * ..., up0, dec0a, dec0b, head; each layer stores its weights (3x3x3:
 * [27][C_in][C_out]; transposed: [8][C_in][C_out]; head: [C]) followed by its
 * bias ([C_out]; head: [1]).  Gradients use the same layout.
 *
 * Volumes are float32 [n][d][h][w]; d, h, w must be powers of two divisible
 * by 2^(levels-1).  The workspace (device, caller-owned, 256-byte aligned)
 * holds the bfloat16 weight copies, every activation the backward needs, the
 * gradients of the activations and the reduction scratch; a backward call
 * reads the activations of the last forward call made on the same workspace
 * with the same parameters and shape.
 */
#define GPAIR_UNET_MAX_LEVELS 4

/* Number of float32 parameters (0 for unsupported levels). */
int64_t gpair_unet_param_count(int levels);

/* Seeded initialisation into host memory (float32 [param_count]): weights
 * N(0, 2 / fan_in) (fan_in = taps * C_in), biases 0.  The normal deviates
 * come from a counter-based generator (SplitMix64 of seed and index, then
 * Box-Muller), so the result does not depend on the platform. */
gpair_status gpair_unet_init_params(int levels, uint64_t seed, float *params_host);

/* Workspace bytes for a batch of n volumes of d x h x w (0 if invalid). */
size_t gpair_unet_workspace_size(int levels, int32_t n, int32_t d, int32_t h, int32_t w);

/* y = net(x_scale * x).  x and y: float32 [n][d][h][w] (device). */
gpair_status gpair_unet_forward(int levels, const float *params, int32_t n, int32_t d,
                                int32_t h, int32_t w, const float *x, float x_scale,
                                float *y, void *workspace, size_t workspace_bytes,
                                gpair_stream stream);

/* grad (float32 [param_count], overwritten) = d(sum gy . y)/d(params) for the
 * last forward on this workspace; gy: float32 [n][d][h][w]. */
gpair_status gpair_unet_backward(int levels, const float *params, int32_t n, int32_t d,
                                 int32_t h, int32_t w, const float *gy, float *grad,
                                 void *workspace, size_t workspace_bytes,
                                 gpair_stream stream);

/*
 * One training step on a batch: forward, MSE loss against target (float32
 * [n][d][h][w]), backward, and one Adam step (beta1, beta2, eps as given; step
 * number t >= 1; no projection) on params with moments m, v (float32
 * [param_count], zero before the first step).  loss: float64 [1] (device),
 * the loss before the update; grad: float32 [param_count] scratch.
 */
gpair_status gpair_unet_train_step(int levels, float *params, float *grad, float *m, float *v,
                                   int32_t t, float lr, float beta1, float beta2, float eps,
                                   int32_t n, int32_t d, int32_t h, int32_t w, const float *x,
                                   float x_scale, const float *target, double *loss,
                                   void *workspace, size_t workspace_bytes,
                                   gpair_stream stream);

/* ------------------------------------------------------------------------ */
/* a8. The learned warm start                                                */
/* ------------------------------------------------------------------------ */
/*
 * Learned start for traces b, on a full-resolution plan whose kernels are a
 * (2d) x (2h) x (2w) grid and a half-resolution plan whose kernels are a
 * d x h x w grid (both in grid order, x fastest, the same sensors and
 * samples):
 *   1. g = A_half^T b                    (gpair_adjoint on the half plan)
 *   2. x_half = net(inv_kappa * g)       (gpair_unet_forward, one volume)
 *   3. x = trilinear x2 upsampling of x_half
 *   4. gpair_warm_rescale on the full plan: A_out = c* x, or 0 (fallback).
 * params: U-Net parameters (device); A_out: device float32 [8 d h w];
 * workspace: device, 256-byte aligned, gpair_warm_start_workspace_size bytes.
 * Synchronises `stream` (step 4).  Errors: INVALID_ARG, WORKSPACE,
 * NONFINITE, HIP.
 */
size_t gpair_warm_start_workspace_size(int levels, int32_t d, int32_t h, int32_t w,
                                       int64_t n_trace_samples);
gpair_status gpair_warm_start(gpair_plan full, const float *sigma_full, gpair_plan half,
                              const float *sigma_half, int levels, const float *params,
                              int32_t d, int32_t h, int32_t w, float inv_kappa,
                              const float *b, float *A_out, void *workspace,
                              size_t workspace_bytes, gpair_warm_report *report,
                              gpair_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* GPAIR_NN_H */
