// nn_api.cpp -- extern "C" entry points of the warm-start network kernels
// (declared in include/gpair_nn.h): shape validation on the host, then the
// launchers of nn_ops.hip on the caller's stream.
#include <cstdint>

#include "nn_internal.h"

using namespace gpair::nn;

namespace {

gpair_status hip_status(hipError_t e) { return e == hipSuccess ? GPAIR_OK : GPAIR_ERR_HIP; }

bool pow2(int32_t x) { return x >= 1 && ilog2(x) >= 0; }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// A view usable by the vectorised kernels: 8-channel groups are 16-byte aligned.
bool view_ok(const gpair_nn_tensor *t, bool vec = true) {
  if (!t || !t->data) return false;
  if (t->n < 1 || !pow2(t->d) || !pow2(t->h) || !pow2(t->w)) return false;
  if (t->c < 1 || t->cs < t->c) return false;
  if (vec && (!aligned16(t->data) || (t->cs % 8) != 0 || (t->c % 8) != 0)) return false;
  return true;
}

bool same_grid(const gpair_nn_tensor *a, const gpair_nn_tensor *b) {
  return a->n == b->n && a->d == b->d && a->h == b->h && a->w == b->w;
}

bool half_grid(const gpair_nn_tensor *coarse, const gpair_nn_tensor *fine) {
  return coarse->n == fine->n && 2 * coarse->d == fine->d && 2 * coarse->h == fine->h &&
         2 * coarse->w == fine->w;
}

Grid grid_of(const gpair_nn_tensor *t) {
  Grid g;
  g.ld = ilog2(t->d);
  g.lh = ilog2(t->h);
  g.lw = ilog2(t->w);
  g.nvox = (int64_t)t->n * t->d * t->h * t->w;
  return g;
}

bool chan_ok(int c) { return c == 16 || c == 32 || c == 64 || c == 128; }

hipStream_t hs(gpair_stream s) { return reinterpret_cast<hipStream_t>(s); }

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

gpair_status gpair_nn_conv3(const gpair_nn_tensor *in, const void *w, const float *bias,
                            const gpair_nn_tensor *out, int epilogue,
                            const gpair_nn_tensor *aux, gpair_stream stream) {
  if (!in || !out || !w || !aligned16(w)) return GPAIR_ERR_INVALID_ARG;
  const int cin = in->c, cout = out->c;
  if (!(cin == 1 || chan_ok(cin)) || !chan_ok(cout)) return GPAIR_ERR_INVALID_ARG;
  if (!view_ok(in, cin != 1) || !view_ok(out) || !same_grid(in, out)) return GPAIR_ERR_INVALID_ARG;
  if (epilogue < GPAIR_NN_EPI_BIAS_RELU || epilogue > GPAIR_NN_EPI_NONE)
    return GPAIR_ERR_INVALID_ARG;
  if ((epilogue == GPAIR_NN_EPI_BIAS_RELU || epilogue == GPAIR_NN_EPI_BIAS) && !bias)
    return GPAIR_ERR_INVALID_ARG;
  if (epilogue == GPAIR_NN_EPI_MASK &&
      (!view_ok(aux) || !same_grid(aux, out) || aux->c != cout))
    return GPAIR_ERR_INVALID_ARG;
  const Grid g = grid_of(out);
  if (cin == 1) {
    if (cout > 32 || epilogue == GPAIR_NN_EPI_MASK) return GPAIR_ERR_INVALID_ARG;
    return hip_status(launch_conv_c1(static_cast<const uint16_t *>(in->data), in->cs, g,
                                     static_cast<const uint16_t *>(w), bias,
                                     static_cast<uint16_t *>(out->data), out->cs, cout,
                                     epilogue, hs(stream)));
  }
  ConvArgs a{};
  a.in = static_cast<const uint16_t *>(in->data);
  a.in_cs = in->cs;
  a.g = g;
  a.w = static_cast<const uint16_t *>(w);
  a.bias = bias;
  a.out = static_cast<uint16_t *>(out->data);
  a.out_cs = out->cs;
  a.aux = epilogue == GPAIR_NN_EPI_MASK ? static_cast<const uint16_t *>(aux->data) : nullptr;
  a.aux_cs = epilogue == GPAIR_NN_EPI_MASK ? aux->cs : 0;
  a.cout = cout;
  a.epi = epilogue;
  return hip_status(launch_conv3(a, cin, kConv3, hs(stream)));
}

size_t gpair_nn_wgrad_partial_size(const gpair_nn_tensor *in, const gpair_nn_tensor *gout,
                                   int taps) {
  if (!in || !gout || (taps != 27 && taps != 8)) return 0;
  const gpair_nn_tensor *b = taps == 27 ? gout : in;
  if (b->n < 1 || !pow2(b->d) || !pow2(b->h) || !pow2(b->w) || in->c < 1 || gout->c < 1)
    return 0;
  return wgrad_scratch_bytes(taps == 27 ? kConv3 : kUpDgrad, grid_of(b), in->c, gout->c);
}

gpair_status gpair_nn_conv3_wgrad(const gpair_nn_tensor *in, const gpair_nn_tensor *gout,
                                  float *partial, float *dw, float *db,
                                  gpair_stream stream) {
  if (!in || !gout || !partial || !dw || !aligned16(partial)) return GPAIR_ERR_INVALID_ARG;
  const int cin = in->c, cout = gout->c;
  if (!(cin == 1 || chan_ok(cin)) || !chan_ok(cout)) return GPAIR_ERR_INVALID_ARG;
  if (cin == 1 && cout > 32) return GPAIR_ERR_INVALID_ARG;
  if (!view_ok(in, cin != 1) || !view_ok(gout) || !same_grid(in, gout))
    return GPAIR_ERR_INVALID_ARG;
  WgradJob j;
  j.mode = kConv3;
  j.x = static_cast<const uint16_t *>(in->data);
  j.x_cs = in->cs;
  j.g = static_cast<const uint16_t *>(gout->data);
  j.g_cs = gout->cs;
  j.base = grid_of(gout);
  j.cin = cin;
  j.cout = cout;
  return hip_status(launch_wgrad_job(j, partial, dw, db, hs(stream)));
}

gpair_status gpair_nn_maxpool2(const gpair_nn_tensor *in, const gpair_nn_tensor *out,
                               uint8_t *argmax, gpair_stream stream) {
  if (!view_ok(in) || !view_ok(out) || !argmax || ((uintptr_t)argmax & 7u))
    return GPAIR_ERR_INVALID_ARG;
  if (!chan_ok(in->c) || out->c != in->c || !half_grid(out, in)) return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_maxpool(static_cast<const uint16_t *>(in->data), in->cs,
                                   grid_of(out), in->c, static_cast<uint16_t *>(out->data),
                                   out->cs, argmax, hs(stream)));
}

gpair_status gpair_nn_maxpool2_backward(const gpair_nn_tensor *gout, const uint8_t *argmax,
                                        const gpair_nn_tensor *gskip,
                                        const gpair_nn_tensor *act,
                                        const gpair_nn_tensor *gin, gpair_stream stream) {
  if (!view_ok(gout) || !view_ok(act) || !view_ok(gin) || !argmax || ((uintptr_t)argmax & 7u))
    return GPAIR_ERR_INVALID_ARG;
  const int c = gout->c;
  if (!chan_ok(c) || act->c != c || gin->c != c) return GPAIR_ERR_INVALID_ARG;
  if (!half_grid(gout, act) || !same_grid(act, gin)) return GPAIR_ERR_INVALID_ARG;
  if (gskip && (!view_ok(gskip) || gskip->c != c || !same_grid(gskip, gin)))
    return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_maxpool_bwd(
      static_cast<const uint16_t *>(gout->data), gout->cs, argmax,
      gskip ? static_cast<const uint16_t *>(gskip->data) : nullptr, gskip ? gskip->cs : 0,
      static_cast<const uint16_t *>(act->data), act->cs, static_cast<uint16_t *>(gin->data),
      gin->cs, grid_of(gin), c, hs(stream)));
}

gpair_status gpair_nn_upconv2(const gpair_nn_tensor *in, const void *w, const float *bias,
                              const gpair_nn_tensor *out, gpair_stream stream) {
  if (!view_ok(in) || !view_ok(out) || !w || !aligned16(w) || !bias)
    return GPAIR_ERR_INVALID_ARG;
  const int cin = in->c, cout = out->c;
  if (!(cin == 32 || cin == 64 || cin == 128) || !(cout == 16 || cout == 32 || cout == 64))
    return GPAIR_ERR_INVALID_ARG;
  if (!half_grid(in, out)) return GPAIR_ERR_INVALID_ARG;
  UpArgs a{};
  a.in = static_cast<const uint16_t *>(in->data);
  a.in_cs = in->cs;
  a.g = grid_of(in);
  a.w = static_cast<const uint16_t *>(w);
  a.bias = bias;
  a.out = static_cast<uint16_t *>(out->data);
  a.out_cs = out->cs;
  a.cout = cout;
  return hip_status(launch_upconv(a, cin, hs(stream)));
}

gpair_status gpair_nn_upconv2_dgrad(const gpair_nn_tensor *gout, const void *wt,
                                    const gpair_nn_tensor *gin, const gpair_nn_tensor *aux,
                                    gpair_stream stream) {
  if (!view_ok(gout) || !view_ok(gin) || !wt || !aligned16(wt)) return GPAIR_ERR_INVALID_ARG;
  const int cup = gout->c, cin = gin->c;  // channels of the upconv output / input
  if (!(cup == 16 || cup == 32 || cup == 64) || !(cin == 32 || cin == 64 || cin == 128))
    return GPAIR_ERR_INVALID_ARG;
  if (!half_grid(gin, gout)) return GPAIR_ERR_INVALID_ARG;
  if (aux && (!view_ok(aux) || aux->c != cin || !same_grid(aux, gin)))
    return GPAIR_ERR_INVALID_ARG;
  ConvArgs a{};
  a.in = static_cast<const uint16_t *>(gout->data);
  a.in_cs = gout->cs;
  a.g = grid_of(gin);
  a.w = static_cast<const uint16_t *>(wt);
  a.bias = nullptr;
  a.out = static_cast<uint16_t *>(gin->data);
  a.out_cs = gin->cs;
  a.aux = aux ? static_cast<const uint16_t *>(aux->data) : nullptr;
  a.aux_cs = aux ? aux->cs : 0;
  a.cout = cin;
  a.epi = aux ? GPAIR_NN_EPI_MASK : GPAIR_NN_EPI_NONE;
  return hip_status(launch_conv3(a, cup, kUpDgrad, hs(stream)));
}

gpair_status gpair_nn_upconv2_wgrad(const gpair_nn_tensor *in, const gpair_nn_tensor *gout,
                                    float *partial, float *dw, float *db,
                                    gpair_stream stream) {
  if (!view_ok(in) || !view_ok(gout) || !partial || !dw || !aligned16(partial))
    return GPAIR_ERR_INVALID_ARG;
  const int cin = in->c, cout = gout->c;
  if (!(cin == 32 || cin == 64 || cin == 128) || !(cout == 16 || cout == 32 || cout == 64))
    return GPAIR_ERR_INVALID_ARG;
  if (!half_grid(in, gout)) return GPAIR_ERR_INVALID_ARG;
  WgradJob j;
  j.mode = kUpDgrad;
  j.x = static_cast<const uint16_t *>(in->data);
  j.x_cs = in->cs;
  j.g = static_cast<const uint16_t *>(gout->data);
  j.g_cs = gout->cs;
  j.base = grid_of(in);
  j.cin = cin;
  j.cout = cout;
  return hip_status(launch_wgrad_job(j, partial, dw, db, hs(stream)));
}

gpair_status gpair_nn_head(const gpair_nn_tensor *in, const float *w, const float *b,
                           float *out, gpair_stream stream) {
  if (!view_ok(in) || !(in->c == 16 || in->c == 32) || !w || !b || !out)
    return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_head(static_cast<const uint16_t *>(in->data), in->cs, in->c,
                                grid_of(in).nvox, w, b, out, hs(stream)));
}

size_t gpair_nn_head_partial_size(const gpair_nn_tensor *in) {
  if (!in || in->c < 1) return 0;
  return round256((size_t)kSumBlocks * (in->c + 1) * sizeof(float));
}

gpair_status gpair_nn_head_backward(const gpair_nn_tensor *in, const float *w,
                                    const float *out, const float *gout,
                                    const gpair_nn_tensor *gin, float *partial, float *dw,
                                    float *db, gpair_stream stream) {
  if (!view_ok(in) || !(in->c == 16 || in->c == 32) || !w || !out || !gout || !partial ||
      !dw || !db)
    return GPAIR_ERR_INVALID_ARG;
  if (!view_ok(gin) || gin->c != in->c || !same_grid(in, gin)) return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_head_bwd(static_cast<const uint16_t *>(in->data), in->cs, in->c,
                                    grid_of(in).nvox, w, out, gout,
                                    static_cast<uint16_t *>(gin->data), gin->cs, partial, dw,
                                    db, hs(stream)));
}

gpair_status gpair_nn_mse(int64_t n, const float *pred, const float *target, float *gpred,
                          double *loss, double *partial, gpair_stream stream) {
  if (n < 1 || !pred || !target || !loss || !partial) return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_mse(n, pred, target, gpred, loss, partial, hs(stream)));
}

gpair_status gpair_nn_pack_weights(const float *master, int taps, int c_in, int c_out,
                                   void *fwd, void *dgrad, gpair_stream stream) {
  if (!master || !fwd || (taps != 27 && taps != 8)) return GPAIR_ERR_INVALID_ARG;
  if (!(c_in == 1 || chan_ok(c_in)) || !chan_ok(c_out)) return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_pack(master, taps, c_in, c_out, static_cast<uint16_t *>(fwd),
                                static_cast<uint16_t *>(dgrad), hs(stream)));
}

gpair_status gpair_nn_from_float(const float *x, float scale, const gpair_nn_tensor *out,
                                 gpair_stream stream) {
  if (!x || !view_ok(out, false) || out->c != 1) return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_from_float(x, scale, static_cast<uint16_t *>(out->data), out->cs,
                                      grid_of(out).nvox, hs(stream)));
}

gpair_status gpair_nn_upsample2(const float *x, int32_t n, int32_t d, int32_t h, int32_t w,
                                float *out, gpair_stream stream) {
  if (!x || !out || n < 1 || d < 1 || h < 1 || w < 1) return GPAIR_ERR_INVALID_ARG;
  return hip_status(launch_upsample2(x, n, d, h, w, out, hs(stream)));
}

}  // extern "C"
