// unet.cpp -- the warm-start U-Net executor (declared in include/gpair_nn.h):
// workspace layout, weight packing, and the forward / backward / training
// sequences of the network, every layer a call of the kernel ABI in
// nn_api.cpp.  No allocation: the caller provides every device buffer.
#include <cmath>
#include <cstring>
#include <vector>

#include "gpair_internal.h"
#include "nn_internal.h"

namespace {

using gpair::nn::ilog2;

enum Kind { kConvLayer, kUpLayer, kHeadLayer };

struct Layer {
  int kind, taps, cin, cout;
  int64_t off_w, off_b;   // float offsets in the parameter vector
  size_t pk_fwd, pk_dg;   // byte offsets of the bfloat16 copies in the workspace
};

int chan(int l) { return 16 << l; }

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// Layer table and workspace layout of one (levels, n, d, h, w).
struct Net {
  int L = 0, n = 0, d = 0, h = 0, w = 0;
  std::vector<Layer> layers;
  int enc_a[4], enc_b[4], up[4], dec_a[4], dec_b[4], bot_a = -1, bot_b = -1, head = -1;
  int64_t nparam = 0;
  // workspace byte offsets
  size_t x_in = 0, y = 0, gpred = 0;
  size_t a[4], cat[4], p[4], am[4], da[4], db[4];
  size_t bota = 0, botb = 0;
  size_t g_a[4], g_cat[4], g_p[4], g_da[4], g_db[4], g_bota = 0, g_botb = 0;
  size_t wg = 0, wg_bytes = 0, headp = 0, msep = 0;
  size_t total = 0;

  int64_t vox(int l) const { return (int64_t)n * (d >> l) * (h >> l) * (w >> l); }

  int add(int kind, int taps, int cin, int cout) {
    Layer ly;
    ly.kind = kind;
    ly.taps = taps;
    ly.cin = cin;
    ly.cout = cout;
    ly.off_w = nparam;
    nparam += (int64_t)taps * cin * cout;
    ly.off_b = nparam;
    nparam += cout;
    ly.pk_fwd = ly.pk_dg = 0;
    layers.push_back(ly);
    return (int)layers.size() - 1;
  }

  void build_layers(int levels) {
    L = levels;
    layers.clear();
    nparam = 0;
    int cin = 1;
    for (int l = 0; l < L - 1; ++l) {
      enc_a[l] = add(kConvLayer, 27, cin, chan(l));
      enc_b[l] = add(kConvLayer, 27, chan(l), chan(l));
      cin = chan(l);
    }
    bot_a = add(kConvLayer, 27, cin, chan(L - 1));
    bot_b = add(kConvLayer, 27, chan(L - 1), chan(L - 1));
    for (int l = L - 2; l >= 0; --l) {
      up[l] = add(kUpLayer, 8, chan(l + 1), chan(l));
      dec_a[l] = add(kConvLayer, 27, 2 * chan(l), chan(l));
      dec_b[l] = add(kConvLayer, 27, chan(l), chan(l));
    }
    head = add(kHeadLayer, 1, chan(0), 1);
  }

  gpair_nn_tensor tv(void *base, size_t off, int level, int c, int cs, int c0 = 0) const {
    gpair_nn_tensor t;
    t.data = static_cast<char *>(base) + off + 2 * (size_t)c0;
    t.n = n;
    t.d = d >> level;
    t.h = h >> level;
    t.w = w >> level;
    t.c = c;
    t.cs = cs;
    return t;
  }

  // Lays out the workspace; returns false for an unsupported shape.
  bool build(int levels, int32_t n_, int32_t d_, int32_t h_, int32_t w_) {
    if (levels < 1 || levels > GPAIR_UNET_MAX_LEVELS || n_ < 1) return false;
    if (ilog2(d_) < levels - 1 || ilog2(h_) < levels - 1 || ilog2(w_) < levels - 1) return false;
    n = n_;
    d = d_;
    h = h_;
    w = w_;
    build_layers(levels);
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off += al(bytes);
      return o;
    };
    auto act = [&](int l, int c) { return take((size_t)vox(l) * c * 2); };
    for (Layer &ly : layers) {
      if (ly.kind == kHeadLayer) continue;
      const size_t b = (size_t)ly.taps * ly.cin * ly.cout * 2;
      ly.pk_fwd = take(b);
      ly.pk_dg = take(b);
    }
    x_in = act(0, 1);
    y = take((size_t)vox(0) * 4);
    gpred = take((size_t)vox(0) * 4);
    for (int l = 0; l < L - 1; ++l) {
      a[l] = act(l, chan(l));
      cat[l] = act(l, 2 * chan(l));
      p[l] = act(l + 1, chan(l));
      am[l] = take((size_t)vox(l + 1) * chan(l));
      da[l] = act(l, chan(l));
      db[l] = act(l, chan(l));
      g_a[l] = act(l, chan(l));
      g_cat[l] = act(l, 2 * chan(l));
      g_p[l] = act(l + 1, chan(l));
      g_da[l] = act(l, chan(l));
      g_db[l] = act(l, chan(l));
    }
    bota = act(L - 1, chan(L - 1));
    botb = act(L - 1, chan(L - 1));
    g_bota = act(L - 1, chan(L - 1));
    g_botb = act(L - 1, chan(L - 1));
    // weight-gradient scratch: the largest any layer needs
    wg_bytes = 0;
    char dummy[16];
    for (const Layer &ly : layers) {
      if (ly.kind == kHeadLayer) continue;
      size_t b;
      if (ly.kind == kConvLayer) {
        const int lvl = level_of(ly);
        gpair_nn_tensor ti = tv(dummy, 0, lvl, ly.cin, ly.cin), tg = tv(dummy, 0, lvl, ly.cout, ly.cout);
        b = gpair_nn_wgrad_partial_size(&ti, &tg, 27);
      } else {
        const int lvl = level_of(ly);  // fine level of the output
        gpair_nn_tensor ti = tv(dummy, 0, lvl + 1, ly.cin, ly.cin),
                        tg = tv(dummy, 0, lvl, ly.cout, ly.cout);
        b = gpair_nn_wgrad_partial_size(&ti, &tg, 8);
      }
      if (b == 0) return false;
      if (b > wg_bytes) wg_bytes = b;
    }
    wg = take(wg_bytes);
    {
      gpair_nn_tensor th = tv(dummy, 0, 0, chan(0), chan(0));
      headp = take(gpair_nn_head_partial_size(&th));
    }
    msep = take(sizeof(double) * GPAIR_NN_MSE_PARTIALS);
    total = off;
    return true;
  }

  // Grid level of a layer's output (for the transposed conv: its fine output).
  int level_of(const Layer &ly) const {
    const int idx = (int)(&ly - layers.data());
    for (int l = 0; l < L - 1; ++l) {
      if (idx == enc_a[l] || idx == enc_b[l] || idx == up[l] || idx == dec_a[l] ||
          idx == dec_b[l])
        return l;
    }
    return idx == head ? 0 : L - 1;
  }
};

#define TRY(expr)                            \
  do {                                       \
    const gpair_status st_ = (expr);         \
    if (st_ != GPAIR_OK) return st_;         \
  } while (0)

gpair_status pack_all(const Net &net, const float *params, void *ws, gpair_stream s) {
  char *base = static_cast<char *>(ws);
  for (const Layer &ly : net.layers) {
    if (ly.kind == kHeadLayer) continue;
    TRY(gpair_nn_pack_weights(params + ly.off_w, ly.taps, ly.cin, ly.cout, base + ly.pk_fwd,
                              base + ly.pk_dg, s));
  }
  return GPAIR_OK;
}

// Forward into the workspace's prediction buffer.
gpair_status forward_ws(const Net &net, const float *params, const float *x, float scale,
                        void *ws, gpair_stream s) {
  char *base = static_cast<char *>(ws);
  const auto &Ly = net.layers;
  TRY(pack_all(net, params, ws, s));
  const int L = net.L;
  gpair_nn_tensor xin = net.tv(ws, net.x_in, 0, 1, 1);
  TRY(gpair_nn_from_float(x, scale, &xin, s));
  gpair_nn_tensor in = xin;
  for (int l = 0; l < L - 1; ++l) {
    const int C = chan(l);
    const Layer &ea = Ly[net.enc_a[l]], &eb = Ly[net.enc_b[l]];
    gpair_nn_tensor a = net.tv(ws, net.a[l], l, C, C);
    gpair_nn_tensor e = net.tv(ws, net.cat[l], l, C, 2 * C, C);
    gpair_nn_tensor p = net.tv(ws, net.p[l], l + 1, C, C);
    TRY(gpair_nn_conv3(&in, base + ea.pk_fwd, params + ea.off_b, &a, GPAIR_NN_EPI_BIAS_RELU,
                       nullptr, s));
    TRY(gpair_nn_conv3(&a, base + eb.pk_fwd, params + eb.off_b, &e, GPAIR_NN_EPI_BIAS_RELU,
                       nullptr, s));
    TRY(gpair_nn_maxpool2(&e, &p, reinterpret_cast<uint8_t *>(base + net.am[l]), s));
    in = p;
  }
  const int CB = chan(L - 1);
  gpair_nn_tensor ba = net.tv(ws, net.bota, L - 1, CB, CB);
  gpair_nn_tensor bb = net.tv(ws, net.botb, L - 1, CB, CB);
  TRY(gpair_nn_conv3(&in, base + Ly[net.bot_a].pk_fwd, params + Ly[net.bot_a].off_b, &ba,
                     GPAIR_NN_EPI_BIAS_RELU, nullptr, s));
  TRY(gpair_nn_conv3(&ba, base + Ly[net.bot_b].pk_fwd, params + Ly[net.bot_b].off_b, &bb,
                     GPAIR_NN_EPI_BIAS_RELU, nullptr, s));
  gpair_nn_tensor hcur = bb;
  for (int l = L - 2; l >= 0; --l) {
    const int C = chan(l);
    const Layer &u = Ly[net.up[l]], &a1 = Ly[net.dec_a[l]], &b1 = Ly[net.dec_b[l]];
    gpair_nn_tensor upo = net.tv(ws, net.cat[l], l, C, 2 * C, 0);
    gpair_nn_tensor cat = net.tv(ws, net.cat[l], l, 2 * C, 2 * C);
    gpair_nn_tensor da = net.tv(ws, net.da[l], l, C, C);
    gpair_nn_tensor db = net.tv(ws, net.db[l], l, C, C);
    TRY(gpair_nn_upconv2(&hcur, base + u.pk_fwd, params + u.off_b, &upo, s));
    TRY(gpair_nn_conv3(&cat, base + a1.pk_fwd, params + a1.off_b, &da, GPAIR_NN_EPI_BIAS_RELU,
                       nullptr, s));
    TRY(gpair_nn_conv3(&da, base + b1.pk_fwd, params + b1.off_b, &db, GPAIR_NN_EPI_BIAS_RELU,
                       nullptr, s));
    hcur = db;
  }
  const Layer &hd = Ly[net.head];
  return gpair_nn_head(&hcur, params + hd.off_w, params + hd.off_b,
                       reinterpret_cast<float *>(base + net.y), s);
}

gpair_status backward_ws(const Net &net, const float *params, const float *gy, float *grad,
                         void *ws, gpair_stream s) {
  char *base = static_cast<char *>(ws);
  float *wg = reinterpret_cast<float *>(base + net.wg);
  const auto &Ly = net.layers;
  const int L = net.L;
  const int C0 = chan(0), CB = chan(L - 1);
  // head
  gpair_nn_tensor hlast = L >= 2 ? net.tv(ws, net.db[0], 0, C0, C0)
                                 : net.tv(ws, net.botb, 0, C0, C0);
  gpair_nn_tensor glast = L >= 2 ? net.tv(ws, net.g_db[0], 0, C0, C0)
                                 : net.tv(ws, net.g_botb, 0, C0, C0);
  const Layer &hd = Ly[net.head];
  TRY(gpair_nn_head_backward(&hlast, params + hd.off_w, reinterpret_cast<const float *>(base + net.y),
                             gy, &glast, reinterpret_cast<float *>(base + net.headp),
                             grad + hd.off_w, grad + hd.off_b, s));
  // decoder, top level first
  for (int l = 0; l < L - 1; ++l) {
    const int C = chan(l);
    const Layer &a1 = Ly[net.dec_a[l]], &b1 = Ly[net.dec_b[l]], &u = Ly[net.up[l]];
    gpair_nn_tensor da = net.tv(ws, net.da[l], l, C, C);
    gpair_nn_tensor gdb = net.tv(ws, net.g_db[l], l, C, C);
    gpair_nn_tensor gda = net.tv(ws, net.g_da[l], l, C, C);
    gpair_nn_tensor cat = net.tv(ws, net.cat[l], l, 2 * C, 2 * C);
    gpair_nn_tensor gcat = net.tv(ws, net.g_cat[l], l, 2 * C, 2 * C);
    gpair_nn_tensor gup = net.tv(ws, net.g_cat[l], l, C, 2 * C, 0);
    TRY(gpair_nn_conv3_wgrad(&da, &gdb, wg, grad + b1.off_w, grad + b1.off_b, s));
    TRY(gpair_nn_conv3(&gdb, base + b1.pk_dg, nullptr, &gda, GPAIR_NN_EPI_MASK, &da, s));
    TRY(gpair_nn_conv3_wgrad(&cat, &gda, wg, grad + a1.off_w, grad + a1.off_b, s));
    TRY(gpair_nn_conv3(&gda, base + a1.pk_dg, nullptr, &gcat, GPAIR_NN_EPI_NONE, nullptr, s));
    const int Cn = chan(l + 1);
    gpair_nn_tensor hin = l + 1 <= L - 2 ? net.tv(ws, net.db[l + 1], l + 1, Cn, Cn)
                                         : net.tv(ws, net.botb, l + 1, Cn, Cn);
    gpair_nn_tensor ghin = l + 1 <= L - 2 ? net.tv(ws, net.g_db[l + 1], l + 1, Cn, Cn)
                                          : net.tv(ws, net.g_botb, l + 1, Cn, Cn);
    TRY(gpair_nn_upconv2_wgrad(&hin, &gup, wg, grad + u.off_w, grad + u.off_b, s));
    TRY(gpair_nn_upconv2_dgrad(&gup, base + u.pk_dg, &ghin, &hin, s));
  }
  // bottom
  {
    const Layer &ba_l = Ly[net.bot_a], &bb_l = Ly[net.bot_b];
    gpair_nn_tensor ba = net.tv(ws, net.bota, L - 1, CB, CB);
    gpair_nn_tensor gbb = net.tv(ws, net.g_botb, L - 1, CB, CB);
    gpair_nn_tensor gba = net.tv(ws, net.g_bota, L - 1, CB, CB);
    TRY(gpair_nn_conv3_wgrad(&ba, &gbb, wg, grad + bb_l.off_w, grad + bb_l.off_b, s));
    TRY(gpair_nn_conv3(&gbb, base + bb_l.pk_dg, nullptr, &gba, GPAIR_NN_EPI_MASK, &ba, s));
    gpair_nn_tensor in_b = L >= 2 ? net.tv(ws, net.p[L - 2], L - 1, chan(L - 2), chan(L - 2))
                                  : net.tv(ws, net.x_in, 0, 1, 1);
    TRY(gpair_nn_conv3_wgrad(&in_b, &gba, wg, grad + ba_l.off_w, grad + ba_l.off_b, s));
    if (L >= 2) {
      gpair_nn_tensor gp = net.tv(ws, net.g_p[L - 2], L - 1, chan(L - 2), chan(L - 2));
      TRY(gpair_nn_conv3(&gba, base + ba_l.pk_dg, nullptr, &gp, GPAIR_NN_EPI_NONE, nullptr, s));
    }
  }
  // encoder, bottom level first
  for (int l = L - 2; l >= 0; --l) {
    const int C = chan(l);
    const Layer &ea = Ly[net.enc_a[l]], &eb = Ly[net.enc_b[l]];
    gpair_nn_tensor e = net.tv(ws, net.cat[l], l, C, 2 * C, C);
    gpair_nn_tensor ge = net.tv(ws, net.g_cat[l], l, C, 2 * C, C);
    gpair_nn_tensor gp = net.tv(ws, net.g_p[l], l + 1, C, C);
    gpair_nn_tensor a = net.tv(ws, net.a[l], l, C, C);
    gpair_nn_tensor ga = net.tv(ws, net.g_a[l], l, C, C);
    TRY(gpair_nn_maxpool2_backward(&gp, reinterpret_cast<const uint8_t *>(base + net.am[l]), &ge,
                                   &e, &ge, s));
    TRY(gpair_nn_conv3_wgrad(&a, &ge, wg, grad + eb.off_w, grad + eb.off_b, s));
    TRY(gpair_nn_conv3(&ge, base + eb.pk_dg, nullptr, &ga, GPAIR_NN_EPI_MASK, &a, s));
    gpair_nn_tensor in_l = l == 0 ? net.tv(ws, net.x_in, 0, 1, 1)
                                  : net.tv(ws, net.p[l - 1], l, chan(l - 1), chan(l - 1));
    TRY(gpair_nn_conv3_wgrad(&in_l, &ga, wg, grad + ea.off_w, grad + ea.off_b, s));
    if (l > 0) {
      gpair_nn_tensor gpp = net.tv(ws, net.g_p[l - 1], l, chan(l - 1), chan(l - 1));
      TRY(gpair_nn_conv3(&ga, base + ea.pk_dg, nullptr, &gpp, GPAIR_NN_EPI_NONE, nullptr, s));
    }
  }
  return GPAIR_OK;
}

uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double unit_open(uint64_t r) { return ((double)(r >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

bool ws_ok(const Net &net, const void *ws, size_t bytes) {
  return ws && ((uintptr_t)ws & 255u) == 0 && bytes >= net.total;
}

}  // namespace

extern "C" {

int64_t gpair_unet_param_count(int levels) {
  if (levels < 1 || levels > GPAIR_UNET_MAX_LEVELS) return 0;
  Net net;
  net.build_layers(levels);
  return net.nparam;
}

gpair_status gpair_unet_init_params(int levels, uint64_t seed, float *params_host) {
  if (levels < 1 || levels > GPAIR_UNET_MAX_LEVELS || !params_host) return GPAIR_ERR_INVALID_ARG;
  Net net;
  net.build_layers(levels);
  const double two_pi = 6.283185307179586476925286766559;
  for (const Layer &ly : net.layers) {
    const int64_t nw = (int64_t)ly.taps * ly.cin * ly.cout;
    const double stdv = std::sqrt(2.0 / (double)(ly.taps * ly.cin));
    for (int64_t i = 0; i < nw; ++i) {
      const uint64_t k = (uint64_t)(ly.off_w + i);
      const double u1 = unit_open(splitmix64(seed ^ splitmix64(2 * k)));
      const double u2 = unit_open(splitmix64(seed ^ splitmix64(2 * k + 1)));
      const double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(two_pi * u2);
      params_host[ly.off_w + i] = (float)(stdv * z);
    }
    for (int c = 0; c < ly.cout; ++c) params_host[ly.off_b + c] = 0.0f;
  }
  return GPAIR_OK;
}

size_t gpair_unet_workspace_size(int levels, int32_t n, int32_t d, int32_t h, int32_t w) {
  Net net;
  if (!net.build(levels, n, d, h, w)) return 0;
  return net.total;
}

gpair_status gpair_unet_forward(int levels, const float *params, int32_t n, int32_t d,
                                int32_t h, int32_t w, const float *x, float x_scale,
                                float *y, void *workspace, size_t workspace_bytes,
                                gpair_stream stream) {
  Net net;
  if (!net.build(levels, n, d, h, w) || !params || !x || !y) return GPAIR_ERR_INVALID_ARG;
  if (!ws_ok(net, workspace, workspace_bytes)) return GPAIR_ERR_WORKSPACE;
  TRY(forward_ws(net, params, x, x_scale, workspace, stream));
  const hipError_t e =
      hipMemcpyAsync(y, static_cast<char *>(workspace) + net.y, sizeof(float) * net.vox(0),
                     hipMemcpyDeviceToDevice, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? GPAIR_OK : GPAIR_ERR_HIP;
}

gpair_status gpair_unet_backward(int levels, const float *params, int32_t n, int32_t d,
                                 int32_t h, int32_t w, const float *gy, float *grad,
                                 void *workspace, size_t workspace_bytes,
                                 gpair_stream stream) {
  Net net;
  if (!net.build(levels, n, d, h, w) || !params || !gy || !grad) return GPAIR_ERR_INVALID_ARG;
  if (!ws_ok(net, workspace, workspace_bytes)) return GPAIR_ERR_WORKSPACE;
  return backward_ws(net, params, gy, grad, workspace, stream);
}

gpair_status gpair_unet_train_step(int levels, float *params, float *grad, float *m, float *v,
                                   int32_t t, float lr, float beta1, float beta2, float eps,
                                   int32_t n, int32_t d, int32_t h, int32_t w, const float *x,
                                   float x_scale, const float *target, double *loss,
                                   void *workspace, size_t workspace_bytes,
                                   gpair_stream stream) {
  Net net;
  if (!net.build(levels, n, d, h, w) || !params || !grad || !m || !v || !x || !target || !loss)
    return GPAIR_ERR_INVALID_ARG;
  if (t < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return GPAIR_ERR_INVALID_ARG;
  if (!ws_ok(net, workspace, workspace_bytes)) return GPAIR_ERR_WORKSPACE;
  char *base = static_cast<char *>(workspace);
  TRY(forward_ws(net, params, x, x_scale, workspace, stream));
  float *pred = reinterpret_cast<float *>(base + net.y);
  float *gpred = reinterpret_cast<float *>(base + net.gpred);
  TRY(gpair_nn_mse(net.vox(0), pred, target, gpred, loss,
                   reinterpret_cast<double *>(base + net.msep), stream));
  TRY(backward_ws(net, params, gpred, grad, workspace, stream));
  const hipError_t e = gpair::launch_adam(net.nparam, params, grad, m, v, 1.0f, lr, beta1, beta2,
                                          eps, t, -INFINITY, INFINITY,
                                          reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? GPAIR_OK : GPAIR_ERR_HIP;
}

size_t gpair_warm_start_workspace_size(int levels, int32_t d, int32_t h, int32_t w,
                                       int64_t n_trace_samples) {
  const size_t u = gpair_unet_workspace_size(levels, 1, d, h, w);
  if (u == 0 || n_trace_samples < 1) return 0;
  const size_t mh = (size_t)d * h * w;
  return al(u) + 2 * al(mh * sizeof(float)) + al((size_t)n_trace_samples * sizeof(float));
}

gpair_status gpair_warm_start(gpair_plan full, const float *sigma_full, gpair_plan half,
                              const float *sigma_half, int levels, const float *params,
                              int32_t d, int32_t h, int32_t w, float inv_kappa,
                              const float *b, float *A_out, void *workspace,
                              size_t workspace_bytes, gpair_warm_report *report,
                              gpair_stream stream) {
  if (!full || !half || !sigma_full || !sigma_half || !params || !b || !A_out || !report)
    return GPAIR_ERR_INVALID_ARG;
  if (!std::isfinite(inv_kappa) || !(inv_kappa > 0.0f)) return GPAIR_ERR_INVALID_ARG;
  gpair_plan_info fi, hi;
  TRY(gpair_plan_get_info(full, &fi));
  TRY(gpair_plan_get_info(half, &hi));
  const int64_t mh = (int64_t)d * h * w;
  if (d < 1 || h < 1 || w < 1 || hi.n_kernels != mh || fi.n_kernels != 8 * mh ||
      fi.n_sensors != hi.n_sensors || fi.n_samples != hi.n_samples)
    return GPAIR_ERR_INVALID_ARG;
  const int64_t nt = (int64_t)fi.n_sensors * fi.n_samples;
  const size_t need = gpair_warm_start_workspace_size(levels, d, h, w, nt);
  if (need == 0) return GPAIR_ERR_INVALID_ARG;
  if (!workspace || ((uintptr_t)workspace & 255u) || workspace_bytes < need)
    return GPAIR_ERR_WORKSPACE;
  char *base = static_cast<char *>(workspace);
  const size_t u = al(gpair_unet_workspace_size(levels, 1, d, h, w));
  float *g = reinterpret_cast<float *>(base + u);
  float *xh = reinterpret_cast<float *>(base + u + al(mh * sizeof(float)));
  float *y = reinterpret_cast<float *>(base + u + 2 * al(mh * sizeof(float)));
  TRY(gpair_adjoint(half, nullptr, sigma_half, b, g, nullptr, stream));
  TRY(gpair_unet_forward(levels, params, 1, d, h, w, g, inv_kappa, xh, workspace, u, stream));
  TRY(gpair_nn_upsample2(xh, 1, d, h, w, A_out, stream));
  return gpair_warm_rescale(full, A_out, sigma_full, b, y, report, stream);
}

}  // extern "C"
