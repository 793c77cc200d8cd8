// C ABI of the convolutional warm-start network (U-Net): parameters, forward
// and backward passes, one training step (mean squared loss, Adam), and the
// warm start of the scattering series built from an operator's state.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"

namespace lsop {
// kernels_nn.hip
hipError_t launch_conv_fwd(int ks, const float* X, int C, const unsigned short* Wb, int N, const float* bias, float* Y,
                           int B, int H, int W, bool relu, hipStream_t s);
hipError_t launch_conv_wgrad(int ks, const float* X, int C, const float* dY, int N, float* dW, int B, int H, int W,
                             hipStream_t s);
hipError_t launch_colsum(const float* dY, int P, int N, float* db, hipStream_t s);
hipError_t launch_relu_bwd(float* g, const float* y, size_t n, hipStream_t s);
hipError_t launch_scale_copy(float* out, const float* z, size_t n, int stride, float scale, hipStream_t s);
hipError_t launch_avgpool2(const float* x, float* y, int B, int h, int w, int C, hipStream_t s);
hipError_t launch_avgpool2_bwd(const float* dy, const float* add, float* dx, int B, int h, int w, int C,
                               hipStream_t s);
hipError_t launch_upcat(const float* lo, const float* skip, float* out, int B, int h, int w, int Cu, int Cs,
                        hipStream_t s);
hipError_t launch_upcat_bwd(const float* dcat, float* dlo, float* dskip, int B, int h, int w, int Cu, int Cs,
                            hipStream_t s);
hipError_t launch_mse(const float* out, const float* t, float* dout, size_t n, double* loss, hipStream_t s);
hipError_t launch_adam(float* P, const float* G, float* M, float* V, size_t n, float lr, double b1, double b2,
                       double eps, int step, hipStream_t s);
hipError_t launch_weights_bf16(const float* Wf, int ks, int Ci, int Co, unsigned short* Wb, unsigned short* WT,
                               hipStream_t s);
template <typename T>
hipError_t launch_pack_inputs(const double* chi, const Cx<T>* psi0, const double* norm2, float* out, int nvec,
                              size_t n, double c0w2, float k0h, float* scale, hipStream_t s);
template <typename T>
hipError_t launch_unpack_output(const Cx<T>* psi0, const float* y, const float* scale, Cx<T>* psi, int nvec, size_t n,
                                hipStream_t s);
template <typename T>
hipError_t launch_pack_target(const Cx<T>* psi, const Cx<T>* psi0, const float* scale, float* t, int nvec, size_t n,
                              hipStream_t s);
}  // namespace lsop

using namespace lsop;

struct unet {
  int levels = 0, base = 0, cin = 0, cout = 0, maxB = 0, maxH = 0, maxW = 0;
  struct Layer {
    int ks = 3, ci = 0, co = 0;
    size_t poff = 0;  // weights at P + poff ([ks^2 ci][co]), bias after them
    unsigned short *wb = nullptr, *wt = nullptr;
  };
  std::vector<Layer> layers;  // e0a, e0b, ..., e(L-1)b, d(L-2)a, ..., d0b, head
  size_t nparams = 0;
  float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
  int step = 0;
  std::vector<float*> ea, eb, pool, cat, da, db, skipg;
  float *ga = nullptr, *gb = nullptr;
  float *xin = nullptr, *yout = nullptr, *dout = nullptr, *scale = nullptr;
  double *dloss = nullptr, *norms = nullptr;
  const float* x_last = nullptr;
  int B = 0, H = 0, W = 0;
  bool have_fwd = false;
  std::vector<void*> owned;
  size_t bytes = 0;

  int ch(int l) const { return base << l; }
  Layer& enc(int l, int part) { return layers[2 * l + part]; }
  Layer& dec(int l, int part) { return layers[2 * levels + 2 * (levels - 2 - l) + part]; }
  Layer& head() { return layers.back(); }
};

namespace {

hipStream_t SS(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <typename P>
int nn_alloc(unet* u, P** out, size_t bytes) {
  void* p = nullptr;
  if (lib_malloc(&p, bytes ? bytes : 16) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LSOP_ENOMEM, "network allocation of " + std::to_string(bytes) + " bytes failed");
  }
  u->owned.push_back(p);
  u->bytes += bytes;
  *out = reinterpret_cast<P*>(p);
  return LSOP_OK;
}

int refresh_weights(unet* u, hipStream_t s) {
  for (auto& L : u->layers) {
    const double kn = (double)L.ks * L.ks * L.ci * L.co;
    LSOP_HIP(prof_launch("unet weights bf16", "k_weights_bf16", kn * 8.0, 0.0, 1, s,
                         [&] { return launch_weights_bf16(u->P + L.poff, L.ks, L.ci, L.co, L.wb, L.wt, s); }));
  }
  return LSOP_OK;
}

// Y = act(conv(X) + bias) with the weights Wb (forward) or WT (data gradient); algorithmic traffic is the input,
// the bf16 weights and the output once each; 2 P K N flops
int conv_launch(const char* use, int ks, const float* X, int ci, const unsigned short* w, int co, const float* bias,
                float* Y, int B, int H, int W, bool relu, hipStream_t s) {
  const double P = (double)B * H * W, K = (double)ks * ks * ci;
  // the launcher takes the vector kernel when channels come in eights and both operands are 16-byte aligned
  const bool vec = ci % 8 == 0 && ((uintptr_t)X % 16) == 0 && ((uintptr_t)w % 16) == 0;
  const char* fn = vec ? (ks == 3 ? "k_conv_fwd_v<3>" : "k_conv_fwd_v<1>") : (ks == 3 ? "k_conv_fwd<3>" : "k_conv_fwd<1>");
  LSOP_HIP(prof_launch(use, fn, P * ci * 4.0 + K * co * 2.0 + P * co * 4.0, 2.0 * P * K * co, P, s,
                       [&] { return launch_conv_fwd(ks, X, ci, w, co, bias, Y, B, H, W, relu, s); }));
  return LSOP_OK;
}

int conv(unet* u, const unet::Layer& L, const float* X, float* Y, bool relu, int B, int H, int W, hipStream_t s) {
  return conv_launch("unet conv forward", L.ks, X, L.ci, L.wb, L.co,
                     u->P + L.poff + (size_t)L.ks * L.ks * L.ci * L.co, Y, B, H, W, relu, s);
}

int forward(unet* u, const float* x, int B, int H, int W, float* y, hipStream_t s) {
  const int Lv = u->levels;
  const float* in = x;
  for (int l = 0; l < Lv; ++l) {
    const int h = H >> l, w = W >> l;
    int st = conv(u, u->enc(l, 0), in, u->ea[l], true, B, h, w, s);
    if (!st) st = conv(u, u->enc(l, 1), u->ea[l], u->eb[l], true, B, h, w, s);
    if (st) return st;
    if (l < Lv - 1) {
      const double e = (double)B * h * w * u->ch(l);
      LSOP_HIP(prof_launch("unet pool", "k_avgpool2", e * 5.0, e, e, s,
                           [&] { return launch_avgpool2(u->eb[l], u->pool[l], B, h / 2, w / 2, u->ch(l), s); }));
      in = u->pool[l];
    }
  }
  const float* prev = u->eb[Lv - 1];
  for (int l = Lv - 2; l >= 0; --l) {
    const int h = H >> l, w = W >> l;
    const double e = (double)B * h * w * (u->ch(l + 1) + u->ch(l));
    LSOP_HIP(prof_launch("unet upsample+concat", "k_upcat", e * 4.0 + (double)B * h * w * (u->ch(l + 1) / 4.0 + u->ch(l)) * 4.0,
                         0.0, e, s,
                         [&] { return launch_upcat(prev, u->eb[l], u->cat[l], B, h / 2, w / 2, u->ch(l + 1), u->ch(l), s); }));
    int st = conv(u, u->dec(l, 0), u->cat[l], u->da[l], true, B, h, w, s);
    if (!st) st = conv(u, u->dec(l, 1), u->da[l], u->db[l], true, B, h, w, s);
    if (st) return st;
    prev = u->db[l];
  }
  int st = conv(u, u->head(), prev, y, false, B, H, W, s);
  if (st) return st;
  u->x_last = x;
  u->B = B;
  u->H = H;
  u->W = W;
  u->have_fwd = true;
  return LSOP_OK;
}

// gradient of one layer: dY (post-activation gradient, masked in place when relu), X its input, Yout its output;
// writes the weight / bias gradients and, when dX != NULL, the input gradient.
int layer_back(unet* u, const unet::Layer& L, float* dY, const float* X, const float* Yout, float* dX, int B, int H,
               int W, hipStream_t s) {
  const double P = (double)B * H * W, K = (double)L.ks * L.ks * L.ci;
  if (Yout)
    LSOP_HIP(prof_launch("unet relu backward", "k_relu_bwd", P * L.co * 12.0, P * L.co, P * L.co, s,
                         [&] { return launch_relu_bwd(dY, Yout, (size_t)B * H * W * L.co, s); }));
  float* gw = u->G + L.poff;
  const bool vec = L.ci % 8 == 0 && L.co % 8 == 0 && ((uintptr_t)X % 16) == 0 && ((uintptr_t)dY % 16) == 0;
  const char* wfn = vec ? (L.ks == 3 ? "k_conv_wgrad_v<3>" : "k_conv_wgrad_v<1>")
                        : (L.ks == 3 ? "k_conv_wgrad<3>" : "k_conv_wgrad<1>");
  LSOP_HIP(prof_launch("unet weight gradient", wfn,
                       P * L.ci * 4.0 + P * L.co * 4.0 + K * L.co * 4.0, 2.0 * P * K * L.co, P, s,
                       [&] { return launch_conv_wgrad(L.ks, X, L.ci, dY, L.co, gw, B, H, W, s); }));
  LSOP_HIP(prof_launch("unet bias gradient", L.co <= 256 ? "k_colsum_flat" : "k_colsum", P * L.co * 4.0, P * L.co, P, s,
                       [&] { return launch_colsum(dY, B * H * W, L.co, gw + (size_t)K * L.co, s); }));
  if (dX) return conv_launch("unet data gradient", L.ks, dY, L.co, L.wt, L.ci, nullptr, dX, B, H, W, false, s);
  return LSOP_OK;
}

int backward(unet* u, const float* dy, hipStream_t s) {
  const int Lv = u->levels, B = u->B, H = u->H, W = u->W;
  LSOP_HIP(hipMemsetAsync(u->G, 0, sizeof(float) * u->nparams, s));
  float *ga = u->ga, *gb = u->gb;
  // head (1x1, no activation): dY is the caller's buffer; copy-free because it is only read
  int st = layer_back(u, u->head(), const_cast<float*>(dy), Lv > 1 ? u->db[0] : u->eb[0], nullptr, ga, B, H, W, s);
  if (st) return st;
  for (int l = 0; l <= Lv - 2; ++l) {
    const int h = H >> l, w = W >> l;
    if ((st = layer_back(u, u->dec(l, 1), ga, u->da[l], u->db[l], gb, B, h, w, s))) return st;
    if ((st = layer_back(u, u->dec(l, 0), gb, u->cat[l], u->da[l], ga, B, h, w, s))) return st;
    const double e = (double)B * h * w * (u->ch(l + 1) + u->ch(l));
    LSOP_HIP(prof_launch("unet upsample+concat backward", "k_upcat_bwd",
                         e * 4.0 + (double)B * h * w * (u->ch(l + 1) / 4.0 + u->ch(l)) * 4.0, e, e, s,
                         [&] { return launch_upcat_bwd(ga, gb, u->skipg[l], B, h / 2, w / 2, u->ch(l + 1), u->ch(l), s); }));
    std::swap(ga, gb);
  }
  for (int l = Lv - 1; l >= 0; --l) {
    const int h = H >> l, w = W >> l;
    if (l < Lv - 1) {
      const double e = (double)B * h * w * u->ch(l);
      LSOP_HIP(prof_launch("unet pool backward", "k_avgpool2_bwd", e * 4.0 * 2.25, e, e, s,
                           [&] { return launch_avgpool2_bwd(ga, u->skipg[l], gb, B, h / 2, w / 2, u->ch(l), s); }));
      std::swap(ga, gb);
    }
    if ((st = layer_back(u, u->enc(l, 1), ga, u->ea[l], u->eb[l], gb, B, h, w, s))) return st;
    const float* in = l == 0 ? u->x_last : u->pool[l - 1];
    if ((st = layer_back(u, u->enc(l, 0), gb, in, u->ea[l], l > 0 ? ga : nullptr, B, h, w, s))) return st;
  }
  return LSOP_OK;
}

int check_shape(const unet* u, int B, int H, int W) {
  const int m = 1 << (u->levels - 1);
  if (B < 1 || B > u->maxB || H < m || W < m || H > u->maxH || W > u->maxW || H % m || W % m)
    return fail(LSOP_EINVAL, "batch / size outside the network's limits or not divisible by 2^(levels-1)");
  return LSOP_OK;
}

}  // namespace

extern "C" {

int unet_create(int levels, int base, int cin, int cout, int max_batch, int max_h, int max_w, unet** out) {
  if (!out) return fail(LSOP_EINVAL, "null output handle");
  *out = nullptr;
  if (levels < 1 || levels > 6 || base < 1 || base > 256 || cin < 1 || cout < 1 || max_batch < 1 || max_h < 1 ||
      max_w < 1)
    return fail(LSOP_EINVAL, "bad network shape");
  unet* u = new unet();
  u->levels = levels;
  u->base = base;
  u->cin = cin;
  u->cout = cout;
  u->maxB = max_batch;
  u->maxH = max_h;
  u->maxW = max_w;
  auto add = [&](int ks, int ci, int co) {
    unet::Layer L;
    L.ks = ks;
    L.ci = ci;
    L.co = co;
    L.poff = u->nparams;
    u->nparams += (size_t)ks * ks * ci * co + co;
    u->layers.push_back(L);
  };
  int prev = cin;
  for (int l = 0; l < levels; ++l) {
    add(3, prev, u->ch(l));
    add(3, u->ch(l), u->ch(l));
    prev = u->ch(l);
  }
  for (int l = levels - 2; l >= 0; --l) {
    add(3, u->ch(l + 1) + u->ch(l), u->ch(l));
    add(3, u->ch(l), u->ch(l));
  }
  add(1, u->ch(0), cout);
  int st = 0;
  const size_t np = u->nparams;
  st |= nn_alloc(u, &u->P, sizeof(float) * np);
  st |= nn_alloc(u, &u->G, sizeof(float) * np);
  st |= nn_alloc(u, &u->M, sizeof(float) * np);
  st |= nn_alloc(u, &u->V, sizeof(float) * np);
  for (auto& L : u->layers) {
    const size_t nw = (size_t)L.ks * L.ks * L.ci * L.co;
    st |= nn_alloc(u, &L.wb, sizeof(unsigned short) * nw);
    st |= nn_alloc(u, &L.wt, sizeof(unsigned short) * nw);
  }
  const size_t P0 = (size_t)max_batch * max_h * max_w;
  u->ea.resize(levels);
  u->eb.resize(levels);
  u->pool.resize(levels);
  u->cat.resize(levels);
  u->da.resize(levels);
  u->db.resize(levels);
  u->skipg.resize(levels);
  for (int l = 0; l < levels && !st; ++l) {
    const size_t Pl = P0 >> (2 * l);
    st |= nn_alloc(u, &u->ea[l], sizeof(float) * Pl * u->ch(l));
    st |= nn_alloc(u, &u->eb[l], sizeof(float) * Pl * u->ch(l));
    if (l < levels - 1) {
      st |= nn_alloc(u, &u->pool[l], sizeof(float) * (Pl / 4) * u->ch(l));
      st |= nn_alloc(u, &u->cat[l], sizeof(float) * Pl * (u->ch(l + 1) + u->ch(l)));
      st |= nn_alloc(u, &u->da[l], sizeof(float) * Pl * u->ch(l));
      st |= nn_alloc(u, &u->db[l], sizeof(float) * Pl * u->ch(l));
      st |= nn_alloc(u, &u->skipg[l], sizeof(float) * Pl * u->ch(l));
    }
  }
  const size_t gmax = P0 * (size_t)std::max(3 * base, std::max(cin, cout));
  st |= nn_alloc(u, &u->ga, sizeof(float) * gmax);
  st |= nn_alloc(u, &u->gb, sizeof(float) * gmax);
  st |= nn_alloc(u, &u->xin, sizeof(float) * P0 * cin);
  st |= nn_alloc(u, &u->yout, sizeof(float) * P0 * cout);
  st |= nn_alloc(u, &u->dout, sizeof(float) * P0 * cout);
  st |= nn_alloc(u, &u->scale, sizeof(float) * max_batch);
  st |= nn_alloc(u, &u->dloss, sizeof(double) * 2);
  st |= nn_alloc(u, &u->norms, sizeof(double) * max_batch);
  if (st) {
    for (void* p : u->owned) (void)hipFree(p);
    delete u;
    return LSOP_ENOMEM;
  }
  *out = u;
  return LSOP_OK;
}

int unet_param_count(const unet* u, size_t* n) {
  if (!u || !n) return fail(LSOP_EINVAL, "null argument");
  *n = u->nparams;
  return LSOP_OK;
}

int unet_set_params(unet* u, const float* params_dev, void* stream) {
  if (!u || !params_dev) return fail(LSOP_EINVAL, "null argument");
  hipStream_t s = SS(stream);
  LSOP_HIP(hipMemcpyAsync(u->P, params_dev, sizeof(float) * u->nparams, hipMemcpyDeviceToDevice, s));
  LSOP_HIP(hipMemsetAsync(u->M, 0, sizeof(float) * u->nparams, s));
  LSOP_HIP(hipMemsetAsync(u->V, 0, sizeof(float) * u->nparams, s));
  u->step = 0;
  return refresh_weights(u, s);
}

int unet_init_params(unet* u, unsigned long long seed, void* stream) {
  if (!u) return fail(LSOP_EINVAL, "null argument");
  hipStream_t s = SS(stream);
  // one standard normal draw per parameter: the range finder's Philox4x32-10 generator, which writes real
  // draws as complex numbers with zero imaginary part (read with stride 2) into a temporary buffer
  Cx<float>* z = nullptr;
  if (lib_malloc(reinterpret_cast<void**>(&z), sizeof(Cx<float>) * u->nparams) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LSOP_ENOMEM, "unet_init_params: temporary of " + std::to_string(u->nparams) + " draws");
  }
  int st = LSOP_OK;
  if (launch_philox_normal<float>(z, 1, u->nparams, seed, s) != hipSuccess) st = fail(LSOP_EHIP, "philox launch");
  for (const auto& L : u->layers) {
    if (st) break;
    const size_t nw = (size_t)L.ks * L.ks * L.ci * L.co;
    if (launch_scale_copy(u->P + L.poff, reinterpret_cast<const float*>(z + L.poff), nw, 2,
                          std::sqrt(2.0f / (float)(L.ks * L.ks * L.ci)), s) != hipSuccess ||
        hipMemsetAsync(u->P + L.poff + nw, 0, sizeof(float) * L.co, s) != hipSuccess)
      st = fail(LSOP_EHIP, "unet_init_params launch");
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(z);
  if (st) return st;
  LSOP_HIP(hipMemsetAsync(u->M, 0, sizeof(float) * u->nparams, s));
  LSOP_HIP(hipMemsetAsync(u->V, 0, sizeof(float) * u->nparams, s));
  u->step = 0;
  return refresh_weights(u, s);
}

int unet_get_params(const unet* u, float* params_dev, void* stream) {
  if (!u || !params_dev) return fail(LSOP_EINVAL, "null argument");
  LSOP_HIP(hipMemcpyAsync(params_dev, u->P, sizeof(float) * u->nparams, hipMemcpyDeviceToDevice, SS(stream)));
  return LSOP_OK;
}

int unet_forward(unet* u, const float* x_dev, int B, int H, int W, float* y_dev, void* stream) {
  if (!u || !x_dev || !y_dev) return fail(LSOP_EINVAL, "null argument");
  int st = check_shape(u, B, H, W);
  if (st) return st;
  return forward(u, x_dev, B, H, W, y_dev, SS(stream));
}

int unet_backward(unet* u, const float* dy_dev, void* stream) {
  if (!u || !dy_dev) return fail(LSOP_EINVAL, "null argument");
  if (!u->have_fwd) return fail(LSOP_EINVAL, "unet_backward needs a preceding unet_forward");
  return backward(u, dy_dev, SS(stream));
}

int unet_get_grads(const unet* u, float* grads_dev, void* stream) {
  if (!u || !grads_dev) return fail(LSOP_EINVAL, "null argument");
  LSOP_HIP(hipMemcpyAsync(grads_dev, u->G, sizeof(float) * u->nparams, hipMemcpyDeviceToDevice, SS(stream)));
  return LSOP_OK;
}

int unet_train_step(unet* u, const float* x_dev, const float* target_dev, int B, int H, int W, float lr,
                    double* loss_host, void* stream) {
  if (!u || !x_dev || !target_dev) return fail(LSOP_EINVAL, "null argument");
  if (!(lr > 0.f)) return fail(LSOP_EINVAL, "lr must be > 0");
  int st = check_shape(u, B, H, W);
  if (st) return st;
  hipStream_t s = SS(stream);
  if ((st = forward(u, x_dev, B, H, W, u->yout, s))) return st;
  LSOP_HIP(hipMemsetAsync(u->dloss, 0, sizeof(double), s));
  const size_t n = (size_t)B * H * W * u->cout;
  LSOP_HIP(prof_launch("unet loss", "k_mse", (double)n * 12.0, 3.0 * n, (double)n, s,
                       [&] { return launch_mse(u->yout, target_dev, u->dout, n, u->dloss, s); }));
  if ((st = backward(u, u->dout, s))) return st;
  ++u->step;
  LSOP_HIP(prof_launch("unet adam", "k_adam", (double)u->nparams * 28.0, 12.0 * u->nparams, (double)u->nparams, s,
                       [&] { return launch_adam(u->P, u->G, u->M, u->V, u->nparams, lr, 0.9, 0.999, 1e-8, u->step, s); }));
  if ((st = refresh_weights(u, s))) return st;
  if (loss_host) {
    LSOP_HIP(hipMemcpyAsync(loss_host, u->dloss, sizeof(double), hipMemcpyDeviceToHost, s));
    LSOP_HIP(hipStreamSynchronize(s));
  }
  return LSOP_OK;
}

int unet_pack_inputs(unet* u, const lsop_op* op, const void* psi0_dev, int nvec, float* x_dev, float* scale_dev,
                     void* stream) {
  if (!u || !op || !psi0_dev || !x_dev || !scale_dev) return fail(LSOP_EINVAL, "null argument");
  if (!op->ready) return fail(LSOP_EINVAL, "operator has no problem set");
  if (op->dims != 2) return fail(LSOP_EUNSUPPORTED, "the warm-start network takes 2D operators");
  if (u->cin != 4) return fail(LSOP_EINVAL, "the warm start takes 4 input channels");
  if (nvec < 1 || nvec > u->maxB) return fail(LSOP_EINVAL, "nvec outside the network's batch limit");
  hipStream_t s = SS(stream);
  const size_t n = op->n();
  const double w = 2.0 * 3.14159265358979323846 * op->freq;
  const double c0w2 = op->c0 * op->c0 / (w * w);
  const float k0h = (float)(op->k0 * op->h);
  if (op->dtype == LSOP_C64) {
    LSOP_HIP(launch_norm2<float>((const Cx<float>*)psi0_dev, u->norms, nullptr, nvec, n, s));
    LSOP_HIP(launch_pack_inputs<float>(op->chi64, (const Cx<float>*)psi0_dev, u->norms, x_dev, nvec, n, c0w2, k0h,
                                       scale_dev, s));
  } else {
    LSOP_HIP(launch_norm2<double>((const Cx<double>*)psi0_dev, u->norms, nullptr, nvec, n, s));
    LSOP_HIP(launch_pack_inputs<double>(op->chi64, (const Cx<double>*)psi0_dev, u->norms, x_dev, nvec, n, c0w2, k0h,
                                        scale_dev, s));
  }
  return LSOP_OK;
}

int unet_pack_target(const lsop_op* op, const void* psi_dev, const void* psi0_dev, const float* scale_dev, int nvec,
                     float* t_dev, void* stream) {
  if (!op || !psi_dev || !psi0_dev || !scale_dev || !t_dev) return fail(LSOP_EINVAL, "null argument");
  if (op->dims != 2) return fail(LSOP_EUNSUPPORTED, "the warm-start network takes 2D operators");
  if (nvec < 1) return fail(LSOP_EINVAL, "nvec must be >= 1");
  hipStream_t s = SS(stream);
  if (op->dtype == LSOP_C64)
    LSOP_HIP(launch_pack_target<float>((const Cx<float>*)psi_dev, (const Cx<float>*)psi0_dev, scale_dev, t_dev, nvec,
                                       op->n(), s));
  else
    LSOP_HIP(launch_pack_target<double>((const Cx<double>*)psi_dev, (const Cx<double>*)psi0_dev, scale_dev, t_dev,
                                        nvec, op->n(), s));
  return LSOP_OK;
}

int unet_warm_start(unet* u, const lsop_op* op, const void* psi0_dev, void* psi_dev, int nvec, void* stream) {
  if (!u || !op || !psi0_dev || !psi_dev) return fail(LSOP_EINVAL, "null argument");
  if (op->dims != 2) return fail(LSOP_EUNSUPPORTED, "the warm-start network takes 2D operators");
  if (u->cout != 2) return fail(LSOP_EINVAL, "the warm start takes 2 output channels");
  int st = check_shape(u, nvec, op->nx, op->nz);
  if (st) return st;
  hipStream_t s = SS(stream);
  if ((st = unet_pack_inputs(u, op, psi0_dev, nvec, u->xin, u->scale, stream))) return st;
  if ((st = forward(u, u->xin, nvec, op->nx, op->nz, u->yout, s))) return st;
  const size_t n = op->n();
  if (op->dtype == LSOP_C64)
    LSOP_HIP(launch_unpack_output<float>((const Cx<float>*)psi0_dev, u->yout, u->scale, (Cx<float>*)psi_dev, nvec, n,
                                         s));
  else
    LSOP_HIP(launch_unpack_output<double>((const Cx<double>*)psi0_dev, u->yout, u->scale, (Cx<double>*)psi_dev, nvec,
                                          n, s));
  return LSOP_OK;
}

int unet_info(const unet* u, size_t* params, size_t* bytes) {
  if (!u) return fail(LSOP_EINVAL, "null network");
  if (params) *params = u->nparams;
  if (bytes) *bytes = u->bytes;
  return LSOP_OK;
}

void unet_destroy(unet* u) {
  if (!u) return;
  (void)hipDeviceSynchronize();
  for (void* p : u->owned) (void)hipFree(p);
  delete u;
}

}  // extern "C"
