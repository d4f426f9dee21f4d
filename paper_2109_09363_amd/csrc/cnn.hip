// Multi-scale CNN initial guess of the pressure (Sec. 3.1: several
// resolutions of the same input, replication padding, ReLU hidden layers,
// bilinear down/up sampling, linear output):
//   x   = [d / s, solid], s = sqrt(mean_F d^2)
//   x_k = 2x2 mean pyramid, k = 0..S-1
//   y_k = conv1x1(relu(conv3x3(... 4 layers ...)))   per scale, own weights
//   t   = y_{S-1};  t = y_k + up2(t) for k = S-2..0;   phi0 = dx^2 s t (fluid)
//
// The 3x3 convolutions are the implicit GEMMs on MFMA of conv_mfma.h; all
// scales of a layer run in one launch over a concatenated tile list.
#include <hip/hip_runtime.h>

#include "../../include/hyproj.h"
#include "common.h"
#include "conv_mfma.h"
#include "internal.h"

namespace hyp {

// ---- pyramid input: level k pixel = mean over its 2^k x 2^k block of ------
// [d/s, solid]; stored NHWC with 2 channels in the storage type.
struct PyrLaunch {
  void* out[kMaxScales];
  int H[kMaxScales], W[kMaxScales];
  size_t px0[kMaxScales];
  int nscales;
  size_t total_px;
  int nx;
};

template <typename T>
__global__ __launch_bounds__(256) void cnn_input(PyrLaunch P, const float* __restrict__ d,
                                                 const uint8_t* __restrict__ cell,
                                                 const Scalars* sc) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= P.total_px) return;
  int k = 0;
  while (k + 1 < P.nscales && gid >= P.px0[k + 1]) ++k;
  const int lp = (int)(gid - P.px0[k]);
  const int X = lp % P.W[k], Y = lp / P.W[k];
  const int B = 1 << k;
  const double s = sc->s;
  const float inv_s = s > 0.0 ? (float)(1.0 / s) : 0.f;
  float sd = 0.f, ss = 0.f;
  for (int yy = 0; yy < B; ++yy)
    for (int xx = 0; xx < B; ++xx) {
      const int c = (Y * B + yy) * P.nx + X * B + xx;
      const bool solid = cell[c] & C_SOLID;
      sd += solid ? 0.f : d[c] * inv_s;
      ss += solid ? 1.f : 0.f;
    }
  const float inv_n = 1.f / (float)(B * B);
  T* o = reinterpret_cast<T*>(P.out[k]) + (size_t)lp * 2;
  o[0] = St<T>::from(sd * inv_n);
  o[1] = St<T>::from(ss * inv_n);
}

// ---- head: y = w_out . act + b_out (1x1, linear) for every pixel ---------
struct HeadLaunch {
  const void* act[kMaxScales];
  const float* w[kMaxScales];
  const float* b[kMaxScales];
  size_t px0[kMaxScales];
  int nscales;
  size_t total_px;
};

template <typename T, int C>
__global__ __launch_bounds__(256) void cnn_head(HeadLaunch Hd, float* __restrict__ y) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= Hd.total_px) return;
  int k = 0;
  while (k + 1 < Hd.nscales && gid >= Hd.px0[k + 1]) ++k;
  const size_t lp = gid - Hd.px0[k];
  const T* a = reinterpret_cast<const T*>(Hd.act[k]) + lp * C;
  const float* w = Hd.w[k];
  float acc = 0.f;
#pragma unroll 8
  for (int c = 0; c < C; ++c) acc += St<T>::to_f(a[c]) * w[c];
  y[gid] = acc + Hd.b[k][0];
}

// ---- t_k = y_k + up2(t_{k+1}); at k = 0 also phi0 = dx^2 s t on fluid -----
__global__ __launch_bounds__(256) void cnn_upsum(int H, int W, const float* __restrict__ yk,
                                                 const float* __restrict__ tc, int Hc, int Wc,
                                                 float* __restrict__ tk, int last, float dx2,
                                                 const uint8_t* __restrict__ cell,
                                                 float* __restrict__ phi, const Scalars* sc) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= H * W) return;
  const int X = gid % W, Y = gid / W;
  float t = yk[gid];
  if (tc) {
    float cy = fminf(fmaxf(0.5f * (float)Y - 0.25f, 0.f), (float)(Hc - 1));
    float cx = fminf(fmaxf(0.5f * (float)X - 0.25f, 0.f), (float)(Wc - 1));
    int y0 = min((int)floorf(cy), max(Hc - 2, 0));
    int x0 = min((int)floorf(cx), max(Wc - 2, 0));
    const float fy = cy - (float)y0, fx = cx - (float)x0;
    const int y1 = min(y0 + 1, Hc - 1), x1 = min(x0 + 1, Wc - 1);
    const float a = tc[y0 * Wc + x0], b = tc[y0 * Wc + x1];
    const float c = tc[y1 * Wc + x0], d = tc[y1 * Wc + x1];
    t += (1.f - fy) * ((1.f - fx) * a + fx * b) + fy * ((1.f - fx) * c + fx * d);
  }
  tk[gid] = t;
  if (last) {
    const double s = sc->s;
    const bool fl = !(cell[gid] & C_SOLID);
    phi[gid] = (fl && s > 0.0) ? (float)((double)dx2 * s) * t : 0.f;
  }
}

// ---- weight images: every 3x3 layer's weights in the LDS layout of the conv
// kernel ([Cout][WSTR], storage type, K zero-padded), written once per
// inference so that a work-group copies them with wide loads.
template <typename T, int C>
struct WImg {
  static constexpr size_t L0 = (size_t)C * ConvGeom<T, 3, 2, C>::WSTR;   // elements, layer 0
  static constexpr size_t L1 = (size_t)C * ConvGeom<T, 3, C, C>::WSTR;   // elements, layers 1..3
  static constexpr size_t PER_SCALE = L0 + 3 * L1;
};

template <typename T, int C>
__global__ __launch_bounds__(256) void cnn_wimg(const float* __restrict__ params, size_t per_scale,
                                                int nscales, T* __restrict__ img) {
  using WI = WImg<T, C>;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= WI::PER_SCALE * nscales) return;
  const int k = (int)(gid / WI::PER_SCALE);
  size_t e = gid % WI::PER_SCALE;
  const float* wk = params + k * per_scale;
  T* ik = img + k * WI::PER_SCALE;
  if (e < WI::L0) {
    write_wimg<T, 3, 2, C>(wk, ik, (int)e);
    return;
  }
  e -= WI::L0;
  const int l = 1 + (int)(e / WI::L1);
  const int el = (int)(e % WI::L1);
  const size_t woff = (size_t)C * 18 + C + (size_t)(l - 1) * ((size_t)C * 9 * C + C);
  write_wimg<T, 3, C, C>(wk + woff, ik + WI::L0 + (size_t)(l - 1) * WI::L1, el);
}

size_t cnn_weight_image_bytes(const NetShape& net) {
  if (net.scales <= 0) return 0;
  if (net.arch != HYP_ARCH_PARALLEL) return pn_weight_image_bytes(net);
  if (net.precision == HYP_PREC_BF16) {
    if (net.channels == 32) return WImg<uint16_t, 32>::PER_SCALE * net.scales * 2;
    if (net.channels == 64) return WImg<uint16_t, 64>::PER_SCALE * net.scales * 2;
  } else {
    if (net.channels == 16) return WImg<float, 16>::PER_SCALE * net.scales * 4;
    if (net.channels == 32) return WImg<float, 32>::PER_SCALE * net.scales * 4;
    if (net.channels == 64) return WImg<float, 64>::PER_SCALE * net.scales * 4;
  }
  return 0;
}

// ---------------------------------------------------------------------------
template <typename T, int C>
static hipError_t run_cnn_t(const Device& dev, const NetShape& net, const WsLayout& Ly, int nx,
                            int ny, double dx, const float* params, const Ws& w, hipStream_t s) {
  const int S = net.scales;
  const size_t per_scale = (size_t)C * 18 + C + 3 * ((size_t)C * 9 * C + C) + C + 1;
  T* in = reinterpret_cast<T*>(w.cnn_in);
  T* a0 = reinterpret_cast<T*>(w.cnn_act0);
  T* a1 = reinterpret_cast<T*>(w.cnn_act1);
  // pyramid input
  PyrLaunch P{};
  P.nscales = S;
  P.total_px = Ly.total_px;
  P.nx = nx;
  for (int k = 0; k < S; ++k) {
    P.out[k] = in + Ly.sc_off_px[k] * 2;
    P.H[k] = Ly.sc_h[k];
    P.W[k] = Ly.sc_w[k];
    P.px0[k] = Ly.sc_off_px[k];
  }
  const int nb_px = (int)((Ly.total_px + 255) / 256);
  hipLaunchKernelGGL(cnn_input<T>, dim3(nb_px), dim3(256), 0, s, P, w.d, w.cell, w.sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  using WI = WImg<T, C>;
  T* img = reinterpret_cast<T*>(w.cnn_w);
  const size_t nimg = WI::PER_SCALE * S;
  hipLaunchKernelGGL((cnn_wimg<T, C>), dim3((unsigned)((nimg + 255) / 256)), dim3(256), 0, s, params,
                     per_scale, S, img);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // four 3x3 layers, all scales per launch
  const T* src = in;
  T* bufs[2] = {a0, a1};
  T* save = reinterpret_cast<T*>(w.cnn_save);
  for (int l = 0; l < 4; ++l) {
    T* dst = net.train ? save + (size_t)l * Ly.total_px * C : bufs[l & 1];
    ConvLaunch L{};
    L.nscales = S;
    int tiles = 0;
    const int cin = l == 0 ? 2 : C;
    size_t woff = l == 0 ? 0 : (size_t)C * 18 + C + (size_t)(l - 1) * ((size_t)C * 9 * C + C);
    for (int k = 0; k < S; ++k) {
      ScaleDesc& D = L.sc[k];
      D.in = src + Ly.sc_off_px[k] * cin;
      D.out = dst + Ly.sc_off_px[k] * C;
      D.wimg = img + k * WI::PER_SCALE + (l == 0 ? 0 : WI::L0 + (size_t)(l - 1) * WI::L1);
      D.b = params + k * per_scale + woff + (size_t)C * 9 * cin;
      D.H = Ly.sc_h[k];
      D.W = Ly.sc_w[k];
      D.tiles_x = (D.W + TW - 1) / TW;
      D.tile0 = tiles;
      D.ostr = C;
      tiles += D.tiles_x * ((D.H + TH - 1) / TH);
    }
    L.total_tiles = tiles;
    // launch on the caller's stream
    e = l == 0 ? launch_conv<T, 3, 2, C, true>(L, dev.cu, s) : launch_conv<T, 3, C, C, true>(L, dev.cu, s);
    if (e != hipSuccess) return e;
    src = dst;
  }
  // 1x1 head for every scale
  HeadLaunch Hd{};
  Hd.nscales = S;
  Hd.total_px = Ly.total_px;
  const size_t hoff = (size_t)C * 18 + C + 3 * ((size_t)C * 9 * C + C);
  for (int k = 0; k < S; ++k) {
    Hd.act[k] = src + Ly.sc_off_px[k] * C;
    Hd.w[k] = params + k * per_scale + hoff;
    Hd.b[k] = Hd.w[k] + C;
    Hd.px0[k] = Ly.sc_off_px[k];
  }
  hipLaunchKernelGGL((cnn_head<T, C>), dim3(nb_px), dim3(256), 0, s, Hd, w.cnn_y);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // coarse-to-fine upsample-sum
  for (int k = S - 1; k >= 0; --k) {
    const int H = Ly.sc_h[k], W = Ly.sc_w[k];
    const float* tc = k == S - 1 ? nullptr : w.cnn_t + Ly.sc_off_px[k + 1];
    const int Hc = k == S - 1 ? 0 : Ly.sc_h[k + 1], Wc = k == S - 1 ? 0 : Ly.sc_w[k + 1];
    hipLaunchKernelGGL(cnn_upsum, dim3((H * W + 255) / 256), dim3(256), 0, s, H, W,
                       w.cnn_y + Ly.sc_off_px[k], tc, Hc, Wc, w.cnn_t + Ly.sc_off_px[k], k == 0 ? 1 : 0,
                       (float)(dx * dx), w.cell, w.phi, w.sc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_cnn(const Device& dev, const NetShape& net, const WsLayout& L, int nx, int ny,
                   double dx, const float* params, const Ws& w, hipStream_t s) {
  if (net.arch != HYP_ARCH_PARALLEL) return run_papernet(dev, net, L, nx, ny, dx, params, w, s);
  if (net.precision == HYP_PREC_BF16) {
    switch (net.channels) {
      case 32: return run_cnn_t<uint16_t, 32>(dev, net, L, nx, ny, dx, params, w, s);
      case 64: return run_cnn_t<uint16_t, 64>(dev, net, L, nx, ny, dx, params, w, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (net.channels) {
    case 16: return run_cnn_t<float, 16>(dev, net, L, nx, ny, dx, params, w, s);
    case 32: return run_cnn_t<float, 32>(dev, net, L, nx, ny, dx, params, w, s);
    case 64: return run_cnn_t<float, 64>(dev, net, L, nx, ny, dx, params, w, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hyp
