// The paper's cascaded MultiScale network and its SmallScale variant as the
// initial guess of the pressure (Sec. 3.1, Fig. 3): three branches at n/4,
// n/2 and n pixels a side, run coarse to fine.  A branch sees the input
// x = [d / s, solid] resampled to its size (bilinear, half-pixel centres),
// plus, below the coarsest, the previous branch's output upsampled x2 as a
// third channel; it opens with a 5x5 convolution, continues with 3x3 ones
// and ends with a 1x1 convolution to one channel; ReLU follows every layer
// but the last two.  phi0 = dx^2 s y_n on fluid cells.
//
// Widths (the paper's figure with them is missing): 64 channels everywhere
// except a 32-channel middle layer in the two finer branches (419,459
// parameters against the paper's 418,640); SmallScale 32 everywhere
// (126,819 against "about 1.3e5").
//
// The paper's Unet (Sec. 3.1, Fig. 4): five scales n .. n/16; two 3x3
// convolutions with ReLU per scale on the way down and 2x2 max pooling
// between scales; on the way up bilinear x2 upsampling, concatenation with
// the encoder output of the same scale (skip channels first) and two 3x3
// convolutions with ReLU; a linear 1x1 output.  Widths 16, 16, 64, 64, 64
// (443,441 parameters against the paper's 443,521).  The encoder writes its
// output straight into the concatenation buffer of its scale, and the
// upsampling writes the other half, so no copy is made.
//
// Every k > 1 layer is one launch of conv_mfma (implicit GEMM on MFMA, FP32
// or BF16 storage); the 1x1 output layer, the resampling and the pooling are
// small elementwise kernels.  The layer weights are re-laid into the LDS
// image of the convolution kernel once per inference, in one launch.
#include <hip/hip_runtime.h>

#include "../../include/hyproj.h"
#include "common.h"
#include "conv_mfma.h"
#include "internal.h"
#include "cascade.h"
#include "unet.h"

namespace hyp {


// Unet layers in parameter order: encoder scales 0..4 (two each), decoder
// scales 3..0 (two each), the 1x1 output.
static int unet_layers(PnLayer* out) {
  int n = 0, cin = 2;
  for (int l = 0; l < kUnetLevels; ++l) {
    out[n++] = {3, cin, kUnetW[l], true};
    out[n++] = {3, kUnetW[l], kUnetW[l], true};
    cin = kUnetW[l];
  }
  for (int l = kUnetLevels - 2; l >= 0; --l) {
    out[n++] = {3, kUnetW[l] + kUnetW[l + 1], kUnetW[l], true};
    out[n++] = {3, kUnetW[l], kUnetW[l], true};
  }
  out[n++] = {1, kUnetW[0], 1, false};
  return n;
}

// Every layer of the network in parameter order; returns the count.
static int all_layers(int arch, PnLayer* out) {
  if (arch == HYP_ARCH_UNET) return unet_layers(out);
  int n = 0;
  for (int b = 0; b < 3; ++b) n += pn_branch(arch, b, out + n);
  return n;
}

// Elements of a layer's weight image ([NCH][Cout][WSTR]).
static size_t wimg_elems(const PnLayer& l, int elt) {
  const int cc = conv_cc(elt, l.ks, l.cin);
  return (size_t)(l.cin / cc) * l.cout * conv_wstr(elt, l.ks, cc);
}

size_t unet_cat_elems(int nx, int ny) { return unet_cat_offset(nx, ny, kUnetLevels - 1); }

int64_t pn_param_count(int arch) {
  PnLayer L[kUnetLayers];
  const int nl = all_layers(arch, L);
  int64_t n = 0;
  for (int i = 0; i < nl; ++i) n += (int64_t)L[i].ks * L[i].ks * L[i].cin * L[i].cout + L[i].cout;
  return n;
}

size_t pn_weight_image_bytes(const NetShape& net) {
  const int elt = net.precision == HYP_PREC_BF16 ? 2 : 4;
  PnLayer L[kUnetLayers];
  const int nl = all_layers(net.arch, L);
  size_t bytes = 0;
  for (int i = 0; i < nl; ++i)
    if (L[i].ks > 1) bytes += wimg_elems(L[i], elt) * elt;
  return bytes;
}

// ---- weight images of every k > 1 layer in one launch -------------------
constexpr int kPnMaxImg = kUnetLayers;
static_assert(kPnMaxImg >= 5 + 2 * kPnMaxLayers, "image table holds every cascade layer");
struct PnImgLaunch {
  size_t src[kPnMaxImg];   // float offset of W in the packed parameters
  size_t dst[kPnMaxImg];   // element offset of the image
  size_t e0[kPnMaxImg + 1];
  int ks[kPnMaxImg], cin[kPnMaxImg], cout[kPnMaxImg], cc[kPnMaxImg], wstr[kPnMaxImg];
  int n;
};

template <typename T>
__global__ __launch_bounds__(256) void pn_wimg(PnImgLaunch D, const float* __restrict__ params,
                                               T* __restrict__ img) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= D.e0[D.n]) return;
  int l = 0;
  while (gid >= D.e0[l + 1]) ++l;
  const size_t e = gid - D.e0[l];
  // [NCH][Cout][WSTR]; column kk = tap * cc + c holds input channel ch * cc + c
  const size_t rowlen = (size_t)D.cout[l] * D.wstr[l];
  const int ch = (int)(e / rowlen);
  const size_t r = e % rowlen;
  const int co = (int)(r / D.wstr[l]), kk = (int)(r % D.wstr[l]);
  float v = 0.f;
  if (kk < D.ks[l] * D.ks[l] * D.cc[l]) {
    const int tap = kk / D.cc[l], c = kk % D.cc[l];
    v = params[D.src[l] + (size_t)co * D.ks[l] * D.ks[l] * D.cin[l] + (size_t)tap * D.cin[l] +
               ch * D.cc[l] + c];
  }
  img[D.dst[l] + e] = St<T>::from(v);
}

// ---- branch input: x resampled to 1/f size, plus up2(y_coarse) ----------
template <typename T>
__global__ __launch_bounds__(256) void pn_input(int H, int W, int f, int nx,
                                                const float* __restrict__ d,
                                                const uint8_t* __restrict__ cell,
                                                const Scalars* sc, const float* __restrict__ yc,
                                                int Hc, int Wc, T* __restrict__ out) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= H * W) return;
  const int X = gid % W, Y = gid / W;
  const double s = sc->s;
  const float inv_s = s > 0.0 ? (float)(1.0 / s) : 0.f;
  float xd = 0.f, xs = 0.f;
  if (f == 1) {
    const int c = Y * nx + X;
    const bool solid = cell[c] & C_SOLID;
    xd = solid ? 0.f : d[c] * inv_s;
    xs = solid ? 1.f : 0.f;
  } else {
    // bilinear at (I + 0.5) f - 0.5 = f I + f/2 - 1 + 0.5: the mean of 2x2
    const int fy = Y * f + f / 2 - 1, fx = X * f + f / 2 - 1;
    for (int yy = 0; yy < 2; ++yy)
      for (int xx = 0; xx < 2; ++xx) {
        const int c = (fy + yy) * nx + fx + xx;
        const bool solid = cell[c] & C_SOLID;
        xd += solid ? 0.f : d[c] * inv_s;
        xs += solid ? 1.f : 0.f;
      }
    xd *= 0.25f;
    xs *= 0.25f;
  }
  const int cin = yc ? 3 : 2;
  T* o = out + (size_t)gid * cin;
  o[0] = St<T>::from(xd);
  o[1] = St<T>::from(xs);
  if (yc) {
    // bilinear x2, half-pixel centres, edge clamp
    const float cy = fminf(fmaxf(0.5f * (float)Y - 0.25f, 0.f), (float)(Hc - 1));
    const float cx = fminf(fmaxf(0.5f * (float)X - 0.25f, 0.f), (float)(Wc - 1));
    const int y0 = min((int)floorf(cy), max(Hc - 2, 0));
    const int x0 = min((int)floorf(cx), max(Wc - 2, 0));
    const float wy = cy - (float)y0, wx = cx - (float)x0;
    const int y1 = min(y0 + 1, Hc - 1), x1 = min(x0 + 1, Wc - 1);
    const float a = yc[y0 * Wc + x0], b = yc[y0 * Wc + x1];
    const float c = yc[y1 * Wc + x0], e = yc[y1 * Wc + x1];
    o[2] = St<T>::from((1.f - wy) * ((1.f - wx) * a + wx * b) + wy * ((1.f - wx) * c + wx * e));
  }
}

// ---- 1x1 output layer; on the finest branch also phi0 = dx^2 s y --------
template <typename T, int C>
__global__ __launch_bounds__(256) void pn_head(int npx, const T* __restrict__ act,
                                               const float* __restrict__ w, float* __restrict__ y,
                                               int last, float dx2, const uint8_t* __restrict__ cell,
                                               float* __restrict__ phi, const Scalars* sc) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= npx) return;
  const T* a = act + (size_t)gid * C;
  float acc = 0.f;
#pragma unroll 8
  for (int c = 0; c < C; ++c) acc += St<T>::to_f(a[c]) * w[c];
  const float v = acc + w[C];
  y[gid] = v;
  if (last) {
    const double s = sc->s;
    const bool fl = !(cell[gid] & C_SOLID);
    phi[gid] = (fl && s > 0.0) ? (float)((double)dx2 * s) * v : 0.f;
  }
}

template <typename T>
static hipError_t pn_conv(const PnLayer& l, ConvLaunch& L, int cu, hipStream_t s) {
  const int k = l.ks, ci = l.cin, co = l.cout;
  const bool r = l.relu;
  // cascaded MultiScale / SmallScale
  if (k == 5 && ci == 2 && co == 64 && r) return launch_conv<T, 5, 2, 64, true>(L, cu, s);
  if (k == 5 && ci == 3 && co == 64 && r) return launch_conv<T, 5, 3, 64, true>(L, cu, s);
  if (k == 5 && ci == 2 && co == 32 && r) return launch_conv<T, 5, 2, 32, true>(L, cu, s);
  if (k == 5 && ci == 3 && co == 32 && r) return launch_conv<T, 5, 3, 32, true>(L, cu, s);
  if (k == 3 && ci == 64 && co == 64) {
    return r ? launch_conv<T, 3, 64, 64, true>(L, cu, s) : launch_conv<T, 3, 64, 64, false>(L, cu, s);
  }
  if (k == 3 && ci == 64 && co == 32 && r) return launch_conv<T, 3, 64, 32, true>(L, cu, s);
  if (k == 3 && ci == 32 && co == 64 && r) return launch_conv<T, 3, 32, 64, true>(L, cu, s);
  if (k == 3 && ci == 32 && co == 32) {
    return r ? launch_conv<T, 3, 32, 32, true>(L, cu, s) : launch_conv<T, 3, 32, 32, false>(L, cu, s);
  }
  // Unet
  if (k == 3 && ci == 2 && co == 16 && r) return launch_conv<T, 3, 2, 16, true>(L, cu, s);
  if (k == 3 && ci == 16 && co == 16 && r) return launch_conv<T, 3, 16, 16, true>(L, cu, s);
  if (k == 3 && ci == 16 && co == 64 && r) return launch_conv<T, 3, 16, 64, true>(L, cu, s);
  if (k == 3 && ci == 128 && co == 64 && r) return launch_conv<T, 3, 128, 64, true>(L, cu, s);
  if (k == 3 && ci == 80 && co == 16 && r) return launch_conv<T, 3, 80, 16, true>(L, cu, s);
  if (k == 3 && ci == 32 && co == 16 && r) return launch_conv<T, 3, 32, 16, true>(L, cu, s);
  return hipErrorInvalidValue;
}

// Offsets of every layer's parameters and weight image; writes the images.
struct PnWeights {
  PnLayer layer[kUnetLayers];
  size_t poff[kUnetLayers], ioff[kUnetLayers];
  int n;
};

template <typename T>
static hipError_t pn_weights(const NetShape& net, const float* params, T* img, PnWeights& P,
                             hipStream_t s) {
  constexpr int ELT = sizeof(T);
  P.n = all_layers(net.arch, P.layer);
  PnImgLaunch D{};
  size_t p = 0, im = 0;
  for (int i = 0; i < P.n; ++i) {
    const PnLayer& l = P.layer[i];
    P.poff[i] = p;
    P.ioff[i] = im;
    if (l.ks > 1) {
      D.src[D.n] = p;
      D.dst[D.n] = im;
      D.ks[D.n] = l.ks;
      D.cin[D.n] = l.cin;
      D.cout[D.n] = l.cout;
      D.cc[D.n] = conv_cc(ELT, l.ks, l.cin);
      D.wstr[D.n] = conv_wstr(ELT, l.ks, D.cc[D.n]);
      D.e0[D.n] = im;
      im += wimg_elems(l, ELT);
      ++D.n;
    }
    p += (size_t)l.ks * l.ks * l.cin * l.cout + l.cout;
  }
  D.e0[D.n] = im;
  if (im * ELT > pn_weight_image_bytes(net)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((pn_wimg<T>), dim3((unsigned)((im + 255) / 256)), dim3(256), 0, s, D, params, img);
  return hipGetLastError();
}

// One k > 1 layer over an H x W map: NHWC input `src`, output `dst` with
// `ostr` elements per pixel.
template <typename T>
static hipError_t pn_layer(const Device& dev, const PnWeights& P, int i, const float* params,
                           const T* img, const T* src, T* dst, int ostr, int H, int W, hipStream_t s) {
  const PnLayer& l = P.layer[i];
  ConvLaunch L{};
  L.nscales = 1;
  ScaleDesc& S = L.sc[0];
  S.in = src;
  S.out = dst;
  S.wimg = img + P.ioff[i];
  S.b = params + P.poff[i] + (size_t)l.ks * l.ks * l.cin * l.cout;
  S.H = H;
  S.W = W;
  S.tiles_x = (W + TW - 1) / TW;
  S.tile0 = 0;
  S.ostr = ostr;
  L.total_tiles = S.tiles_x * ((H + TH - 1) / TH);
  return pn_conv<T>(l, L, dev.cu, s);
}

template <typename T>
static hipError_t pn_head_launch(const PnWeights& P, int i, const float* params, const T* act,
                                 int npx, float* y, int last, double dx, const Ws& w, hipStream_t s) {
  const float* hw = params + P.poff[i];
  const float dx2 = (float)(dx * dx);
  const int C = P.layer[i].cin;
  const dim3 grid((npx + 255) / 256);
  if (C == 64)
    hipLaunchKernelGGL((pn_head<T, 64>), grid, dim3(256), 0, s, npx, act, hw, y, last, dx2, w.cell, w.phi, w.sc);
  else if (C == 32)
    hipLaunchKernelGGL((pn_head<T, 32>), grid, dim3(256), 0, s, npx, act, hw, y, last, dx2, w.cell, w.phi, w.sc);
  else if (C == 16)
    hipLaunchKernelGGL((pn_head<T, 16>), grid, dim3(256), 0, s, npx, act, hw, y, last, dx2, w.cell, w.phi, w.sc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
static hipError_t run_pn_t(const Device& dev, const NetShape& net, const WsLayout& Ly, int nx,
                           int ny, double dx, const float* params, const Ws& w, hipStream_t s) {
  T* img = reinterpret_cast<T*>(w.cnn_w);
  PnWeights P;
  hipError_t err = pn_weights<T>(net, params, img, P, s);
  if (err != hipSuccess) return err;
  T* in = reinterpret_cast<T*>(w.cnn_in);
  T* bufs[2] = {reinterpret_cast<T*>(w.cnn_act0), reinterpret_cast<T*>(w.cnn_act1)};
  // with net.train every branch input and layer output goes to its own
  // buffer of the saved activations (cascade.h) for the backward pass
  const bool train = net.train && w.cnn_save;
  const PnSave SV = pn_save_layout(net.arch, nx, ny);
  T* save = reinterpret_cast<T*>(w.cnn_save);
  const float* yc = nullptr;
  int Hc = 0, Wc = 0, li = 0;
  for (int b = 0; b < 3; ++b) {
    const int k = 2 - b;  // scale index, 0 = finest
    const int H = Ly.sc_h[k], W = Ly.sc_w[k], f = 1 << k;
    const int npx = H * W;
    PnLayer L[kPnMaxLayers];
    const int nl = pn_branch(net.arch, b, L);
    T* bin = train ? save + SV.in[b] : in;
    hipLaunchKernelGGL((pn_input<T>), dim3((npx + 255) / 256), dim3(256), 0, s, H, W, f, nx, w.d,
                       w.cell, w.sc, yc, Hc, Wc, bin);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const T* src = bin;
    int used = 0;
    for (int i = 0; i + 1 < nl; ++i, ++li) {
      T* dst = train ? save + SV.out[b][i] : bufs[used];
      used ^= 1;
      err = pn_layer<T>(dev, P, li, params, img, src, dst, P.layer[li].cout, H, W, s);
      if (err != hipSuccess) return err;
      src = dst;
    }
    float* y = w.cnn_y + Ly.sc_off_px[k];
    err = pn_head_launch<T>(P, li, params, src, npx, y, b == 2 ? 1 : 0, dx, w, s);
    if (err != hipSuccess) return err;
    ++li;
    yc = y;
    Hc = H;
    Wc = W;
  }
  return hipSuccess;
}

// ---- Unet pieces ----------------------------------------------------------
// 2x2 max pooling of the first C channels of a map with `istr` elements per
// pixel into a contiguous (H/2, W/2, C) map.
template <typename T>
__global__ __launch_bounds__(256) void unet_pool(int Ho, int Wo, int C, const T* __restrict__ in,
                                                 int istr, T* __restrict__ out) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)Ho * Wo * C) return;
  const int c = (int)(gid % C);
  const size_t px = gid / C;
  const int X = (int)(px % Wo), Y = (int)(px / Wo);
  const int Wi = 2 * Wo;
  const T* a = in + ((size_t)(2 * Y) * Wi + 2 * X) * istr + c;
  const float m = fmaxf(fmaxf(St<T>::to_f(a[0]), St<T>::to_f(a[istr])),
                        fmaxf(St<T>::to_f(a[(size_t)Wi * istr]), St<T>::to_f(a[(size_t)Wi * istr + istr])));
  out[gid] = St<T>::from(m);
}

// Bilinear x2 (half-pixel centres, edge clamp) of a contiguous (Hc, Wc, C)
// map into channels [0, C) of a map with `ostr` elements per pixel.
template <typename T>
__global__ __launch_bounds__(256) void unet_up2(int Hc, int Wc, int C, const T* __restrict__ in,
                                                T* __restrict__ out, int ostr) {
  const int H = 2 * Hc, W = 2 * Wc;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)H * W * C) return;
  const int c = (int)(gid % C);
  const size_t px = gid / C;
  const int X = (int)(px % W), Y = (int)(px / W);
  const float cy = fminf(fmaxf(0.5f * (float)Y - 0.25f, 0.f), (float)(Hc - 1));
  const float cx = fminf(fmaxf(0.5f * (float)X - 0.25f, 0.f), (float)(Wc - 1));
  const int y0 = min((int)floorf(cy), max(Hc - 2, 0));
  const int x0 = min((int)floorf(cx), max(Wc - 2, 0));
  const float wy = cy - (float)y0, wx = cx - (float)x0;
  const int y1 = min(y0 + 1, Hc - 1), x1 = min(x0 + 1, Wc - 1);
  const float a = St<T>::to_f(in[((size_t)y0 * Wc + x0) * C + c]);
  const float b = St<T>::to_f(in[((size_t)y0 * Wc + x1) * C + c]);
  const float e = St<T>::to_f(in[((size_t)y1 * Wc + x0) * C + c]);
  const float f = St<T>::to_f(in[((size_t)y1 * Wc + x1) * C + c]);
  out[px * ostr + c] =
      St<T>::from((1.f - wy) * ((1.f - wx) * a + wx * b) + wy * ((1.f - wx) * e + wx * f));
}

// With net.train every layer output goes to its own buffer of the saved
// activations (unet.h) instead of the two alternating maps, so that the
// backward pass finds them.
template <typename T>
static hipError_t run_unet_t(const Device& dev, const NetShape& net, int nx, int ny, double dx,
                             const float* params, const Ws& w, hipStream_t s) {
  T* img = reinterpret_cast<T*>(w.cnn_w);
  PnWeights P;
  hipError_t err = pn_weights<T>(net, params, img, P, s);
  if (err != hipSuccess) return err;
  T* in = reinterpret_cast<T*>(w.cnn_in);
  T* cat = reinterpret_cast<T*>(w.cnn_cat);
  const bool train = net.train && w.cnn_save;
  const UnetSave SV = unet_save_layout(nx, ny);
  T* save = reinterpret_cast<T*>(w.cnn_save);
  T* act0 = reinterpret_cast<T*>(w.cnn_act0);
  T* act1 = reinterpret_cast<T*>(w.cnn_act1);
  auto c1 = [&](int l) { return train ? save + SV.c1[l] : act0; };
  auto c2_bottom = [&]() { return train ? save + SV.c2_bottom : act1; };
  auto pooled = [&](int l) { return train ? save + SV.pool[l] : act1; };
  auto d1 = [&](int l) { return train ? save + SV.d1[l] : act0; };
  auto d2 = [&](int l) { return train ? save + SV.d2[l] : act1; };
  hipLaunchKernelGGL((pn_input<T>), dim3((nx * ny + 255) / 256), dim3(256), 0, s, ny, nx, 1, nx,
                     w.d, w.cell, w.sc, (const float*)nullptr, 0, 0, in);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  int li = 0;
  const T* src = in;
  // encoder: the second layer of scale l writes the skip channels of the
  // scale's concatenation buffer (the bottom scale its own map)
  for (int l = 0; l < kUnetLevels; ++l) {
    const int H = ny >> l, W = nx >> l;
    err = pn_layer<T>(dev, P, li++, params, img, src, c1(l), kUnetW[l], H, W, s);
    if (err != hipSuccess) return err;
    if (l + 1 < kUnetLevels) {
      T* cl = cat + unet_cat_offset(nx, ny, l);
      const int cs = kUnetW[l] + kUnetW[l + 1];
      err = pn_layer<T>(dev, P, li++, params, img, c1(l), cl, cs, H, W, s);
      if (err != hipSuccess) return err;
      const size_t nout = (size_t)(H / 2) * (W / 2) * kUnetW[l];
      hipLaunchKernelGGL((unet_pool<T>), dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, H / 2,
                         W / 2, kUnetW[l], cl, cs, pooled(l));
      err = hipGetLastError();
      if (err != hipSuccess) return err;
      src = pooled(l);
    } else {
      err = pn_layer<T>(dev, P, li++, params, img, c1(l), c2_bottom(), kUnetW[l], H, W, s);
      if (err != hipSuccess) return err;
      src = c2_bottom();
    }
  }
  // decoder: upsample the coarser output into the upper channels of the
  // concatenation buffer, then two layers
  for (int l = kUnetLevels - 2; l >= 0; --l) {
    const int H = ny >> l, W = nx >> l;
    T* cl = cat + unet_cat_offset(nx, ny, l);
    const int cs = kUnetW[l] + kUnetW[l + 1];
    const size_t nup = (size_t)H * W * kUnetW[l + 1];
    hipLaunchKernelGGL((unet_up2<T>), dim3((unsigned)((nup + 255) / 256)), dim3(256), 0, s, H / 2, W / 2,
                       kUnetW[l + 1], src, cl + kUnetW[l], cs);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    err = pn_layer<T>(dev, P, li++, params, img, cl, d1(l), kUnetW[l], H, W, s);
    if (err != hipSuccess) return err;
    err = pn_layer<T>(dev, P, li++, params, img, d1(l), d2(l), kUnetW[l], H, W, s);
    if (err != hipSuccess) return err;
    src = d2(l);
  }
  return pn_head_launch<T>(P, li, params, src, nx * ny, w.cnn_y, 1, dx, w, s);
}

hipError_t run_papernet(const Device& dev, const NetShape& net, const WsLayout& L, int nx, int ny,
                        double dx, const float* params, const Ws& w, hipStream_t s) {
  if (net.arch == HYP_ARCH_UNET) {
    if (net.precision == HYP_PREC_BF16) return run_unet_t<uint16_t>(dev, net, nx, ny, dx, params, w, s);
    return run_unet_t<float>(dev, net, nx, ny, dx, params, w, s);
  }
  if (net.arch != HYP_ARCH_MULTISCALE && net.arch != HYP_ARCH_SMALLSCALE) return hipErrorInvalidValue;
  if (net.precision == HYP_PREC_BF16) return run_pn_t<uint16_t>(dev, net, L, nx, ny, dx, params, w, s);
  return run_pn_t<float>(dev, net, L, nx, ny, dx, params, w, s);
}

}  // namespace hyp
