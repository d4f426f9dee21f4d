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
// Every k > 1 layer is one launch of conv_mfma (implicit GEMM on MFMA, FP32
// or BF16 storage); the 1x1 output layer and the resampling are small
// elementwise kernels.  The layer weights are re-laid into the LDS image of
// the convolution kernel once per inference, in one launch.
#include <hip/hip_runtime.h>

#include "../../include/hyproj.h"
#include "common.h"
#include "conv_mfma.h"
#include "internal.h"

namespace hyp {

struct PnLayer {
  int ks, cin, cout;
  bool relu;
};

constexpr int kPnMaxLayers = 7;

// Layers of branch b (0 = coarsest); returns the layer count.
static int pn_branch(int arch, int b, PnLayer* out) {
  const int a = arch == HYP_ARCH_MULTISCALE ? 64 : 32;
  const int mid = 32;
  if (b == 0) {
    const PnLayer L[5] = {{5, 2, a, true}, {3, a, a, true}, {3, a, a, true}, {3, a, a, false},
                          {1, a, 1, false}};
    for (int i = 0; i < 5; ++i) out[i] = L[i];
    return 5;
  }
  const PnLayer L[7] = {{5, 3, a, true},   {3, a, a, true}, {3, a, mid, true}, {3, mid, a, true},
                        {3, a, a, true},   {3, a, a, false}, {1, a, 1, false}};
  for (int i = 0; i < 7; ++i) out[i] = L[i];
  return 7;
}

int64_t pn_param_count(int arch) {
  int64_t n = 0;
  PnLayer L[kPnMaxLayers];
  for (int b = 0; b < 3; ++b) {
    const int nl = pn_branch(arch, b, L);
    for (int i = 0; i < nl; ++i) n += (int64_t)L[i].ks * L[i].ks * L[i].cin * L[i].cout + L[i].cout;
  }
  return n;
}

size_t pn_weight_image_bytes(const NetShape& net) {
  const int elt = net.precision == HYP_PREC_BF16 ? 2 : 4;
  size_t bytes = 0;
  PnLayer L[kPnMaxLayers];
  for (int b = 0; b < 3; ++b) {
    const int nl = pn_branch(net.arch, b, L);
    for (int i = 0; i < nl; ++i)
      if (L[i].ks > 1) bytes += (size_t)L[i].cout * conv_wstr(elt, L[i].ks, L[i].cin) * elt;
  }
  return bytes;
}

// ---- weight images of every k > 1 layer in one launch -------------------
constexpr int kPnMaxImg = 3 * kPnMaxLayers;
struct PnImgLaunch {
  size_t src[kPnMaxImg];   // float offset of W in the packed parameters
  size_t dst[kPnMaxImg];   // element offset of the image
  size_t e0[kPnMaxImg + 1];
  int ktot[kPnMaxImg], wstr[kPnMaxImg];
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
  const int co = (int)(e / D.wstr[l]), kk = (int)(e % D.wstr[l]);
  const float v = kk < D.ktot[l] ? params[D.src[l] + (size_t)co * D.ktot[l] + kk] : 0.f;
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
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t run_pn_t(const Device& dev, const NetShape& net, const WsLayout& Ly, int nx,
                           int ny, double dx, const float* params, const Ws& w, hipStream_t s) {
  constexpr int ELT = sizeof(T);
  PnLayer layers[3][kPnMaxLayers];
  int nl[3];
  for (int b = 0; b < 3; ++b) nl[b] = pn_branch(net.arch, b, layers[b]);
  // parameter offsets and weight images
  PnImgLaunch D{};
  size_t poff[3][kPnMaxLayers], ioff[3][kPnMaxLayers];
  size_t p = 0, im = 0, e = 0;
  for (int b = 0; b < 3; ++b)
    for (int i = 0; i < nl[b]; ++i) {
      const PnLayer& l = layers[b][i];
      poff[b][i] = p;
      ioff[b][i] = im;
      if (l.ks > 1) {
        const int wstr = conv_wstr(ELT, l.ks, l.cin);
        D.src[D.n] = p;
        D.dst[D.n] = im;
        D.ktot[D.n] = l.ks * l.ks * l.cin;
        D.wstr[D.n] = wstr;
        D.e0[D.n] = e;
        e += (size_t)l.cout * wstr;
        im += (size_t)l.cout * wstr;
        ++D.n;
      }
      p += (size_t)l.ks * l.ks * l.cin * l.cout + l.cout;
    }
  D.e0[D.n] = e;
  if (im * ELT > pn_weight_image_bytes(net)) return hipErrorInvalidValue;
  T* img = reinterpret_cast<T*>(w.cnn_w);
  hipLaunchKernelGGL((pn_wimg<T>), dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, D, params, img);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  T* in = reinterpret_cast<T*>(w.cnn_in);
  T* bufs[2] = {reinterpret_cast<T*>(w.cnn_act0), reinterpret_cast<T*>(w.cnn_act1)};
  const float* yc = nullptr;
  int Hc = 0, Wc = 0;
  for (int b = 0; b < 3; ++b) {
    const int k = 2 - b;  // scale index, 0 = finest
    const int H = Ly.sc_h[k], W = Ly.sc_w[k], f = 1 << k;
    const int npx = H * W;
    hipLaunchKernelGGL((pn_input<T>), dim3((npx + 255) / 256), dim3(256), 0, s, H, W, f, nx, w.d,
                       w.cell, w.sc, yc, Hc, Wc, in);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const T* src = in;
    int used = 0;
    for (int i = 0; i + 1 < nl[b]; ++i) {
      const PnLayer& l = layers[b][i];
      T* dst = bufs[used];
      used ^= 1;
      ConvLaunch L{};
      L.nscales = 1;
      ScaleDesc& S = L.sc[0];
      S.in = src;
      S.out = dst;
      S.wimg = img + ioff[b][i];
      S.b = params + poff[b][i] + (size_t)l.ks * l.ks * l.cin * l.cout;
      S.H = H;
      S.W = W;
      S.tiles_x = (W + TW - 1) / TW;
      S.tile0 = 0;
      L.total_tiles = S.tiles_x * ((H + TH - 1) / TH);
      err = pn_conv<T>(l, L, dev.cu, s);
      if (err != hipSuccess) return err;
      src = dst;
    }
    const PnLayer& h = layers[b][nl[b] - 1];
    float* y = w.cnn_y + Ly.sc_off_px[k];
    const float* hw = params + poff[b][nl[b] - 1];
    const int last = b == 2 ? 1 : 0;
    const float dx2 = (float)(dx * dx);
    if (h.cin == 64)
      hipLaunchKernelGGL((pn_head<T, 64>), dim3((npx + 255) / 256), dim3(256), 0, s, npx, src, hw, y,
                         last, dx2, w.cell, w.phi, w.sc);
    else
      hipLaunchKernelGGL((pn_head<T, 32>), dim3((npx + 255) / 256), dim3(256), 0, s, npx, src, hw, y,
                         last, dx2, w.cell, w.phi, w.sc);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    yc = y;
    Hc = H;
    Wc = W;
  }
  return hipSuccess;
}

hipError_t run_papernet(const Device& dev, const NetShape& net, const WsLayout& L, int nx, int ny,
                        double dx, const float* params, const Ws& w, hipStream_t s) {
  if (net.arch != HYP_ARCH_MULTISCALE && net.arch != HYP_ARCH_SMALLSCALE) return hipErrorInvalidValue;
  if (net.precision == HYP_PREC_BF16) return run_pn_t<uint16_t>(dev, net, L, nx, ny, dx, params, w, s);
  return run_pn_t<float>(dev, net, L, nx, ny, dx, params, w, s);
}

}  // namespace hyp
