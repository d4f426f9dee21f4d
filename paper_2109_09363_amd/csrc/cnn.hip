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

#include <vector>

#include "../../include/hyproj.h"
#include "batch.h"
#include "common.h"
#include "conv_mfma.h"
#include "internal.h"

namespace hyp {

// ---- pyramid input: level k pixel = mean of the 2x2 level k-1 pixels it ---
// covers (level 0 = [d/s, solid]); a work-group reduces a 32x32 region of
// level 0 in LDS level by level (FP32), storing every level NHWC with 2
// channels in the storage type.  Levels never straddle regions: the grid
// sides are multiples of 2^(S-1) <= 16.
struct PyrLaunch {
  void* out[kMaxScales];
  int H[kMaxScales], W[kMaxScales];
  size_t px0[kMaxScales];
  int nscales;
  size_t total_px;
  int nx, rtx;  // rtx: 32x32 regions per row
};

template <typename T>
__device__ __forceinline__ void cnn_input_body(const PyrLaunch& P, int region,
                                               const float* __restrict__ d,
                                               const uint8_t* __restrict__ cell, const Scalars* sc,
                                               float (*lv)[32][33]) {
  const int x0 = (region % P.rtx) * 32, y0 = (region / P.rtx) * 32;
  const double s = sc->s;
  const float inv_s = s > 0.0 ? (float)(1.0 / s) : 0.f;
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int ly = e >> 5, lx = e & 31, gx = x0 + lx, gy = y0 + ly;
    float vd = 0.f, vs = 0.f;
    if (gx < P.W[0] && gy < P.H[0]) {
      const int c = gy * P.nx + gx;
      const bool solid = cell[c] & C_SOLID;
      vd = solid ? 0.f : d[c] * inv_s;
      vs = solid ? 1.f : 0.f;
      T* o = reinterpret_cast<T*>(P.out[0]) + (size_t)c * 2;
      o[0] = St<T>::from(vd);
      o[1] = St<T>::from(vs);
    }
    lv[0][ly][lx] = vd;
    lv[1][ly][lx] = vs;
  }
  for (int k = 1; k < P.nscales; ++k) {
    const int m = 32 >> k;
    const int t = threadIdx.x, ly = t / m, lx = t % m;
    const bool act = t < m * m;
    float a = 0.f, b = 0.f;
    __syncthreads();
    if (act) {
      a = 0.25f * ((lv[0][2 * ly][2 * lx] + lv[0][2 * ly][2 * lx + 1]) +
                   (lv[0][2 * ly + 1][2 * lx] + lv[0][2 * ly + 1][2 * lx + 1]));
      b = 0.25f * ((lv[1][2 * ly][2 * lx] + lv[1][2 * ly][2 * lx + 1]) +
                   (lv[1][2 * ly + 1][2 * lx] + lv[1][2 * ly + 1][2 * lx + 1]));
    }
    __syncthreads();
    if (act) {
      lv[0][ly][lx] = a;
      lv[1][ly][lx] = b;
      const int gx = (x0 >> k) + lx, gy = (y0 >> k) + ly;
      if (gx < P.W[k] && gy < P.H[k]) {
        T* o = reinterpret_cast<T*>(P.out[k]) + ((size_t)gy * P.W[k] + gx) * 2;
        o[0] = St<T>::from(a);
        o[1] = St<T>::from(b);
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void cnn_input(PyrLaunch P, const float* __restrict__ d,
                                                 const uint8_t* __restrict__ cell,
                                                 const Scalars* sc) {
  __shared__ float lv[2][32][33];  // [channel][y][x] of the current level
  cnn_input_body<T>(P, blockIdx.x, d, cell, sc, lv);
}

// ---- t_k = y_k + up2(t_{k+1}); at k = 0 also phi0 = dx^2 s t on fluid -----
__device__ __forceinline__ void upsum_body(int gid, int H, int W, const float* __restrict__ yk,
                                           const float* __restrict__ tc, int Hc, int Wc,
                                           float* __restrict__ tk, int last, float dx2,
                                           const uint8_t* __restrict__ cell,
                                           float* __restrict__ phi, const Scalars* sc) {
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

__global__ __launch_bounds__(256) void cnn_upsum(int H, int W, const float* __restrict__ yk,
                                                 const float* __restrict__ tc, int Hc, int Wc,
                                                 float* __restrict__ tk, int last, float dx2,
                                                 const uint8_t* __restrict__ cell,
                                                 float* __restrict__ phi, const Scalars* sc) {
  upsum_body(blockIdx.x * blockDim.x + threadIdx.x, H, W, yk, tc, Hc, Wc, tk, last, dx2, cell, phi,
             sc);
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
  P.rtx = (nx + 31) / 32;
  const int nreg = P.rtx * ((ny + 31) / 32);
  hipLaunchKernelGGL(cnn_input<T>, dim3(nreg), dim3(256), 0, s, P, w.d, w.cell, w.sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  using WI = WImg<T, C>;
  T* img = reinterpret_cast<T*>(w.cnn_w);
  const size_t nimg = WI::PER_SCALE * S;
  hipLaunchKernelGGL((cnn_wimg<T, C>), dim3((unsigned)((nimg + 255) / 256)), dim3(256), 0, s, params,
                     per_scale, S, img);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // four 3x3 layers, all scales per launch; the last one also forms the 1x1
  // head y_k in its epilogue (and stores its activations only for training)
  const T* src = in;
  T* bufs[2] = {a0, a1};
  T* save = reinterpret_cast<T*>(w.cnn_save);
  const size_t hoff = (size_t)C * 18 + C + 3 * ((size_t)C * 9 * C + C);
  for (int l = 0; l < 4; ++l) {
    T* dst = net.train ? save + (size_t)l * Ly.total_px * C : bufs[l & 1];
    ConvLaunch L{};
    L.nscales = S;
    L.skip_store = (l == 3 && !net.train) ? 1 : 0;
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
      D.hw = params + k * per_scale + hoff;
      D.y = w.cnn_y + Ly.sc_off_px[k];
      tiles += D.tiles_x * ((D.H + TH - 1) / TH);
    }
    L.total_tiles = tiles;
    // launch on the caller's stream
    if (l == 0)
      e = launch_conv<T, 3, 2, C, true>(L, dev.cu, s);
    else if (l < 3)
      e = launch_conv<T, 3, C, C, true>(L, dev.cu, s);
    else
      e = launch_conv<T, 3, C, C, true, true>(L, dev.cu, s);
    if (e != hipSuccess) return e;
    src = dst;
  }
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

// ---------------------------------------------------------------------------
// A batch of grids (batch.h) through the same network: one launch per phase
// over every instance.  The pyramid input and the upsample-sum find their
// instance in the batch's range tables; the four convolution launches walk
// descriptor tables of (scale, instance) pairs in device memory, ordered
// scale by scale so that consecutive tiles share the weights held in LDS;
// one weight image (in the first instance's workspace) serves every
// instance.  Device layout of the tables: 4 x ndesc ScaleDesc, then one
// PyrLaunch per instance.
// ---------------------------------------------------------------------------
size_t cnn_batch_bytes(const NetShape& net, int n) {
  const size_t ndesc = (size_t)n * net.scales;
  return 4 * ndesc * sizeof(ScaleDesc) + (size_t)n * sizeof(PyrLaunch);
}

template <typename T, int C>
static void cnn_batch_fill(const NetShape& net, int n, const WsLayout* Ly, const Ws* ws,
                           const float* params, ScaleDesc* desc, PyrLaunch* pyr, int* tiles) {
  const int S = net.scales;
  const size_t per_scale = (size_t)C * 18 + C + 3 * ((size_t)C * 9 * C + C) + C + 1;
  const size_t hoff = (size_t)C * 18 + C + 3 * ((size_t)C * 9 * C + C);
  using WI = WImg<T, C>;
  const T* img = reinterpret_cast<const T*>(ws[0].cnn_w);
  for (int l = 0; l < 4; ++l) {
    const int cin = l == 0 ? 2 : C;
    const size_t woff = l == 0 ? 0 : (size_t)C * 18 + C + (size_t)(l - 1) * ((size_t)C * 9 * C + C);
    int t = 0;
    ScaleDesc* out = desc + (size_t)l * n * S;
    for (int k = 0; k < S; ++k) {
      for (int i = 0; i < n; ++i) {
        // layer l reads the previous layer's output (act0/act1 alternate)
        const T* in = reinterpret_cast<const T*>(l == 0 ? ws[i].cnn_in
                                                        : (l & 1 ? ws[i].cnn_act0 : ws[i].cnn_act1));
        T* dst = reinterpret_cast<T*>(l & 1 ? ws[i].cnn_act1 : ws[i].cnn_act0);
        ScaleDesc& D = out[(size_t)k * n + i];
        D.in = in + Ly[i].sc_off_px[k] * cin;
        D.out = dst + Ly[i].sc_off_px[k] * C;
        D.wimg = img + k * WI::PER_SCALE + (l == 0 ? 0 : WI::L0 + (size_t)(l - 1) * WI::L1);
        D.b = params + k * per_scale + woff + (size_t)C * 9 * cin;
        D.H = Ly[i].sc_h[k];
        D.W = Ly[i].sc_w[k];
        D.tiles_x = (D.W + TW - 1) / TW;
        D.tile0 = t;
        D.ostr = C;
        D.hw = params + k * per_scale + hoff;
        D.y = ws[i].cnn_y + Ly[i].sc_off_px[k];
        t += D.tiles_x * ((D.H + TH - 1) / TH);
      }
    }
    tiles[l] = t;
  }
  for (int i = 0; i < n; ++i) {
    PyrLaunch& P = pyr[i];
    P = PyrLaunch{};
    P.nscales = S;
    P.total_px = Ly[i].total_px;
    P.nx = Ly[i].sc_w[0];
    for (int k = 0; k < S; ++k) {
      P.out[k] = reinterpret_cast<T*>(ws[i].cnn_in) + Ly[i].sc_off_px[k] * 2;
      P.H[k] = Ly[i].sc_h[k];
      P.W[k] = Ly[i].sc_w[k];
      P.px0[k] = Ly[i].sc_off_px[k];
    }
    P.rtx = (P.nx + 31) / 32;
  }
}

// Fills the tables on the host and uploads them (synchronous, once per batch).
hipError_t cnn_batch_setup(const NetShape& net, int n, const WsLayout* Ly, const Ws* ws,
                           const float* params, void* dev_tables, int* tiles) {
  if (net.arch != HYP_ARCH_PARALLEL || net.train) return hipErrorInvalidValue;
  const size_t ndesc = (size_t)n * net.scales;
  std::vector<ScaleDesc> desc(4 * ndesc);
  std::vector<PyrLaunch> pyr(n);
  if (net.precision == HYP_PREC_BF16) {
    if (net.channels == 32) cnn_batch_fill<uint16_t, 32>(net, n, Ly, ws, params, desc.data(), pyr.data(), tiles);
    else if (net.channels == 64) cnn_batch_fill<uint16_t, 64>(net, n, Ly, ws, params, desc.data(), pyr.data(), tiles);
    else return hipErrorInvalidValue;
  } else {
    if (net.channels == 16) cnn_batch_fill<float, 16>(net, n, Ly, ws, params, desc.data(), pyr.data(), tiles);
    else if (net.channels == 32) cnn_batch_fill<float, 32>(net, n, Ly, ws, params, desc.data(), pyr.data(), tiles);
    else if (net.channels == 64) cnn_batch_fill<float, 64>(net, n, Ly, ws, params, desc.data(), pyr.data(), tiles);
    else return hipErrorInvalidValue;
  }
  char* d = reinterpret_cast<char*>(dev_tables);
  hipError_t e = hipMemcpy(d, desc.data(), desc.size() * sizeof(ScaleDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(d + desc.size() * sizeof(ScaleDesc), pyr.data(), pyr.size() * sizeof(PyrLaunch),
                  hipMemcpyHostToDevice);
  return e;
}

template <typename T>
__global__ __launch_bounds__(256) void cnn_input_batch(const BInst* __restrict__ I,
                                                       const PyrLaunch* __restrict__ pyr,
                                                       const int* first, int n) {
  __shared__ float lv[2][32][33];
  const int i = batch_find(first, n, blockIdx.x);
  const BInst& B = I[i];
  cnn_input_body<T>(pyr[i], blockIdx.x - first[i], B.w.d, B.w.cell, B.w.sc, lv);
}

__global__ __launch_bounds__(256) void upsum_batch(const BInst* __restrict__ I, const int* first,
                                                   int n, int k) {
  const int i = batch_find(first, n, blockIdx.x);
  const BInst& B = I[i];
  const int H = B.sc_h[k], W = B.sc_w[k];
  const bool top = k + 1 >= B.S;
  upsum_body((blockIdx.x - first[i]) * blockDim.x + threadIdx.x, H, W, B.w.cnn_y + B.sc_off_px[k],
             top ? nullptr : B.w.cnn_t + B.sc_off_px[k + 1], top ? 0 : B.sc_h[k + 1],
             top ? 0 : B.sc_w[k + 1], B.w.cnn_t + B.sc_off_px[k], k == 0 ? 1 : 0,
             (float)(B.dx * B.dx), B.w.cell, B.w.phi, B.w.sc);
}

template <typename T, int C>
static hipError_t run_cnn_batch_t(const Device& dev, const NetShape& net, const BInst* I,
                                  const BatchRanges& R, const void* tables, const int* tiles,
                                  const Ws& w0, const float* params, hipStream_t s) {
  const int S = net.scales, n = R.n;
  const size_t ndesc = (size_t)n * S;
  const ScaleDesc* desc = reinterpret_cast<const ScaleDesc*>(tables);
  const PyrLaunch* pyr = reinterpret_cast<const PyrLaunch*>(desc + 4 * ndesc);
  if (R.total[RK_REG] > 0)
    hipLaunchKernelGGL(cnn_input_batch<T>, dim3(R.total[RK_REG]), dim3(256), 0, s, I, pyr,
                       R.of(RK_REG), n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  using WI = WImg<T, C>;
  const size_t per_scale = (size_t)C * 18 + C + 3 * ((size_t)C * 9 * C + C) + C + 1;
  const size_t nimg = WI::PER_SCALE * S;
  hipLaunchKernelGGL((cnn_wimg<T, C>), dim3((unsigned)((nimg + 255) / 256)), dim3(256), 0, s, params,
                     per_scale, S, reinterpret_cast<T*>(w0.cnn_w));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int l = 0; l < 4; ++l) {
    ConvLaunch L{};
    L.table = desc + (size_t)l * ndesc;
    L.ndesc = (int)ndesc;
    L.total_tiles = tiles[l];
    L.skip_store = l == 3 ? 1 : 0;
    if (l == 0) e = launch_conv<T, 3, 2, C, true>(L, dev.cu, s);
    else if (l < 3) e = launch_conv<T, 3, C, C, true>(L, dev.cu, s);
    else e = launch_conv<T, 3, C, C, true, true>(L, dev.cu, s);
    if (e != hipSuccess) return e;
  }
  for (int k = S - 1; k >= 0; --k) {
    const int nb = R.total[RK_LVL0 + k];
    if (nb > 0)
      hipLaunchKernelGGL(upsum_batch, dim3(nb), dim3(256), 0, s, I, R.of(RK_LVL0 + k), n, k);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_cnn_batch(const Device& dev, const NetShape& net, const BInst* I,
                         const BatchRanges& R, const void* tables, const int* tiles, const Ws& w0,
                         const float* params, hipStream_t s) {
  if (net.arch != HYP_ARCH_PARALLEL) return hipErrorInvalidValue;
  if (net.precision == HYP_PREC_BF16) {
    switch (net.channels) {
      case 32: return run_cnn_batch_t<uint16_t, 32>(dev, net, I, R, tables, tiles, w0, params, s);
      case 64: return run_cnn_batch_t<uint16_t, 64>(dev, net, I, R, tables, tiles, w0, params, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (net.channels) {
    case 16: return run_cnn_batch_t<float, 16>(dev, net, I, R, tables, tiles, w0, params, s);
    case 32: return run_cnn_batch_t<float, 32>(dev, net, I, R, tables, tiles, w0, params, s);
    case 64: return run_cnn_batch_t<float, 64>(dev, net, I, R, tables, tiles, w0, params, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hyp
