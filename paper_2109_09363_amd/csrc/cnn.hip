// Multi-scale CNN initial guess of the pressure (Sec. 3.1: several
// resolutions of the same input, replication padding, ReLU hidden layers,
// bilinear down/up sampling, linear output):
//   x   = [d / s, solid], s = sqrt(mean_F d^2)
//   x_k = 2x2 mean pyramid, k = 0..S-1
//   y_k = conv1x1(relu(conv3x3(... 4 layers ...)))   per scale, own weights
//   t   = y_{S-1};  t = y_k + up2(t) for k = S-2..0;   phi0 = dx^2 s t (fluid)
//
// The 3x3 convolutions are implicit GEMMs on MFMA: D[cout][px] =
// sum_k W[cout][k] X[k][px] with k = (tap, cin).  One template serves both
// precisions: FP32 storage with v_mfma_f32_16x16x4f32, and BF16 storage with
// the gfx950 v_mfma_f32_16x16x32_bf16 (FP32 accumulation).  Activations are
// NHWC so a lane's K-fragment is 16 contiguous bytes in LDS.  All scales of
// a layer run in one launch over a concatenated tile list.
#include <hip/hip_runtime.h>

#include "../../include/hyproj.h"
#include "common.h"
#include "internal.h"

namespace hyp {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename T> struct St;
template <> struct St<float> {
  static __device__ __forceinline__ float from(float f) { return f; }
  static __device__ __forceinline__ float to_f(float x) { return x; }
};
template <> struct St<uint16_t> {
  static __device__ __forceinline__ uint16_t from(float f) { return f2bf(f); }
  static __device__ __forceinline__ float to_f(uint16_t x) { return bf2f(x); }
};

constexpr int kMaxScales = 5;
constexpr int TW = 16;        // tile width (pixels)
constexpr int TH = 16;        // tile height: 4 waves x 4 rows
constexpr int EW = TW + 2, EH = TH + 2;

struct ScaleDesc {
  const void* in;     // NHWC input activations (storage type)
  void* out;          // NHWC output activations
  const void* wimg;   // weights as the LDS image: [Cout][WSTR] storage type, zero-padded K
  const float* b;     // FP32 bias [Cout]
  int H, W;
  int tiles_x, tile0; // tile columns, first global tile index of this scale
};

struct ConvLaunch {
  ScaleDesc sc[kMaxScales];
  int nscales, total_tiles, tiles_per_wg;
};

template <typename T, int CIN, int COUT>
struct ConvGeom {
  static constexpr int ELT = sizeof(T);
  static constexpr int KSTEP = (ELT == 4) ? 16 : 32;          // K per fragment step
  static constexpr int KTOT = 9 * CIN;
  static constexpr int KPAD = ((KTOT + KSTEP - 1) / KSTEP) * KSTEP;
  static constexpr int WSTR = KPAD + 16 / ELT;                // LDS weight row stride (elts)
  static constexpr int PSTR = (CIN == 2 ? 2 : CIN + 16 / ELT); // LDS pixel stride (elts)
  static constexpr size_t TILE_LDS = (size_t)EH * EW * PSTR * ELT;
  // output channels per pass: all of them unless their weights and the
  // input tile overflow the 160 KB of LDS (FP32 64 -> 64: 16 per pass)
  static constexpr int CT = ((size_t)COUT * WSTR * ELT + TILE_LDS <= 160 * 1024) ? COUT : 16;
  static constexpr int PASSES = COUT / CT;
  static constexpr int MB = CT / 16;                          // cout blocks per pass
  static constexpr size_t LDS = (size_t)CT * WSTR * ELT + TILE_LDS;
};

// Fragment loads.  FP32: a lane holds 4 consecutive K values (one float4) and
// feeds them to 4 MFMAs; BF16: 8 consecutive K values (16 bytes) for one MFMA.
template <typename T, int CIN, int COUT>
__device__ __forceinline__ void conv_tile(const T* __restrict__ wl, const T* __restrict__ xl,
                                          floatx4 (&acc)[ConvGeom<T, CIN, COUT>::MB][4],
                                          int wave, int lane) {
  using Gm = ConvGeom<T, CIN, COUT>;
  const int col = lane & 15, g = lane >> 4;
  if constexpr (CIN == 2) {
    // K = 18 (tap, cin) gathered per element, zero-padded to KPAD
    for (int k0 = 0; k0 < Gm::KPAD; k0 += Gm::KSTEP) {
      constexpr int PER = (sizeof(T) == 4) ? 4 : 8;
      T bv[4][PER];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int row = wave * 4 + nb;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          const int k = k0 + g * PER + e;
          T val = St<T>::from(0.f);
          if (k < 18) {
            const int tap = k >> 1, ci = k & 1;
            val = xl[((row + tap / 3) * EW + col + tap % 3) * Gm::PSTR + ci];
          }
          bv[nb][e] = val;
        }
      }
#pragma unroll
      for (int mb = 0; mb < Gm::MB; ++mb) {
        const T* wrow = wl + (mb * 16 + col) * Gm::WSTR + k0 + g * PER;
        if constexpr (sizeof(T) == 4) {
          const float4 a = *reinterpret_cast<const float4*>(wrow);
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bv[nb][0], acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bv[nb][1], acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, bv[nb][2], acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, bv[nb][3], acc[mb][nb], 0, 0, 0);
          }
        } else {
          const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(wrow));
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
            uint4 raw;
            uint16_t* r16 = reinterpret_cast<uint16_t*>(&raw);
#pragma unroll
            for (int e = 0; e < 8; ++e) r16[e] = bv[nb][e];
            const bf16x8 b = __builtin_bit_cast(bf16x8, raw);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mb][nb], 0, 0, 0);
          }
        }
      }
    }
  } else {
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap % 3;
#pragma unroll
      for (int c0 = 0; c0 < CIN; c0 += Gm::KSTEP) {
        const int k0 = tap * CIN + c0;
        if constexpr (sizeof(T) == 4) {
          float4 bv[4];
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
            const int row = wave * 4 + nb;
            bv[nb] = *reinterpret_cast<const float4*>(
                xl + ((row + ky) * EW + col + kx) * Gm::PSTR + c0 + g * 4);
          }
#pragma unroll
          for (int mb = 0; mb < Gm::MB; ++mb) {
            const float4 a = *reinterpret_cast<const float4*>(wl + (mb * 16 + col) * Gm::WSTR + k0 + g * 4);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bv[nb].x, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bv[nb].y, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, bv[nb].z, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, bv[nb].w, acc[mb][nb], 0, 0, 0);
            }
          }
        } else {
          bf16x8 bv[4];
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
            const int row = wave * 4 + nb;
            bv[nb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                xl + ((row + ky) * EW + col + kx) * Gm::PSTR + c0 + g * 8));
          }
#pragma unroll
          for (int mb = 0; mb < Gm::MB; ++mb) {
            const bf16x8 a = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4*>(wl + (mb * 16 + col) * Gm::WSTR + k0 + g * 8));
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv[nb], acc[mb][nb], 0, 0, 0);
          }
        }
      }
    }
  }
}

template <typename T, int CIN, int COUT>
__global__ __launch_bounds__(256) void conv3x3_relu(ConvLaunch L) {
  using Gm = ConvGeom<T, CIN, COUT>;
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  T* wl = reinterpret_cast<T*>(lds_raw);
  T* xl = wl + Gm::CT * Gm::WSTR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t_begin = blockIdx.x * L.tiles_per_wg;
  const int t_end = min(t_begin + L.tiles_per_wg, L.total_tiles);
  int cur = -1;
  // copy cout rows [co0, co0 + CT) of the layer's weight image into LDS with
  // 16-byte loads, several in flight per thread
  auto load_weights = [&](const void* img, int co0) {
    __syncthreads();
    constexpr int N16 = Gm::CT * Gm::WSTR * Gm::ELT / 16;
    const uint4* src = reinterpret_cast<const uint4*>(img) + (size_t)co0 * Gm::WSTR * Gm::ELT / 16;
    uint4* dstl = reinterpret_cast<uint4*>(wl);
#pragma unroll 8
    for (int e = threadIdx.x; e < N16; e += 256) dstl[e] = src[e];
  };
  for (int t = t_begin; t < t_end; ++t) {
    int k = 0;
    while (k + 1 < L.nscales && t >= L.sc[k + 1].tile0) ++k;
    const ScaleDesc& S = L.sc[k];
    if (Gm::PASSES == 1 && k != cur) {
      load_weights(S.wimg, 0);
      cur = k;
    }
    const int lt = t - S.tile0;
    const int x0 = (lt % S.tiles_x) * TW, y0 = (lt / S.tiles_x) * TH;
    const T* in = reinterpret_cast<const T*>(S.in);
    // input tile with a one-pixel replicated border (coordinates clamped)
    if constexpr (CIN == 2) {
      for (int e = threadIdx.x; e < EH * EW; e += blockDim.x) {
        const int gy = min(max(y0 - 1 + e / EW, 0), S.H - 1);
        const int gx = min(max(x0 - 1 + e % EW, 0), S.W - 1);
        const T* src = in + ((size_t)gy * S.W + gx) * 2;
        xl[e * Gm::PSTR] = src[0];
        xl[e * Gm::PSTR + 1] = src[1];
      }
    } else {
      constexpr int CH = CIN * sizeof(T) / 16;  // 16-byte chunks per pixel
#pragma unroll 4
      for (int e = threadIdx.x; e < EH * EW * CH; e += blockDim.x) {
        const int pix = e / CH, ch = e % CH;
        const int gy = min(max(y0 - 1 + pix / EW, 0), S.H - 1);
        const int gx = min(max(x0 - 1 + pix % EW, 0), S.W - 1);
        const uint4 v = *reinterpret_cast<const uint4*>(
            reinterpret_cast<const char*>(in + ((size_t)gy * S.W + gx) * CIN) + ch * 16);
        *reinterpret_cast<uint4*>(reinterpret_cast<char*>(xl + pix * Gm::PSTR) + ch * 16) = v;
      }
    }
    const int col = lane & 15, g = lane >> 4;
    T* out = reinterpret_cast<T*>(S.out);
    for (int pass = 0; pass < Gm::PASSES; ++pass) {
      if (Gm::PASSES > 1) load_weights(S.wimg, pass * Gm::CT);
      __syncthreads();
      floatx4 acc[Gm::MB][4];
#pragma unroll
      for (int mb = 0; mb < Gm::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
      conv_tile<T, CIN, COUT>(wl, xl, acc, wave, lane);
      // epilogue: bias + ReLU; lane holds couts 4g..4g+3 of block mb for pixel col
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int gy = y0 + wave * 4 + nb, gx = x0 + col;
        if (gy >= S.H || gx >= S.W) continue;
        T* dst = out + ((size_t)gy * S.W + gx) * COUT;
#pragma unroll
        for (int mb = 0; mb < Gm::MB; ++mb) {
          const int co = pass * Gm::CT + mb * 16 + g * 4;
          float v0 = fmaxf(acc[mb][nb][0] + S.b[co + 0], 0.f);
          float v1 = fmaxf(acc[mb][nb][1] + S.b[co + 1], 0.f);
          float v2 = fmaxf(acc[mb][nb][2] + S.b[co + 2], 0.f);
          float v3 = fmaxf(acc[mb][nb][3] + S.b[co + 3], 0.f);
          if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4*>(dst + co) = make_float4(v0, v1, v2, v3);
          } else {
            uint2 pk;
            pk.x = (uint32_t)f2bf(v0) | ((uint32_t)f2bf(v1) << 16);
            pk.y = (uint32_t)f2bf(v2) | ((uint32_t)f2bf(v3) << 16);
            *reinterpret_cast<uint2*>(dst + co) = pk;
          }
        }
      }
    }
    __syncthreads();
  }
}

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
template <typename T, int CIN, int COUT>
__device__ __forceinline__ void write_wimg(const float* __restrict__ w, T* __restrict__ img, int e) {
  using Gm = ConvGeom<T, CIN, COUT>;
  const int co = e / Gm::WSTR, kk = e % Gm::WSTR;
  const float v = kk < Gm::KTOT ? w[co * Gm::KTOT + kk] : 0.f;
  img[e] = St<T>::from(v);
}

template <typename T, int C>
struct WImg {
  static constexpr size_t L0 = (size_t)C * ConvGeom<T, 2, C>::WSTR;   // elements, layer 0
  static constexpr size_t L1 = (size_t)C * ConvGeom<T, C, C>::WSTR;   // elements, layers 1..3
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
    write_wimg<T, 2, C>(wk, ik, (int)e);
    return;
  }
  e -= WI::L0;
  const int l = 1 + (int)(e / WI::L1);
  const int el = (int)(e % WI::L1);
  const size_t woff = (size_t)C * 18 + C + (size_t)(l - 1) * ((size_t)C * 9 * C + C);
  write_wimg<T, C, C>(wk + woff, ik + WI::L0 + (size_t)(l - 1) * WI::L1, el);
}

size_t cnn_weight_image_bytes(const NetShape& net) {
  if (net.scales <= 0) return 0;
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
      tiles += D.tiles_x * ((D.H + TH - 1) / TH);
    }
    L.total_tiles = tiles;
    // launch on the caller's stream
    using Gm0 = ConvGeom<T, 2, C>;
    using Gm1 = ConvGeom<T, C, C>;
    if (l == 0) {
      e = hipFuncSetAttribute((const void*)conv3x3_relu<T, 2, C>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)Gm0::LDS);
      if (e != hipSuccess) return e;
      const int G = min(tiles, dev.cu * 2);
      L.tiles_per_wg = (tiles + G - 1) / G;
      const int nwg = (tiles + L.tiles_per_wg - 1) / L.tiles_per_wg;
      hipLaunchKernelGGL((conv3x3_relu<T, 2, C>), dim3(nwg), dim3(256), Gm0::LDS, s, L);
    } else {
      e = hipFuncSetAttribute((const void*)conv3x3_relu<T, C, C>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)Gm1::LDS);
      if (e != hipSuccess) return e;
      const int G = min(tiles, dev.cu * 2);
      L.tiles_per_wg = (tiles + G - 1) / G;
      const int nwg = (tiles + L.tiles_per_wg - 1) / L.tiles_per_wg;
      hipLaunchKernelGGL((conv3x3_relu<T, C, C>), dim3(nwg), dim3(256), Gm1::LDS, s, L);
    }
    e = hipGetLastError();
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
