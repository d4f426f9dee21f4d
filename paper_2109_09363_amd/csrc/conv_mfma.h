// k x k convolution with replicated edges, bias and optional ReLU as an
// implicit GEMM on MFMA (the convolution layers of Sec. 3.1's networks):
//   D[cout][px] = b[cout] + sum_k W[cout][k] X[k][px],  k = (tap, cin).
// One template serves both precisions: FP32 storage with
// v_mfma_f32_16x16x4f32, and BF16 storage with the gfx950
// v_mfma_f32_16x16x32_bf16, or v_mfma_f32_16x16x16_bf16 where the input
// width is a multiple of 16 but not of 32 (FP32 accumulation).  Activations
// are NHWC so a lane's K-fragment is 8-16 contiguous bytes in LDS; inputs of
// 2 or 3 channels (the network inputs) are gathered element by element.
// A work-group computes 16x16-pixel tiles (BF16 layers on wide inputs with
// 8 waves of 2 rows, the others with 4 waves of 4 rows); every scale of a
// layer can run in one launch over a concatenated tile list.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace hyp {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

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
constexpr int TW = 16;  // tile width (pixels)
constexpr int TH = 16;  // tile height

struct ScaleDesc {
  const void* in;     // NHWC input activations (storage type)
  void* out;          // NHWC output activations
  const void* wimg;   // weights as the LDS image: [Cout][WSTR] storage type, zero-padded K
  const float* b;     // FP32 bias [Cout]
  int H, W;
  int ostr;           // output elements per pixel (Cout, or wider inside a concatenation)
  int tiles_x, tile0; // tile columns, first global tile index of this scale
  const float* hw;    // fused 1x1 head (HEAD instances): w[Cout] then bias
  float* y;           // ... its FP32 output, one value per pixel
};

struct ConvLaunch {
  ScaleDesc sc[kMaxScales];
  const ScaleDesc* table;  // non-null: `ndesc` descriptors in device memory in
  int ndesc;               // tile0 order instead of sc[] (batches of grids)
  int nscales, total_tiles, tiles_per_wg;
  int skip_store;     // HEAD instances: 1 = do not store the activations
};

// K step of one MFMA fragment and the padded weight row, shared by the
// kernels and the host code that writes weight images.  BF16 uses 32-wide
// fragments unless the (not gathered) input width is an odd multiple of 16.
__host__ __device__ constexpr int conv_kstep(int elt, int cin) {
  return elt == 4 ? 16 : ((cin >= 8 && cin % 32 != 0) ? 16 : 32);
}
__host__ __device__ constexpr int conv_wstr(int elt, int ks, int cin) {
  return ((ks * ks * cin + conv_kstep(elt, cin) - 1) / conv_kstep(elt, cin)) * conv_kstep(elt, cin) +
         16 / elt;
}
// Input channels per pass over the input: all of them when the input tile
// with its border and 16 output rows of weights fit the 160 KB of LDS,
// else chunks of 64 (FP32 inputs of 128 channels).
__host__ __device__ constexpr int conv_cc(int elt, int ks, int cin) {
  return (cin < 8 || (size_t)(TH + ks - 1) * (TW + ks - 1) * (cin + 16 / elt) * elt +
                             (size_t)16 * conv_wstr(elt, ks, cin) * elt <= 160 * 1024)
             ? cin
             : 64;
}

template <typename T, int KS, int CIN, int COUT>
struct ConvGeom {
  static constexpr int ELT = sizeof(T);
  static constexpr bool SMALL = CIN < 8;                      // gathered input channels
  static constexpr int CC = conv_cc(ELT, KS, CIN);            // input channels per chunk
  static constexpr int NCH = CIN / CC;                        // chunks
  static constexpr int KSTEP = conv_kstep(ELT, CC);           // K per fragment step
  static constexpr int HALO = KS / 2;
  static constexpr int EW = TW + KS - 1, EH = TH + KS - 1;    // input tile with halo
  static constexpr int KTOT = KS * KS * CC;                   // K of one chunk
  static constexpr int KPAD = ((KTOT + KSTEP - 1) / KSTEP) * KSTEP;
  static constexpr int WSTR = conv_wstr(ELT, KS, CC);         // LDS weight row stride (elts)
  static constexpr int PSTR = SMALL ? CIN : CC + 16 / ELT;    // LDS pixel stride (elts)
  static constexpr size_t TILE_LDS = (((size_t)EH * EW * PSTR * ELT + 15) / 16) * 16;
  // output channels per pass: all of them unless their weights and the
  // input tile overflow the 160 KB of LDS (FP32 64 -> 64: 16 per pass)
  static constexpr int CT = ((size_t)COUT * WSTR * ELT + TILE_LDS <= 160 * 1024) ? COUT : 16;
  static constexpr int PASSES = COUT / CT;
  static constexpr int MB = CT / 16;                          // cout blocks per pass
  // bias and (head layers) the 1x1 head's weights of the scale, FP32
  static constexpr size_t PARAM_LDS = (size_t)(2 * COUT + 4) * 4;
  static constexpr size_t LDS = (size_t)CT * WSTR * ELT + TILE_LDS + PARAM_LDS;
  // waves per work-group: BF16 layers on wide inputs run 8 waves of 2 tile
  // rows, so that two waves share each SIMD and one's epilogue, barrier and
  // LDS waits overlap the other's MFMAs (their 220+ registers allow no
  // second work-group per CU); the rest 4 waves of 4 rows
  static constexpr int NW = (ELT == 2 && !SMALL) ? 8 : 4;
  static constexpr int RPW = TH / NW;                         // tile rows per wave
  static constexpr int NT = 64 * NW;                          // threads
  static_assert(TH % NW == 0, "whole rows per wave");
  static_assert(COUT % 16 == 0, "output channels in blocks of 16");
  static_assert(CIN % CC == 0, "whole input chunks");
  static_assert(SMALL || CC % KSTEP == 0, "input channels in whole K fragments");
  static_assert(KS % 2 == 1, "odd kernel size");
  static_assert(LDS <= 160 * 1024, "tile and weights fit the LDS of a CU");
};

// Fragment loads.  FP32: a lane holds 4 consecutive K values (one float4) and
// feeds them to 4 MFMAs; BF16: 8 consecutive K values (16 bytes) for one MFMA.
template <typename T, int KS, int CIN, int COUT>
__device__ __forceinline__ void conv_tile(const T* __restrict__ wl, const T* __restrict__ xl,
                                          floatx4 (&acc)[ConvGeom<T, KS, CIN, COUT>::MB][ConvGeom<T, KS, CIN, COUT>::RPW],
                                          int wave, int lane) {
  using Gm = ConvGeom<T, KS, CIN, COUT>;
  constexpr int EW = Gm::EW;
  const int col = lane & 15, g = lane >> 4;
  if constexpr (Gm::SMALL) {
    // K = KS*KS*CIN (tap, cin) gathered per element, zero-padded to KPAD
    for (int k0 = 0; k0 < Gm::KPAD; k0 += Gm::KSTEP) {
      constexpr int PER = (sizeof(T) == 4) ? 4 : 8;
      T bv[Gm::RPW][PER];
#pragma unroll
      for (int nb = 0; nb < Gm::RPW; ++nb) {
        const int row = wave * Gm::RPW + nb;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          const int k = k0 + g * PER + e;
          T val = St<T>::from(0.f);
          if (k < Gm::KTOT) {
            const int tap = k / CIN, ci = k % CIN;
            val = xl[((row + tap / KS) * EW + col + tap % KS) * Gm::PSTR + ci];
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
          for (int nb = 0; nb < Gm::RPW; ++nb) {
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bv[nb][0], acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bv[nb][1], acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, bv[nb][2], acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, bv[nb][3], acc[mb][nb], 0, 0, 0);
          }
        } else {
          const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(wrow));
#pragma unroll
          for (int nb = 0; nb < Gm::RPW; ++nb) {
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
    // taps unrolled: a loop over them made the compiler rotate the
    // accumulators between registers at every iteration
#pragma unroll
    for (int tap = 0; tap < KS * KS; ++tap) {
      const int ky = tap / KS, kx = tap % KS;
#pragma unroll
      for (int c0 = 0; c0 < Gm::CC; c0 += Gm::KSTEP) {
        const int k0 = tap * Gm::CC + c0;
        if constexpr (sizeof(T) == 4) {
          float4 bv[Gm::RPW];
#pragma unroll
          for (int nb = 0; nb < Gm::RPW; ++nb) {
            const int row = wave * Gm::RPW + nb;
            bv[nb] = *reinterpret_cast<const float4*>(
                xl + ((row + ky) * EW + col + kx) * Gm::PSTR + c0 + g * 4);
          }
#pragma unroll
          for (int mb = 0; mb < Gm::MB; ++mb) {
            const float4 a = *reinterpret_cast<const float4*>(wl + (mb * 16 + col) * Gm::WSTR + k0 + g * 4);
#pragma unroll
            for (int nb = 0; nb < Gm::RPW; ++nb) {
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bv[nb].x, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bv[nb].y, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, bv[nb].z, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, bv[nb].w, acc[mb][nb], 0, 0, 0);
            }
          }
        } else if constexpr (Gm::KSTEP == 16) {
          // BF16 with 16-wide fragments: 4 consecutive K values per lane
          shortx4 bv[Gm::RPW];
#pragma unroll
          for (int nb = 0; nb < Gm::RPW; ++nb) {
            const int row = wave * Gm::RPW + nb;
            bv[nb] = *reinterpret_cast<const shortx4*>(
                xl + ((row + ky) * EW + col + kx) * Gm::PSTR + c0 + g * 4);
          }
#pragma unroll
          for (int mb = 0; mb < Gm::MB; ++mb) {
            const shortx4 a =
                *reinterpret_cast<const shortx4*>(wl + (mb * 16 + col) * Gm::WSTR + k0 + g * 4);
#pragma unroll
            for (int nb = 0; nb < Gm::RPW; ++nb)
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv[nb], acc[mb][nb], 0, 0, 0);
          }
        } else {
          bf16x8 bv[Gm::RPW];
#pragma unroll
          for (int nb = 0; nb < Gm::RPW; ++nb) {
            const int row = wave * Gm::RPW + nb;
            bv[nb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                xl + ((row + ky) * EW + col + kx) * Gm::PSTR + c0 + g * 8));
          }
#pragma unroll
          for (int mb = 0; mb < Gm::MB; ++mb) {
            const bf16x8 a = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4*>(wl + (mb * 16 + col) * Gm::WSTR + k0 + g * 8));
#pragma unroll
            for (int nb = 0; nb < Gm::RPW; ++nb)
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv[nb], acc[mb][nb], 0, 0, 0);
          }
        }
      }
    }
  }
}

// The 16-byte pieces of an input tile (replicated border) that thread
// threadIdx.x loads into registers, and their store into the LDS tile.
template <typename T, int CIN, int EW, int HALO, int PCH, int NPIECE, int NPF, int NT>
__device__ __forceinline__ void conv_prefetch(const ScaleDesc& S, int x0, int y0, u32x4 (&pf)[NPF]) {
  const T* in = reinterpret_cast<const T*>(S.in);
#pragma unroll
  for (int i = 0; i < NPF; ++i) {
    const int e = threadIdx.x + NT * i;
    if (NT * (i + 1) <= NPIECE || e < NPIECE) {
      const int pix = e / PCH, piece = e % PCH;
      const int gy = min(max(y0 - HALO + pix / EW, 0), S.H - 1);
      const int gx = min(max(x0 - HALO + pix % EW, 0), S.W - 1);
      pf[i] = gld(reinterpret_cast<const u32x4*>(
          reinterpret_cast<const char*>(in + ((size_t)gy * S.W + gx) * CIN) + piece * 16));
    }
  }
}

template <typename T, int PSTR, int PCH, int NPIECE, int NPF, int NT>
__device__ __forceinline__ void conv_commit(T* xl, const u32x4 (&pf)[NPF]) {
#pragma unroll
  for (int i = 0; i < NPF; ++i) {
    const int e = threadIdx.x + NT * i;
    if (NT * (i + 1) <= NPIECE || e < NPIECE) {
      const int pix = e / PCH, piece = e % PCH;
      *reinterpret_cast<u32x4*>(reinterpret_cast<char*>(xl + pix * PSTR) + piece * 16) = pf[i];
    }
  }
}

// HEAD: the layer is followed by a linear 1x1 convolution to one channel;
// its output y = sum_c w_c a_c + b is formed in the epilogue from the
// activations as stored (rounded to the storage type), summed over the
// lane's output channels and across the four lane groups of a pixel.
template <typename T, int KS, int CIN, int COUT, bool RELU, bool HEAD = false>
__global__ __launch_bounds__((ConvGeom<T, KS, CIN, COUT>::NT)) void conv_mfma(ConvLaunch L) {
  using Gm = ConvGeom<T, KS, CIN, COUT>;
  constexpr int EW = Gm::EW, EH = Gm::EH, HALO = Gm::HALO;
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  T* wl = reinterpret_cast<T*>(lds_raw);
  T* xl = wl + Gm::CT * Gm::WSTR;
  float* pl = reinterpret_cast<float*>(lds_raw + Gm::CT * Gm::WSTR * Gm::ELT + Gm::TILE_LDS);  // bias, head
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t_begin = blockIdx.x * L.tiles_per_wg;
  const int t_end = min(t_begin + L.tiles_per_wg, L.total_tiles);
  const void* cur = nullptr;  // weight image in LDS
  // copy cout rows [co0, co0 + CT) of input chunk ch of the layer's weight
  // image ([NCH][Cout][WSTR]) into LDS with 16-byte loads, several in flight
  // per thread
  // LDS row R = 16 mb + 4 g + i (the MFMA's output row) holds local output
  // channel (CT / 4) g + 4 mb + i, so that the lanes of group g end up with
  // CT / 4 consecutive channels of their pixel
  auto load_weights = [&](const ScaleDesc& S, int ch, int co0) {
    __syncthreads();
    constexpr int RP = Gm::WSTR * Gm::ELT / 16;  // 16-byte pieces per row
    constexpr int N16 = Gm::CT * RP;
    const u32x4* src = reinterpret_cast<const u32x4*>(S.wimg) + ((size_t)ch * COUT + co0) * RP;
    u32x4* dstl = reinterpret_cast<u32x4*>(wl);
    // piece e of the LDS image comes from piece src_piece(e) of the rows
    // (16 rows per pass: the identity)
    auto src_piece = [](int e) {
      if constexpr (Gm::CT == 16) {
        return e;
      } else {
        const int R = e / RP, r = R & 15;
        return ((Gm::CT / 4) * (r >> 2) + 4 * (R >> 4) + (r & 3)) * RP + e % RP;
      }
    };
    // NB loads in flight per thread before their LDS writes
    constexpr int NB = 8;
    for (int e0 = threadIdx.x; e0 < N16; e0 += NB * Gm::NT) {
      u32x4 v[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int e = e0 + k * Gm::NT;
        if (e < N16) v[k] = gld(src + src_piece(e));
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int e = e0 + k * Gm::NT;
        if (e < N16) dstl[e] = v[k];
      }
    }
    // the epilogue's parameters (every bias, then the head's weights and
    // bias), once per tile: they serve all passes
    if (ch == 0 && co0 == 0) {
      for (int e = threadIdx.x; e < COUT; e += Gm::NT) pl[e] = gld(S.b + e);
      if constexpr (HEAD)
        for (int e = threadIdx.x; e <= COUT; e += Gm::NT) pl[COUT + e] = gld(S.hw + e);
    }
  };
  // input tile (channels of chunk ch) with a HALO-pixel replicated border
  auto load_tile = [&](const ScaleDesc& S, int x0, int y0, int ch) {
    const T* in = reinterpret_cast<const T*>(S.in);
    if constexpr (Gm::SMALL) {
      for (int e = threadIdx.x; e < EH * EW; e += blockDim.x) {
        const int gy = min(max(y0 - HALO + e / EW, 0), S.H - 1);
        const int gx = min(max(x0 - HALO + e % EW, 0), S.W - 1);
        const T* src = in + ((size_t)gy * S.W + gx) * CIN;
#pragma unroll
        for (int c = 0; c < CIN; ++c) xl[e * Gm::PSTR + c] = gld(src + c);
      }
    } else {
      constexpr int CH = Gm::CC * sizeof(T) / 16;  // 16-byte pieces per pixel
#pragma unroll 4
      for (int e = threadIdx.x; e < EH * EW * CH; e += blockDim.x) {
        const int pix = e / CH, piece = e % CH;
        const int gy = min(max(y0 - HALO + pix / EW, 0), S.H - 1);
        const int gx = min(max(x0 - HALO + pix % EW, 0), S.W - 1);
        const u32x4 v = gld(reinterpret_cast<const u32x4*>(reinterpret_cast<const char*>(
            in + ((size_t)gy * S.W + gx) * CIN + ch * Gm::CC) + piece * 16));
        *reinterpret_cast<u32x4*>(reinterpret_cast<char*>(xl + pix * Gm::PSTR) + piece * 16) = v;
      }
    }
  };
  // Wide inputs held whole in LDS are software-pipelined: the next tile's
  // 16-byte pieces are loaded into registers before this tile's MFMAs and
  // written to LDS after them, so their latency hides behind the math.
  constexpr bool PIPE = !Gm::SMALL && Gm::NCH == 1;
  constexpr int PCH = Gm::SMALL ? 1 : Gm::CC * (int)sizeof(T) / 16;  // pieces per pixel
  constexpr int NPIECE = EH * EW * PCH;
  constexpr int NPF = PIPE ? (NPIECE + Gm::NT - 1) / Gm::NT : 1;
  u32x4 pf[NPF];
  // the descriptor of global tile t (a scale, or a scale of one grid of a
  // batch) and the tile's origin
  auto locate = [&](int t, int& x0, int& y0) -> ScaleDesc {
    ScaleDesc D;
    if (L.table) {
      int lo = 0, hi = L.ndesc;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cld_int(&L.table[mid].tile0) <= t) lo = mid;
        else hi = mid;
      }
      D = cld(L.table, lo);
    } else {
      int k = 0;
      while (k + 1 < L.nscales && t >= cld_int(&L.sc[k + 1].tile0)) ++k;
      D = cld(L.sc, k);
    }
    const int lt = t - D.tile0;
    x0 = (lt % D.tiles_x) * TW;
    y0 = (lt / D.tiles_x) * TH;
    return D;
  };
  if constexpr (PIPE) {
    if (t_begin < t_end) {
      int x0, y0;
      const ScaleDesc D = locate(t_begin, x0, y0);
      conv_prefetch<T, CIN, EW, HALO, PCH, NPIECE, NPF, Gm::NT>(D, x0, y0, pf);
      conv_commit<T, Gm::PSTR, PCH, NPIECE, NPF, Gm::NT>(xl, pf);
    }
  }
  for (int t = t_begin; t < t_end; ++t) {
    int x0, y0;
    const ScaleDesc S = locate(t, x0, y0);
    if (Gm::PASSES == 1 && Gm::NCH == 1 && S.wimg != cur) {
      load_weights(S, 0, 0);
      cur = S.wimg;
    }
    if constexpr (!PIPE && Gm::NCH == 1) load_tile(S, x0, y0, 0);
    const int col = lane & 15, g = lane >> 4;
    T* out = reinterpret_cast<T*>(S.out);
    float hpart[Gm::RPW] = {};  // HEAD: partial 1x1 sums per row
    for (int pass = 0; pass < Gm::PASSES; ++pass) {
      floatx4 acc[Gm::MB][Gm::RPW];
#pragma unroll
      for (int mb = 0; mb < Gm::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < Gm::RPW; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
      if constexpr (Gm::NCH == 1) {
        if (Gm::PASSES > 1) load_weights(S, 0, pass * Gm::CT);
        __syncthreads();
        // issued after the last barrier before the MFMAs, so that no barrier
        // waits for these loads before the math starts
        if constexpr (PIPE) {
          if (pass == 0 && t + 1 < t_end) {
            int xn, yn;
            const ScaleDesc Dn = locate(t + 1, xn, yn);
            conv_prefetch<T, CIN, EW, HALO, PCH, NPIECE, NPF, Gm::NT>(Dn, xn, yn, pf);
          }
        }
        conv_tile<T, KS, CIN, COUT>(wl, xl, acc, wave, lane);
      } else {
        // K walks the input in chunks: weights and tile of each chunk
        for (int ch = 0; ch < Gm::NCH; ++ch) {
          load_weights(S, ch, pass * Gm::CT);
          load_tile(S, x0, y0, ch);
          __syncthreads();
          conv_tile<T, KS, CIN, COUT>(wl, xl, acc, wave, lane);
        }
      }
      // epilogue: bias (+ ReLU); the lanes of group g hold output channels
      // c0 .. c0 + CT/4 - 1 of pixel col of row nb (block mb: 4 of them)
#pragma unroll
      for (int nb = 0; nb < Gm::RPW; ++nb) {
        const int gy = y0 + wave * Gm::RPW + nb, gx = x0 + col;
        const bool inside = gy < S.H && gx < S.W;
        if (!HEAD && !inside) continue;
        const int c0 = pass * Gm::CT + g * (Gm::CT / 4);
        float v[Gm::MB][4];
#pragma unroll
        for (int mb = 0; mb < Gm::MB; ++mb) {
          const float4 bias = *reinterpret_cast<const float4*>(pl + c0 + 4 * mb);
          v[mb][0] = acc[mb][nb][0] + bias.x;
          v[mb][1] = acc[mb][nb][1] + bias.y;
          v[mb][2] = acc[mb][nb][2] + bias.z;
          v[mb][3] = acc[mb][nb][3] + bias.w;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if constexpr (RELU) v[mb][i] = fmaxf(v[mb][i], 0.f);
          if constexpr (HEAD) {
            const float4 hw = *reinterpret_cast<const float4*>(pl + COUT + c0 + 4 * mb);
            hpart[nb] += St<T>::to_f(St<T>::from(v[mb][0])) * hw.x + St<T>::to_f(St<T>::from(v[mb][1])) * hw.y +
                         St<T>::to_f(St<T>::from(v[mb][2])) * hw.z + St<T>::to_f(St<T>::from(v[mb][3])) * hw.w;
          }
        }
        if (HEAD && (!inside || L.skip_store)) continue;
        T* dst = out + ((size_t)gy * S.W + gx) * S.ostr + c0;
        if constexpr (sizeof(T) == 4) {
#pragma unroll
          for (int mb = 0; mb < Gm::MB; ++mb)
            gst(reinterpret_cast<floatx4*>(dst + 4 * mb), floatx4{v[mb][0], v[mb][1], v[mb][2], v[mb][3]});
        } else {
          // 8 channels (16 bytes) per store
#pragma unroll
          for (int h = 0; h < Gm::MB; h += 2) {
            const uint32_t p0 = (uint32_t)f2bf(v[h][0]) | ((uint32_t)f2bf(v[h][1]) << 16);
            const uint32_t p1 = (uint32_t)f2bf(v[h][2]) | ((uint32_t)f2bf(v[h][3]) << 16);
            if (h + 1 < Gm::MB) {
              const uint32_t p2 = (uint32_t)f2bf(v[h + 1][0]) | ((uint32_t)f2bf(v[h + 1][1]) << 16);
              const uint32_t p3 = (uint32_t)f2bf(v[h + 1][2]) | ((uint32_t)f2bf(v[h + 1][3]) << 16);
              gst(reinterpret_cast<u32x4*>(dst + 4 * h), u32x4{p0, p1, p2, p3});
            } else {
              gst(reinterpret_cast<u32x2*>(dst + 4 * h), u32x2{p0, p1});
            }
          }
        }
      }
    }
    if constexpr (HEAD) {
      // the four lane groups (g) of a pixel hold disjoint output channels
#pragma unroll
      for (int nb = 0; nb < Gm::RPW; ++nb) {
        float hs = hpart[nb];
        hs += __shfl_xor(hs, 16);
        hs += __shfl_xor(hs, 32);
        const int gy = y0 + wave * Gm::RPW + nb, gx = x0 + col;
        if (g == 0 && gy < S.H && gx < S.W) gst(S.y + (size_t)gy * S.W + gx, hs + pl[2 * COUT]);
      }
    }
    __syncthreads();
    if constexpr (PIPE) {
      if (t + 1 < t_end) conv_commit<T, Gm::PSTR, PCH, NPIECE, NPF, Gm::NT>(xl, pf);
    }
  }
}

// One element of a layer's weight image: chunk ch, row co, column kk of the
// [NCH][Cout][WSTR] LDS layout (storage type, K zero-padded) from the packed
// FP32 weights W[Cout][KS][KS][Cin]; column kk = tap * CC + c holds input
// channel ch * CC + c.
template <typename T, int KS, int CIN, int COUT>
__device__ __forceinline__ void write_wimg(const float* __restrict__ w, T* __restrict__ img, int e) {
  using Gm = ConvGeom<T, KS, CIN, COUT>;
  const int ch = e / (COUT * Gm::WSTR), r = e % (COUT * Gm::WSTR);
  const int co = r / Gm::WSTR, kk = r % Gm::WSTR;
  float v = 0.f;
  if (kk < Gm::KTOT) {
    const int tap = kk / Gm::CC, c = kk % Gm::CC;
    v = w[(size_t)co * KS * KS * CIN + tap * CIN + ch * Gm::CC + c];
  }
  img[e] = St<T>::from(v);
}

// Launch one layer over the tile list of L on stream s: as many work-groups
// as the LDS of the CUs holds at once (up to 2 per CU), so that every one
// loads its weights once and all run in a single round, each over a run of
// whole tiles.
template <typename T, int KS, int CIN, int COUT, bool RELU, bool HEAD = false>
hipError_t launch_conv(ConvLaunch& L, int cu, hipStream_t s) {
  using Gm = ConvGeom<T, KS, CIN, COUT>;
  hipError_t e = hipFuncSetAttribute((const void*)conv_mfma<T, KS, CIN, COUT, RELU, HEAD>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)Gm::LDS);
  if (e != hipSuccess) return e;
  const int tiles = L.total_tiles;
  if (tiles <= 0) return hipSuccess;
  const int per_cu = (int)((size_t)160 * 1024 / Gm::LDS);
  const int G = min(tiles, cu * (per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu)));
  L.tiles_per_wg = (tiles + G - 1) / G;
  const int nwg = (tiles + L.tiles_per_wg - 1) / L.tiles_per_wg;
  hipLaunchKernelGGL((conv_mfma<T, KS, CIN, COUT, RELU, HEAD>), dim3(nwg), dim3(Gm::NT), Gm::LDS, s, L);
  return hipGetLastError();
}

}  // namespace hyp
