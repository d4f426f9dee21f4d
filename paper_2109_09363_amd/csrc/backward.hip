// Adjoint of the hybrid projection for training with the solver in the loop
// (the gradient of the correction of Eq. 2 is known, Sec. 3.2):
//
//   loss = scale * sum_F r^2,   r = d - L phi_K,
//   phi_K = K Jacobi sweeps from phi0 = dx^2 s CNN([d/s, solid]; theta).
//
// Reverse sweep (L symmetric on fluid cells, kinv = 1/k_c):
//   lam_r = 2 scale r;  lam_phi = -L lam_r;  lam_d = lam_r
//   K times: lam_d -= omega dx^2 kinv lam;  lam <- (1-omega) lam + omega sum_n kinv_n lam_n
//   CNN: lam_t0 = dx^2 s lam_phi0, upsample-sum transpose, 1x1 head, four
//   3x3 layers (ReLU masks, weight gradients, input gradients with the
//   replicate-padding adjoint), 2x2-mean pyramid transpose, the d/s
//   normalisation with ds/dd, then D^T onto the faces.
// Every reduction (loss, lambda_s, weight and bias gradients) is two-stage
// with a fixed order, so the result is bitwise reproducible.  Activations
// may be stored as FP32 or BF16; the adjoint arithmetic is FP32.
#include "../../include/hyproj.h"
#include "common.h"
#include "internal.h"
#include "cascade.h"
#include "unet.h"

namespace hyp {

template <typename T> __device__ __forceinline__ float ld(const T* p);
template <> __device__ __forceinline__ float ld<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float ld<uint16_t>(const uint16_t* p) {
  return __uint_as_float((uint32_t)(*p) << 16);
}

// ---- solver part ----------------------------------------------------------
__global__ __launch_bounds__(256) void bw_init(int nx, int ny, float inv_dx2, float scale2,
                                               const uint8_t* __restrict__ cell,
                                               const float* __restrict__ d,
                                               const float* __restrict__ phi,
                                               float* __restrict__ lam_r, float* __restrict__ lam_d,
                                               double* __restrict__ blockpart) {
  __shared__ double red[4];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double rr = 0.0;
  if (c < nx * ny) {
    const uint8_t ci = cell[c];
    float lam = 0.f;
    if (!(ci & C_SOLID)) {
      const int j = c / nx;
      const float pe = (ci & C_E) ? phi[c + 1] : 0.f;
      const float pw = (ci & C_W) ? phi[c - 1] : 0.f;
      const float pn = ((ci & C_N) && j + 1 < ny) ? phi[c + nx] : 0.f;
      const float ps = (ci & C_S) ? phi[c - nx] : 0.f;
      const float r = d[c] - (((pe + pw) + (pn + ps)) - (float)cell_k(ci) * phi[c]) * inv_dx2;
      lam = scale2 * r;
      rr = (double)r * (double)r;
    }
    lam_r[c] = lam;
    lam_d[c] = lam;
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) blockpart[blockIdx.x] = rr;
}

__global__ __launch_bounds__(256) void bw_loss_finish(int nblocks, const double* __restrict__ bp,
                                                      double scale, Scalars* sc, double* loss_out) {
  __shared__ double red[4];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) a += bp[b];
  a = block_sum(a, red);
  if (threadIdx.x == 0) {
    sc->loss = scale * a;
    if (loss_out) *loss_out = scale * a;
  }
}

// out = -L in on fluid cells
__global__ __launch_bounds__(256) void bw_neglap(int nx, int ny, float inv_dx2,
                                                 const uint8_t* __restrict__ cell,
                                                 const float* __restrict__ in,
                                                 float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  const uint8_t ci = cell[c];
  float o = 0.f;
  if (!(ci & C_SOLID)) {
    const int j = c / nx;
    const float e = (ci & C_E) ? in[c + 1] : 0.f;
    const float w = (ci & C_W) ? in[c - 1] : 0.f;
    const float n = ((ci & C_N) && j + 1 < ny) ? in[c + nx] : 0.f;
    const float s = (ci & C_S) ? in[c - nx] : 0.f;
    o = -(((e + w) + (n + s)) - (float)cell_k(ci) * in[c]) * inv_dx2;
  }
  out[c] = o;
}

__device__ __forceinline__ float kinv_of(uint8_t c) {
  return (c & C_SOLID) ? 0.f : 1.f / (float)cell_k(c);
}

// one reversed Jacobi sweep
__global__ __launch_bounds__(256) void bw_jacobi(int nx, int ny, float omega, float wdx2,
                                                 const uint8_t* __restrict__ cell,
                                                 const float* __restrict__ lam,
                                                 float* __restrict__ lam_out,
                                                 float* __restrict__ lam_d) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  const uint8_t ci = cell[c];
  if (ci & C_SOLID) {
    lam_out[c] = 0.f;
    return;
  }
  const int j = c / nx;
  float sum = 0.f;
  if (ci & C_E) sum += kinv_of(cell[c + 1]) * lam[c + 1];
  if (ci & C_W) sum += kinv_of(cell[c - 1]) * lam[c - 1];
  if ((ci & C_N) && j + 1 < ny) sum += kinv_of(cell[c + nx]) * lam[c + nx];
  if (ci & C_S) sum += kinv_of(cell[c - nx]) * lam[c - nx];
  const float l = lam[c];
  lam_out[c] = (1.f - omega) * l + omega * sum;
  lam_d[c] -= wdx2 * kinv_of(ci) * l;
}

// lam_t0 = dx^2 s lam_phi0 (fluid); partial sums of lam_phi0 * t0 for lam_s
__global__ __launch_bounds__(256) void bw_phi0(int n, float dx2, const uint8_t* __restrict__ cell,
                                               const float* __restrict__ lam,
                                               const float* __restrict__ t0,
                                               float* __restrict__ lam_t0,
                                               double* __restrict__ blockpart, const Scalars* sc) {
  __shared__ double red[4];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double a = 0.0;
  const float s = (float)sc->s;
  if (c < n) {
    const bool fl = !(cell[c] & C_SOLID);
    const float l = fl ? lam[c] : 0.f;
    lam_t0[c] = dx2 * s * l;
    a = (double)l * (double)t0[c];
  }
  a = block_sum(a, red);
  if (threadIdx.x == 0) blockpart[blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void bw_lams_set(int nblocks, const double* __restrict__ bp,
                                                   double dx2, Scalars* sc) {
  __shared__ double red[4];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) a += bp[b];
  a = block_sum(a, red);
  if (threadIdx.x == 0) sc->lam_s = dx2 * a;
}

// Adjoint of up2 (bilinear x2, half-pixel centres, clamp): a coarse pixel
// gathers from the fine pixels whose interpolation stencil uses it.
__device__ __forceinline__ void up_axis(int J, int nc, int* i0, int* i1, float* f) {
  float c = fminf(fmaxf(0.5f * (float)J - 0.25f, 0.f), (float)(nc - 1));
  int a = min((int)floorf(c), max(nc - 2, 0));
  *i0 = a;
  *i1 = min(a + 1, nc - 1);
  *f = c - (float)a;
}

__global__ __launch_bounds__(256) void bw_up2T(int Hc, int Wc, const float* __restrict__ fine,
                                               float* __restrict__ coarse) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= Hc * Wc) return;
  const int X = gid % Wc, Y = gid / Wc;
  const int Hf = 2 * Hc, Wf = 2 * Wc;
  float acc = 0.f;
  for (int J = max(2 * Y - 2, 0); J <= min(2 * Y + 3, Hf - 1); ++J) {
    int y0, y1;
    float fy;
    up_axis(J, Hc, &y0, &y1, &fy);
    const float wy = (y0 == Y ? 1.f - fy : 0.f) + (y1 == Y ? fy : 0.f);
    if (wy == 0.f) continue;
    for (int I = max(2 * X - 2, 0); I <= min(2 * X + 3, Wf - 1); ++I) {
      int x0, x1;
      float fx;
      up_axis(I, Wc, &x0, &x1, &fx);
      const float wx = (x0 == X ? 1.f - fx : 0.f) + (x1 == X ? fx : 0.f);
      if (wx == 0.f) continue;
      acc += wy * wx * fine[J * Wf + I];
    }
  }
  coarse[gid] = acc;
}

// ---- CNN part ---------------------------------------------------------------
// head: lam_pre3[px][c] = lam_y[px] wo[c] (times h4 > 0 when the head's
// input layer has a ReLU); partial dwo, dbo
template <typename T, int C, bool MASK = true>
__global__ __launch_bounds__(256) void bw_head(int npx, const float* __restrict__ lam_y,
                                               const T* __restrict__ h4,
                                               const float* __restrict__ wo,
                                               float* __restrict__ lam_pre,
                                               float* __restrict__ part) {
  const int p0 = blockIdx.x * 256;
  const int px = p0 + threadIdx.x;
  if (px < npx) {
    const float ly = lam_y[px];
    for (int c = 0; c < C; ++c) {
      const float h = ld<T>(h4 + (size_t)px * C + c);
      lam_pre[(size_t)px * C + c] = (!MASK || h > 0.f) ? ly * wo[c] : 0.f;
    }
  }
  if (threadIdx.x <= C) {
    float acc = 0.f;
    const int c = threadIdx.x;
    for (int q = p0; q < min(p0 + 256, npx); ++q)
      acc += lam_y[q] * (c < C ? ld<T>(h4 + (size_t)q * C + c) : 1.f);
    part[(size_t)blockIdx.x * (C + 1) + c] = acc;
  }
}

// fixed-order sum of per-block partials into the packed gradient
__global__ __launch_bounds__(256) void bw_part_finish(int nblocks, int nout,
                                                      const float* __restrict__ part,
                                                      float* __restrict__ out, int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout) return;
  float acc = 0.f;
  for (int b = 0; b < nblocks; ++b) acc += part[(size_t)b * nout + e];
  out[e] = accumulate ? out[e] + acc : acc;
}

constexpr int BT = 16;       // backward tile side
constexpr int BE = BT + 2;

// Weight and bias gradients of one 3x3 layer at one scale:
//   dW[co][tap][ci] = sum_px lam_pre[px][co] in[clamp(px + tap - 1)][ci]
//   db[co]          = sum_px lam_pre[px][co]
// grid.x blocks take tiles bx, bx + gridDim.x, ...; grid.y splits the
// outputs into chunks of 256 * NACC; partials go to part[bx][out].
template <typename T, int CIN, int COUT, int NACC>
__global__ __launch_bounds__(256) void bw_wgrad(int H, int W, const T* __restrict__ in,
                                                const float* __restrict__ lam_pre,
                                                float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) float lds_w[];
  float* lt = lds_w;                 // [BT*BT][COUT]
  float* xt = lds_w + BT * BT * COUT; // [BE*BE][CIN]
  constexpr int NOUT = COUT * 9 * CIN + COUT;
  const int tiles_x = (W + BT - 1) / BT, tiles = tiles_x * ((H + BT - 1) / BT);
  const int e0 = blockIdx.y * 256 * NACC;
  float acc[NACC];
#pragma unroll
  for (int m = 0; m < NACC; ++m) acc[m] = 0.f;
  for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int x0 = (t % tiles_x) * BT, y0 = (t / tiles_x) * BT;
    __syncthreads();
    for (int e = threadIdx.x; e < BT * BT * COUT; e += 256) {
      const int q = e / COUT, co = e % COUT;
      const int gy = y0 + q / BT, gx = x0 + q % BT;
      lt[e] = (gy < H && gx < W) ? lam_pre[((size_t)gy * W + gx) * COUT + co] : 0.f;
    }
    for (int e = threadIdx.x; e < BE * BE * CIN; e += 256) {
      const int q = e / CIN, ci = e % CIN;
      const int gy = min(max(y0 - 1 + q / BE, 0), H - 1);
      const int gx = min(max(x0 - 1 + q % BE, 0), W - 1);
      xt[e] = ld<T>(in + ((size_t)gy * W + gx) * CIN + ci);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NACC; ++m) {
      const int e = e0 + m * 256 + threadIdx.x;
      if (e >= NOUT) break;
      float a = 0.f;
      if (e < COUT * 9 * CIN) {
        const int co = e / (9 * CIN), rem = e % (9 * CIN), tap = rem / CIN, ci = rem % CIN;
        const int ky = tap / 3, kx = tap % 3;
        for (int q = 0; q < BT * BT; ++q)
          a += lt[q * COUT + co] * xt[((q / BT + ky) * BE + (q % BT) + kx) * CIN + ci];
      } else {
        const int co = e - COUT * 9 * CIN;
        for (int q = 0; q < BT * BT; ++q) a += lt[q * COUT + co];
      }
      acc[m] += a;
    }
  }
#pragma unroll
  for (int m = 0; m < NACC; ++m) {
    const int e = e0 + m * 256 + threadIdx.x;
    if (e < NOUT) part[(size_t)blockIdx.x * NOUT + e] = acc[m];
  }
}

// Input gradient of one 3x3 layer (transposed convolution with the
// replicate-padding adjoint): lam_in[y][x][ci] = sum over taps and the
// output pixels whose clamped stencil reads (y, x).  With MASK the result
// is multiplied by (h_in > 0), the ReLU of the layer below; with ONLY_C0
// only input channel 0 is produced (the normalised divergence).
template <typename T, int CIN, int COUT, bool MASK, bool ONLY_C0>
__global__ __launch_bounds__(256) void bw_dgrad(int H, int W, const float* __restrict__ lam_pre,
                                                const float* __restrict__ Wt,
                                                const T* __restrict__ h_in,
                                                float* __restrict__ lam_in) {
  extern __shared__ __attribute__((aligned(16))) float lds_d[];  // [BE*BE][COUT]
  const int tiles_x = (W + BT - 1) / BT;
  const int x0 = (blockIdx.x % tiles_x) * BT, y0 = (blockIdx.x / tiles_x) * BT;
  for (int e = threadIdx.x; e < BE * BE * COUT; e += 256) {
    const int q = e / COUT, co = e % COUT;
    const int gy = y0 - 1 + q / BE, gx = x0 - 1 + q % BE;
    lds_d[e] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? lam_pre[((size_t)gy * W + gx) * COUT + co] : 0.f;
  }
  __syncthreads();
  const int ty = threadIdx.x / BT, tx = threadIdx.x % BT;
  const int y = y0 + ty, x = x0 + tx;
  if (y >= H || x >= W) return;
  constexpr int NC = ONLY_C0 ? 1 : CIN;
  float acc[NC];
#pragma unroll
  for (int ci = 0; ci < NC; ++ci) acc[ci] = 0.f;
  for (int ky = 0; ky < 3; ++ky) {
    int cy[2], ny_ = 0;
    { const int p = y - ky + 1; if (p >= 0 && p < H) cy[ny_++] = p; }
    if (y == 0 && ky == 0) cy[ny_++] = 0;
    if (y == H - 1 && ky == 2) cy[ny_++] = H - 1;
    for (int kx = 0; kx < 3; ++kx) {
      int cx[2], nx_ = 0;
      { const int p = x - kx + 1; if (p >= 0 && p < W) cx[nx_++] = p; }
      if (x == 0 && kx == 0) cx[nx_++] = 0;
      if (x == W - 1 && kx == 2) cx[nx_++] = W - 1;
      const float* wk = Wt + (ky * 3 + kx) * CIN;
      for (int a = 0; a < ny_; ++a)
        for (int b = 0; b < nx_; ++b) {
          const float* lp = lds_d + ((cy[a] - y0 + 1) * BE + (cx[b] - x0 + 1)) * COUT;
          for (int co = 0; co < COUT; ++co) {
            const float l = lp[co];
            const float* wr = wk + (size_t)co * 9 * CIN;
#pragma unroll
            for (int ci = 0; ci < NC; ++ci) acc[ci] += wr[ci] * l;
          }
        }
    }
  }
  const size_t px = (size_t)y * W + x;
  if constexpr (ONLY_C0) {
    lam_in[px] = acc[0];
  } else {
#pragma unroll
    for (int ci = 0; ci < NC; ++ci) {
      float v = acc[ci];
      if (MASK) v = ld<T>(h_in + px * CIN + ci) > 0.f ? v : 0.f;
      lam_in[px * CIN + ci] = v;
    }
  }
}

// pyramid transpose: lam_x(c) = sum_k lam_xk[parent] / 4^k on fluid cells;
// partial sums of lam_x * d for lam_s.
struct PyrT {
  const float* lx[5];
  int nscales;
};

__device__ __forceinline__ float pyr_lam(const PyrT& P, int i, int j, int nx) {
  float a = 0.f;
  for (int k = 0; k < P.nscales; ++k) {
    const int Wk = nx >> k;
    a += P.lx[k][(j >> k) * Wk + (i >> k)] * (1.f / (float)(1 << (2 * k)));
  }
  return a;
}

__global__ __launch_bounds__(256) void bw_pyr_sum(int nx, int ny, PyrT P,
                                                  const uint8_t* __restrict__ cell,
                                                  const float* __restrict__ d,
                                                  double* __restrict__ blockpart) {
  __shared__ double red[4];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double a = 0.0;
  if (c < nx * ny && !(cell[c] & C_SOLID)) a = (double)pyr_lam(P, c % nx, c / nx, nx) * (double)d[c];
  a = block_sum(a, red);
  if (threadIdx.x == 0) blockpart[blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void bw_lams_add(int nblocks, const double* __restrict__ bp,
                                                   Scalars* sc) {
  __shared__ double red[4];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) a += bp[b];
  a = block_sum(a, red);
  if (threadIdx.x == 0) {
    const double s = sc->s;
    if (s > 0.0) sc->lam_s -= a / (s * s);
  }
}

__global__ __launch_bounds__(256) void bw_dnorm(int nx, int ny, PyrT P,
                                                const uint8_t* __restrict__ cell,
                                                const float* __restrict__ d,
                                                float* __restrict__ lam_d, const Scalars* sc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny || (cell[c] & C_SOLID)) return;
  const double s = sc->s;
  if (!(s > 0.0)) return;
  const float inv_s = (float)(1.0 / s);
  const float ks = (float)(sc->lam_s / ((double)sc->nF * s));
  lam_d[c] += pyr_lam(P, c % nx, c / nx, nx) * inv_s + ks * d[c];
}

// D^T: face gradients from lam_d (open interior faces, open top faces,
// inflow faces; closed faces get 0)
__global__ __launch_bounds__(256) void bw_faces(int nx, int ny, float inv_dx,
                                                const uint8_t* __restrict__ cell,
                                                const float* __restrict__ lam_d,
                                                float* __restrict__ du, float* __restrict__ dv,
                                                int accumulate) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  const int i = c % nx, j = c / nx, U = nx + 1;
  const uint8_t ci = cell[c];
  const bool fl = !(ci & C_SOLID);
  const float l = fl ? lam_d[c] : 0.f;
  float gw = 0.f, gs = 0.f, gn = 0.f;
  if (fl && (ci & C_W)) gw = (lam_d[c - 1] - l) * inv_dx;
  if (j == 0) gs = (fl && (ci & C_INFLOW)) ? -l * inv_dx : 0.f;
  else if (fl && (ci & C_S)) gs = (lam_d[c - nx] - l) * inv_dx;
  if (j == ny - 1 && fl && (ci & C_N)) gn = l * inv_dx;
  if (du) {
    du[j * U + i] = accumulate ? du[j * U + i] + gw : gw;
    if (i == nx - 1 && !accumulate) du[j * U + nx] = 0.f;
  }
  if (dv) {
    dv[j * nx + i] = accumulate ? dv[j * nx + i] + gs : gs;
    if (j == ny - 1) dv[ny * nx + i] = accumulate ? dv[ny * nx + i] + gn : gn;
  }
}

// ---------------------------------------------------------------------------
template <typename T, int CIN, int COUT>
static hipError_t wgrad_layer(int H, int W, const T* in, const float* lam_pre, float* part,
                              size_t part_n, float* dst, int accumulate, hipStream_t s) {
  constexpr int NACC = 36;
  constexpr int NOUT = COUT * 9 * CIN + COUT;
  const int tiles = ((W + BT - 1) / BT) * ((H + BT - 1) / BT);
  const int gx = min(tiles, kWgBlocks);
  if ((size_t)gx * NOUT > part_n) return hipErrorInvalidValue;
  const int gy = (NOUT + 256 * NACC - 1) / (256 * NACC);
  const size_t lds = sizeof(float) * (BT * BT * COUT + BE * BE * CIN);
  auto k = bw_wgrad<T, CIN, COUT, NACC>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(gx, gy), dim3(256), lds, s, H, W, in, lam_pre, part);
  hipLaunchKernelGGL(bw_part_finish, dim3((NOUT + 255) / 256), dim3(256), 0, s, gx, NOUT, part,
                     dst, accumulate);
  return hipGetLastError();
}

template <typename T, int CIN, int COUT, bool MASK, bool ONLY_C0>
static hipError_t dgrad_layer(int H, int W, const float* lam_pre, const float* Wt, const T* h_in,
                              float* lam_in, hipStream_t s) {
  const int tiles = ((W + BT - 1) / BT) * ((H + BT - 1) / BT);
  const size_t lds = sizeof(float) * BE * BE * COUT;
  auto k = bw_dgrad<T, CIN, COUT, MASK, ONLY_C0>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(tiles), dim3(256), lds, s, H, W, lam_pre, Wt, h_in, lam_in);
  return hipGetLastError();
}

template <typename T, int C>
static hipError_t backward_cnn(const NetShape& net, const WsLayout& Ly, int nx, int ny,
                               const float* params, float* dparams, int acc, const Ws& w,
                               hipStream_t s) {
  const int S = net.scales;
  const size_t per_scale = (size_t)C * 18 + C + 3 * ((size_t)C * 9 * C + C) + C + 1;
  const size_t hoff = (size_t)C * 18 + C + 3 * ((size_t)C * 9 * C + C);
  const T* save = reinterpret_cast<const T*>(w.cnn_save);
  const T* in = reinterpret_cast<const T*>(w.cnn_in);
  auto act = [&](int l) { return save + (size_t)l * Ly.total_px * C; };  // output of layer l
  hipError_t e = hipSuccess;
  for (int k = 0; k < S; ++k) {
    const int H = Ly.sc_h[k], W = Ly.sc_w[k], npx = H * W;
    const size_t off = Ly.sc_off_px[k];
    const float* pk = params + k * per_scale;
    float* gk = dparams ? dparams + k * per_scale : nullptr;
    float* la = w.bw_a + off * C;  // lambda_pre of the current layer
    float* lb = w.bw_b + off * C;
    // head
    const int nbh = (npx + 255) / 256;
    if ((size_t)nbh * (C + 1) > w.bw_part_n) return hipErrorInvalidValue;
    hipLaunchKernelGGL((bw_head<T, C>), dim3(nbh), dim3(256), 0, s, npx, w.bw_t + off,
                       act(3) + off * C, pk + hoff, la, w.bw_part);
    if (gk) hipLaunchKernelGGL(bw_part_finish, dim3(1), dim3(256), 0, s, nbh, C + 1, w.bw_part,
                               gk + hoff, acc);
    for (int l = 3; l >= 0; --l) {
      const size_t woff = l == 0 ? 0 : (size_t)C * 18 + C + (size_t)(l - 1) * ((size_t)C * 9 * C + C);
      const float* Wt = pk + woff;
      if (l == 0) {
        if (gk) e = wgrad_layer<T, 2, C>(H, W, in + off * 2, la, w.bw_part, w.bw_part_n, gk + woff, acc, s);
        if (e != hipSuccess) return e;
        e = dgrad_layer<T, 2, C, false, true>(H, W, la, Wt, nullptr, w.bw_x + off, s);
      } else {
        if (gk) e = wgrad_layer<T, C, C>(H, W, act(l - 1) + off * C, la, w.bw_part, w.bw_part_n, gk + woff, acc, s);
        if (e != hipSuccess) return e;
        e = dgrad_layer<T, C, C, true, false>(H, W, la, Wt, act(l - 1) + off * C, lb, s);
        float* t = la; la = lb; lb = t;
      }
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The Unet's backward pass (Sec. 3.1's Unet, FP32 training).  The forward
// kept every layer's output (unet.h); lambda maps alternate between bw_a
// and bw_b.  Decoder scales 0..3 first (the reverse of the forward), each
// splitting the gradient of its concatenation into the skip part (kept per
// scale) and the part of the upsampled coarser map (upsampling adjoint, then
// that map's ReLU mask); then encoder scales 4..0, where the gradient of a
// pooled map goes to the window maxima (max-pooling adjoint), is added to
// the skip part and masked by the encoder output's ReLU.
// ---------------------------------------------------------------------------

// Weight and bias gradients of a KS x KS layer over input channels
// [ci0, ci0 + CC) of a CIN-channel input (chunks keep the tile in LDS):
// part[bx][e], e over (co, tap, c) of the chunk, then the biases (chunk 0).
template <int KS, int CIN, int CC, int COUT, int NACC>
__global__ __launch_bounds__(256) void bw_wgrad_c(int H, int W, const float* __restrict__ in, int ci0,
                                                  const float* __restrict__ lam_pre,
                                                  float* __restrict__ part) {
  constexpr int HK = KS / 2, BK = BT + KS - 1, NT = KS * KS;
  extern __shared__ __attribute__((aligned(16))) float lds_c[];
  float* lt = lds_c;                  // [BT*BT][COUT]
  float* xt = lds_c + BT * BT * COUT; // [BK*BK][CC]
  const int nw = COUT * NT * CC, nout = nw + (ci0 == 0 ? COUT : 0);
  const int tiles_x = (W + BT - 1) / BT, tiles = tiles_x * ((H + BT - 1) / BT);
  const int e0 = blockIdx.y * 256 * NACC;
  float acc[NACC];
#pragma unroll
  for (int m = 0; m < NACC; ++m) acc[m] = 0.f;
  for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int x0 = (t % tiles_x) * BT, y0 = (t / tiles_x) * BT;
    __syncthreads();
    for (int e = threadIdx.x; e < BT * BT * COUT; e += 256) {
      const int q = e / COUT, co = e % COUT;
      const int gy = y0 + q / BT, gx = x0 + q % BT;
      lt[e] = (gy < H && gx < W) ? lam_pre[((size_t)gy * W + gx) * COUT + co] : 0.f;
    }
    for (int e = threadIdx.x; e < BK * BK * CC; e += 256) {
      const int q = e / CC, c = e % CC;
      const int gy = min(max(y0 - HK + q / BK, 0), H - 1);
      const int gx = min(max(x0 - HK + q % BK, 0), W - 1);
      xt[e] = in[((size_t)gy * W + gx) * CIN + ci0 + c];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NACC; ++m) {
      const int e = e0 + m * 256 + threadIdx.x;
      if (e >= nout) break;
      float a = 0.f;
      if (e < nw) {
        const int co = e / (NT * CC), rem = e % (NT * CC), tap = rem / CC, c = rem % CC;
        const int ky = tap / KS, kx = tap % KS;
        for (int q = 0; q < BT * BT; ++q)
          a += lt[q * COUT + co] * xt[((q / BT + ky) * BK + (q % BT) + kx) * CC + c];
      } else {
        const int co = e - nw;
        for (int q = 0; q < BT * BT; ++q) a += lt[q * COUT + co];
      }
      acc[m] += a;
    }
  }
#pragma unroll
  for (int m = 0; m < NACC; ++m) {
    const int e = e0 + m * 256 + threadIdx.x;
    if (e < nout) part[(size_t)blockIdx.x * nout + e] = acc[m];
  }
}

// fixed-order sum of a chunk's partials into the layer's packed gradient
// (W[Cout][ks][ks][Cin] then b[Cout])
__global__ __launch_bounds__(256) void bw_part_finish_c(int nblocks, int ks, int cin, int cc, int cout,
                                                        int ci0, const float* __restrict__ part,
                                                        float* __restrict__ out, int accumulate) {
  const int nt = ks * ks;
  const int nw = cout * nt * cc, nout = nw + (ci0 == 0 ? cout : 0);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout) return;
  float acc = 0.f;
  for (int b = 0; b < nblocks; ++b) acc += part[(size_t)b * nout + e];
  size_t idx;
  if (e < nw) {
    const int co = e / (nt * cc), rem = e % (nt * cc), tap = rem / cc, c = rem % cc;
    idx = (size_t)co * nt * cin + (size_t)tap * cin + ci0 + c;
  } else {
    idx = (size_t)cout * nt * cin + (e - nw);
  }
  out[idx] = accumulate ? out[idx] + acc : acc;
}

template <int KS, int CIN, int CC, int COUT>
static hipError_t unet_wgrad_t(int H, int W, const float* in, const float* lam_pre, float* part,
                               size_t part_n, float* dst, int accumulate, hipStream_t s) {
  constexpr int NACC = 36, BK = BT + KS - 1;
  const int tiles = ((W + BT - 1) / BT) * ((H + BT - 1) / BT);
  const int gx = min(tiles, kWgBlocks);
  const size_t lds = sizeof(float) * (BT * BT * COUT + BK * BK * CC);
  auto k = bw_wgrad_c<KS, CIN, CC, COUT, NACC>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  for (int ci0 = 0; ci0 < CIN; ci0 += CC) {
    const int nout = COUT * KS * KS * CC + (ci0 == 0 ? COUT : 0);
    if ((size_t)gx * nout > part_n) return hipErrorInvalidValue;
    const int gy = (nout + 256 * NACC - 1) / (256 * NACC);
    hipLaunchKernelGGL(k, dim3(gx, gy), dim3(256), lds, s, H, W, in, ci0, lam_pre, part);
    hipLaunchKernelGGL(bw_part_finish_c, dim3((nout + 255) / 256), dim3(256), 0, s, gx, KS, CIN, CC, COUT,
                       ci0, part, dst, accumulate);
  }
  return hipGetLastError();
}

// weight gradients of the FP32 layers of the Unet and of the cascades
static hipError_t unet_wgrad(int cin, int cout, int H, int W, const float* in, const float* lam_pre,
                             float* part, size_t part_n, float* dst, int acc, hipStream_t s) {
  if (cin == 2 && cout == 16) return unet_wgrad_t<3, 2, 2, 16>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 16 && cout == 16) return unet_wgrad_t<3, 16, 16, 16>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 16 && cout == 64) return unet_wgrad_t<3, 16, 16, 64>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 64 && cout == 64) return unet_wgrad_t<3, 64, 64, 64>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 128 && cout == 64) return unet_wgrad_t<3, 128, 64, 64>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 80 && cout == 16) return unet_wgrad_t<3, 80, 80, 16>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 32 && cout == 16) return unet_wgrad_t<3, 32, 32, 16>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 64 && cout == 32) return unet_wgrad_t<3, 64, 64, 32>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 32 && cout == 64) return unet_wgrad_t<3, 32, 32, 64>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  if (cin == 32 && cout == 32) return unet_wgrad_t<3, 32, 32, 32>(H, W, in, lam_pre, part, part_n, dst, acc, s);
  return hipErrorInvalidValue;
}

// input gradient; mask: multiply by (h_in > 0), the ReLU of the input map
static hipError_t unet_dgrad(int cin, int cout, bool mask, int H, int W, const float* lam_pre,
                             const float* Wt, const float* h_in, float* lam_in, hipStream_t s) {
  if (cin == 16 && cout == 16)
    return mask ? dgrad_layer<float, 16, 16, true, false>(H, W, lam_pre, Wt, h_in, lam_in, s)
                : dgrad_layer<float, 16, 16, false, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  if (cin == 64 && cout == 64)
    return mask ? dgrad_layer<float, 64, 64, true, false>(H, W, lam_pre, Wt, h_in, lam_in, s)
                : dgrad_layer<float, 64, 64, false, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  if (cin == 32 && cout == 32 && mask) return dgrad_layer<float, 32, 32, true, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  if (cin == 64 && cout == 32 && mask) return dgrad_layer<float, 64, 32, true, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  if (cin == 32 && cout == 64 && mask) return dgrad_layer<float, 32, 64, true, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  if (mask) return hipErrorInvalidValue;
  if (cin == 16 && cout == 64) return dgrad_layer<float, 16, 64, false, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  if (cin == 128 && cout == 64) return dgrad_layer<float, 128, 64, false, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  if (cin == 80 && cout == 16) return dgrad_layer<float, 80, 16, false, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  if (cin == 32 && cout == 16) return dgrad_layer<float, 32, 16, false, false>(H, W, lam_pre, Wt, h_in, lam_in, s);
  return hipErrorInvalidValue;
}

// channels [0, C) of a map with `istr` elements per pixel into a contiguous map
__global__ __launch_bounds__(256) void unet_skip_copy(size_t npx, int C, const float* __restrict__ src,
                                                      int istr, float* __restrict__ dst) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= npx * C) return;
  dst[gid] = src[(gid / C) * istr + gid % C];
}

// Max-pooling adjoint at fine scale (H, W, C): a fine element receives its
// window's gradient when it is the window's maximum (the first of the
// window, row-major, that attains it); plus the skip gradient; times the
// ReLU mask of the encoder output c2 (channels [0, C) of a map with
// `istr` elements per pixel).
__global__ __launch_bounds__(256) void unet_pool_bw(int H, int W, int C, const float* __restrict__ c2,
                                                    int istr, const float* __restrict__ lam_pool,
                                                    const float* __restrict__ skip,
                                                    float* __restrict__ out) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)H * W * C) return;
  const int c = (int)(gid % C);
  const size_t px = gid / C;
  const int x = (int)(px % W), y = (int)(px / W);
  const int X = x >> 1, Y = y >> 1, Wo = W >> 1;
  const float* wnd = c2 + ((size_t)(2 * Y) * W + 2 * X) * istr + c;
  const float v0 = wnd[0], v1 = wnd[istr], v2 = wnd[(size_t)W * istr], v3 = wnd[(size_t)W * istr + istr];
  const float m = fmaxf(fmaxf(v0, v1), fmaxf(v2, v3));
  const int first = v0 == m ? 0 : (v1 == m ? 1 : (v2 == m ? 2 : 3));
  const int me = (y & 1) * 2 + (x & 1);
  float g = skip[gid];
  if (me == first) g += lam_pool[((size_t)Y * Wo + X) * C + c];
  out[gid] = c2[px * istr + c] > 0.f ? g : 0.f;
}

// Upsampling adjoint: coarse (Hc, Wc, C) from the fine gradient's channels
// [off, off + C) (`istr` per pixel), times the ReLU mask of the coarse map
// `act` (none when act is null).
__global__ __launch_bounds__(256) void unet_up_bw(int Hc, int Wc, int C, const float* __restrict__ fine,
                                                  int istr, int off, const float* __restrict__ act,
                                                  float* __restrict__ out) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)Hc * Wc * C) return;
  const int c = (int)(gid % C);
  const size_t px = gid / C;
  const int X = (int)(px % Wc), Y = (int)(px / Wc);
  const int Hf = 2 * Hc, Wf = 2 * Wc;
  float acc = 0.f;
  for (int J = max(2 * Y - 2, 0); J <= min(2 * Y + 3, Hf - 1); ++J) {
    int y0, y1;
    float fy;
    up_axis(J, Hc, &y0, &y1, &fy);
    const float wy = (y0 == Y ? 1.f - fy : 0.f) + (y1 == Y ? fy : 0.f);
    if (wy == 0.f) continue;
    for (int I = max(2 * X - 2, 0); I <= min(2 * X + 3, Wf - 1); ++I) {
      int x0, x1;
      float fx;
      up_axis(I, Wc, &x0, &x1, &fx);
      const float wx = (x0 == X ? 1.f - fx : 0.f) + (x1 == X ? fx : 0.f);
      if (wx == 0.f) continue;
      acc += wy * wx * fine[((size_t)J * Wf + I) * istr + off + c];
    }
  }
  out[gid] = (!act || act[gid] > 0.f) ? acc : 0.f;
}

static hipError_t unet_backward(int nx, int ny, const float* params, float* dparams, int acc,
                                const Ws& w, hipStream_t s) {
  const UnetSave SV = unet_save_layout(nx, ny);
  const float* save = reinterpret_cast<const float*>(w.cnn_save);
  float* skipg = reinterpret_cast<float*>(w.cnn_save);
  const float* cat = reinterpret_cast<const float*>(w.cnn_cat);
  const float* x = reinterpret_cast<const float*>(w.cnn_in);
  // parameter offsets of the layers (unet.h order)
  size_t poff[kUnetLayers + 1];
  int lcin[kUnetLayers], lcout[kUnetLayers];
  {
    int n = 0, cin = 2;
    for (int l = 0; l < kUnetLevels; ++l) {
      lcin[n] = cin; lcout[n++] = kUnetW[l];
      lcin[n] = kUnetW[l]; lcout[n++] = kUnetW[l];
      cin = kUnetW[l];
    }
    for (int l = kUnetLevels - 2; l >= 0; --l) {
      lcin[n] = kUnetW[l] + kUnetW[l + 1]; lcout[n++] = kUnetW[l];
      lcin[n] = kUnetW[l]; lcout[n++] = kUnetW[l];
    }
    lcin[n] = kUnetW[0]; lcout[n++] = 1;
    size_t o = 0;
    for (int i = 0; i < kUnetLayers; ++i) {
      poff[i] = o;
      const int k = i == kUnetLayers - 1 ? 1 : 3;
      o += (size_t)k * k * lcin[i] * lcout[i] + lcout[i];
    }
    poff[kUnetLayers] = o;
  }
  float* A = w.bw_a;
  float* B = w.bw_b;
  hipError_t e = hipSuccess;
  auto grad_of = [&](int i) { return dparams ? dparams + poff[i] : nullptr; };
  auto layer_bw = [&](int i, int H, int W, const float* in, const float* lam_pre, bool mask,
                      const float* h_in, float* lam_in) -> hipError_t {
    hipError_t r = hipSuccess;
    if (dparams) r = unet_wgrad(lcin[i], lcout[i], H, W, in, lam_pre, w.bw_part, w.bw_part_n, grad_of(i), acc, s);
    if (r != hipSuccess || !lam_in) return r;
    return unet_dgrad(lcin[i], lcout[i], mask, H, W, lam_pre, params + poff[i], h_in, lam_in, s);
  };
  // the 1x1 output: lambda of the last decoder layer's pre-activation
  const int n = nx * ny, head = kUnetLayers - 1, nbh = (n + 255) / 256;
  if ((size_t)nbh * (kUnetW[0] + 1) > w.bw_part_n) return hipErrorInvalidValue;
  hipLaunchKernelGGL((bw_head<float, 16>), dim3(nbh), dim3(256), 0, s, n, w.bw_t, save + SV.d2[0],
                     params + poff[head], A, w.bw_part);
  if (dparams)
    hipLaunchKernelGGL(bw_part_finish, dim3(1), dim3(256), 0, s, nbh, kUnetW[0] + 1, w.bw_part,
                       grad_of(head), acc);
  // decoder scales 0..3: A holds the lambda of the second layer's pre-activation
  for (int l = 0; l + 1 < kUnetLevels; ++l) {
    const int H = ny >> l, W = nx >> l, wl = kUnetW[l], wu = kUnetW[l + 1], cs = wl + wu;
    const int L2 = kUnetLayers - 2 - 2 * l, L1 = L2 - 1;
    const float* cl = cat + unet_cat_offset(nx, ny, l);
    if ((e = layer_bw(L2, H, W, save + SV.d1[l], A, true, save + SV.d1[l], B)) != hipSuccess) return e;
    if ((e = layer_bw(L1, H, W, cl, B, false, nullptr, A)) != hipSuccess) return e;
    const size_t npx = (size_t)H * W;
    hipLaunchKernelGGL(unet_skip_copy, dim3((unsigned)((npx * wl + 255) / 256)), dim3(256), 0, s, npx, wl, A,
                       cs, skipg + SV.skip_grad[l]);
    const float* coarse = l + 2 < kUnetLevels ? save + SV.d2[l + 1] : save + SV.c2_bottom;
    const size_t nc = (size_t)(H / 2) * (W / 2) * wu;
    hipLaunchKernelGGL(unet_up_bw, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, H / 2, W / 2, wu, A,
                       cs, wl, coarse, B);
    float* t = A; A = B; B = t;
  }
  // encoder scales 4..0: A holds the lambda of the second layer's pre-activation
  for (int l = kUnetLevels - 1; l >= 0; --l) {
    const int H = ny >> l, W = nx >> l, wl = kUnetW[l];
    const int L2 = 2 * l + 1, L1 = 2 * l;
    if ((e = layer_bw(L2, H, W, save + SV.c1[l], A, true, save + SV.c1[l], B)) != hipSuccess) return e;
    if (l == 0) {
      if (dparams && (e = unet_wgrad(2, wl, H, W, x, B, w.bw_part, w.bw_part_n, grad_of(L1), acc, s)) != hipSuccess)
        return e;
      if ((e = dgrad_layer<float, 2, 16, false, true>(H, W, B, params + poff[L1], nullptr, w.bw_x, s)) != hipSuccess)
        return e;
    } else {
      const int wp = kUnetW[l - 1], csp = wp + wl;
      if ((e = layer_bw(L1, H, W, save + SV.pool[l - 1], B, false, nullptr, A)) != hipSuccess) return e;
      const float* c2 = cat + unet_cat_offset(nx, ny, l - 1);
      const size_t nf = (size_t)(2 * H) * (2 * W) * wp;
      hipLaunchKernelGGL(unet_pool_bw, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, 2 * H, 2 * W, wp,
                         c2, csp, A, save + SV.skip_grad[l - 1], B);
      float* t = A; A = B; B = t;
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The cascade's backward pass (Sec. 3.1's MultiScale / SmallScale, FP32
// training).  The forward kept every branch input and layer output
// (cascade.h).  Branches from the finest to the coarsest: the 1x1 head, the
// 3x3 layers (ReLU masks of the layer below), the opening 5x5 layer down to
// the gradient of the branch input, whose channel 0 (d / s) is kept per
// scale and whose channel 2 (the up-sampled coarser output) goes through
// the transposed bilinear x2 to the coarser branch's output.  Finally the
// three channel-0 maps are summed at full resolution through the adjoints
// of the input down-sampling (to 1/2: the 2x2 mean; to 1/4: the mean of the
// central 2x2 pixels of every 4x4 block).
// ---------------------------------------------------------------------------

// Input gradient of a KS x KS layer (odd KS) with the replicate-padding
// adjoint: output pixel p reads input clamp(p + o) at tap offset o, so
// input pixel q receives every p with clamp(p + o) = q (one inside the map;
// at the first and last row or column the ones that clamp onto it).
template <int KS, int CIN, int COUT, bool MASK>
__global__ __launch_bounds__(256) void bw_dgrad_k(int H, int W, const float* __restrict__ lam_pre,
                                                  const float* __restrict__ Wt,
                                                  const float* __restrict__ h_in,
                                                  float* __restrict__ lam_in) {
  constexpr int HK = KS / 2, BK = BT + 2 * HK;
  extern __shared__ __attribute__((aligned(16))) float lds_k[];  // [BK*BK][COUT]
  const int tiles_x = (W + BT - 1) / BT;
  const int x0 = (blockIdx.x % tiles_x) * BT, y0 = (blockIdx.x / tiles_x) * BT;
  for (int e = threadIdx.x; e < BK * BK * COUT; e += 256) {
    const int q = e / COUT, co = e % COUT;
    const int gy = y0 - HK + q / BK, gx = x0 - HK + q % BK;
    lds_k[e] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? lam_pre[((size_t)gy * W + gx) * COUT + co] : 0.f;
  }
  __syncthreads();
  const int y = y0 + threadIdx.x / BT, x = x0 + threadIdx.x % BT;
  if (y >= H || x >= W) return;
  // the range [lo, hi] of output positions p with clamp(p + o) = q
  auto range = [](int q, int o, int n, int* lo, int* hi) {
    if (q > 0 && q < n - 1) {
      *lo = *hi = q - o;
      if (q - o < 0 || q - o >= n) *hi = *lo - 1;
    } else if (q == 0) {
      *lo = 0;
      *hi = o <= 0 ? min(-o, n - 1) : -1;
    } else {
      *lo = o >= 0 ? max(n - 1 - o, 0) : n;
      *hi = n - 1;
    }
  };
  float acc[CIN];
#pragma unroll
  for (int ci = 0; ci < CIN; ++ci) acc[ci] = 0.f;
  for (int ky = 0; ky < KS; ++ky) {
    int ya, yb;
    range(y, ky - HK, H, &ya, &yb);
    for (int kx = 0; kx < KS; ++kx) {
      int xa, xb;
      range(x, kx - HK, W, &xa, &xb);
      const float* wk = Wt + (ky * KS + kx) * CIN;
      for (int py = ya; py <= yb; ++py)
        for (int px = xa; px <= xb; ++px) {
          const float* lp = lds_k + ((py - y0 + HK) * BK + (px - x0 + HK)) * COUT;
          for (int co = 0; co < COUT; ++co) {
            const float l = lp[co];
            const float* wr = wk + (size_t)co * KS * KS * CIN;
#pragma unroll
            for (int ci = 0; ci < CIN; ++ci) acc[ci] += wr[ci] * l;
          }
        }
    }
  }
  const size_t pix = (size_t)y * W + x;
#pragma unroll
  for (int ci = 0; ci < CIN; ++ci) {
    float v = acc[ci];
    if (MASK) v = h_in[pix * CIN + ci] > 0.f ? v : 0.f;
    lam_in[pix * CIN + ci] = v;
  }
}

template <int KS, int CIN, int COUT>
static hipError_t dgrad_k(int H, int W, const float* lam_pre, const float* Wt, float* lam_in,
                          hipStream_t s) {
  constexpr int BK = BT + KS - 1;
  const int tiles = ((W + BT - 1) / BT) * ((H + BT - 1) / BT);
  const size_t lds = sizeof(float) * BK * BK * COUT;
  auto k = bw_dgrad_k<KS, CIN, COUT, false>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(tiles), dim3(256), lds, s, H, W, lam_pre, Wt, nullptr, lam_in);
  return hipGetLastError();
}

// the opening 5x5 layer of a branch: weight gradient and input gradient
static hipError_t pn_first_bw(int cin, int cout, int H, int W, const float* in, const float* lam_pre,
                              const float* Wt, float* part, size_t part_n, float* dst, int acc,
                              float* lam_in, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (cin == 2 && cout == 64) {
    if (dst) e = unet_wgrad_t<5, 2, 2, 64>(H, W, in, lam_pre, part, part_n, dst, acc, s);
    return e != hipSuccess ? e : dgrad_k<5, 2, 64>(H, W, lam_pre, Wt, lam_in, s);
  }
  if (cin == 3 && cout == 64) {
    if (dst) e = unet_wgrad_t<5, 3, 3, 64>(H, W, in, lam_pre, part, part_n, dst, acc, s);
    return e != hipSuccess ? e : dgrad_k<5, 3, 64>(H, W, lam_pre, Wt, lam_in, s);
  }
  if (cin == 2 && cout == 32) {
    if (dst) e = unet_wgrad_t<5, 2, 2, 32>(H, W, in, lam_pre, part, part_n, dst, acc, s);
    return e != hipSuccess ? e : dgrad_k<5, 2, 32>(H, W, lam_pre, Wt, lam_in, s);
  }
  if (cin == 3 && cout == 32) {
    if (dst) e = unet_wgrad_t<5, 3, 3, 32>(H, W, in, lam_pre, part, part_n, dst, acc, s);
    return e != hipSuccess ? e : dgrad_k<5, 3, 32>(H, W, lam_pre, Wt, lam_in, s);
  }
  return hipErrorInvalidValue;
}

// lam_x at full resolution += the adjoints of the down-sampled copies:
// a quarter of the half-resolution value of the 2x2 block, and a quarter of
// the quarter-resolution value for the central 2x2 pixels of a 4x4 block
__global__ __launch_bounds__(256) void pn_x_combine(int nx, int ny, float* __restrict__ l0,
                                                    const float* __restrict__ l1,
                                                    const float* __restrict__ l2) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  const int i = c % nx, j = c / nx;
  float a = l0[c] + 0.25f * l1[(j >> 1) * (nx >> 1) + (i >> 1)];
  const int ri = i & 3, rj = j & 3;
  if ((ri == 1 || ri == 2) && (rj == 1 || rj == 2)) a += 0.25f * l2[(j >> 2) * (nx >> 2) + (i >> 2)];
  l0[c] = a;
}

static hipError_t cascade_backward(int arch, const WsLayout& Ly, int nx, int ny, const float* params,
                                   float* dparams, int acc, const Ws& w, hipStream_t s) {
  const PnSave SV = pn_save_layout(arch, nx, ny);
  const float* save = reinterpret_cast<const float*>(w.cnn_save);
  PnLayer Lb[kPnBranches][kPnMaxLayers];
  size_t poff[kPnBranches][kPnMaxLayers];
  int nl[kPnBranches];
  size_t o = 0;
  for (int b = 0; b < kPnBranches; ++b) {
    nl[b] = pn_branch(arch, b, Lb[b]);
    for (int i = 0; i < nl[b]; ++i) {
      poff[b][i] = o;
      o += (size_t)Lb[b][i].ks * Lb[b][i].ks * Lb[b][i].cin * Lb[b][i].cout + Lb[b][i].cout;
    }
  }
  float* A = w.bw_a;
  float* B = w.bw_b;
  hipError_t e = hipSuccess;
  for (int b = kPnBranches - 1; b >= 0; --b) {
    const int k = kPnBranches - 1 - b;  // scale index, 0 = finest
    const int H = Ly.sc_h[k], W = Ly.sc_w[k], npx = H * W;
    const float* lam_y = w.bw_t + Ly.sc_off_px[k];
    // the 1x1 head; its input layer has no ReLU
    const int hi = nl[b] - 1, C = Lb[b][hi].cin, nbh = (npx + 255) / 256;
    if ((size_t)nbh * (C + 1) > w.bw_part_n) return hipErrorInvalidValue;
    const float* hin = save + SV.out[b][hi - 1];
    if (C == 64)
      hipLaunchKernelGGL((bw_head<float, 64, false>), dim3(nbh), dim3(256), 0, s, npx, lam_y, hin,
                         params + poff[b][hi], A, w.bw_part);
    else
      hipLaunchKernelGGL((bw_head<float, 32, false>), dim3(nbh), dim3(256), 0, s, npx, lam_y, hin,
                         params + poff[b][hi], A, w.bw_part);
    if (dparams)
      hipLaunchKernelGGL(bw_part_finish, dim3(1), dim3(256), 0, s, nbh, C + 1, w.bw_part,
                         dparams + poff[b][hi], acc);
    // 3x3 layers: A holds the gradient of layer i's pre-activation
    for (int i = hi - 1; i >= 1; --i) {
      const PnLayer& l = Lb[b][i];
      const float* in = save + SV.out[b][i - 1];
      if (dparams && (e = unet_wgrad(l.cin, l.cout, H, W, in, A, w.bw_part, w.bw_part_n, dparams + poff[b][i],
                                     acc, s)) != hipSuccess)
        return e;
      if ((e = unet_dgrad(l.cin, l.cout, Lb[b][i - 1].relu, H, W, A, params + poff[b][i], in, B, s)) != hipSuccess)
        return e;
      float* t = A; A = B; B = t;
    }
    // the opening 5x5 layer down to the branch input's gradient (in B)
    const PnLayer& l0 = Lb[b][0];
    if ((e = pn_first_bw(l0.cin, l0.cout, H, W, save + SV.in[b], A, params + poff[b][0], w.bw_part,
                         w.bw_part_n, dparams ? dparams + poff[b][0] : nullptr, acc, B, s)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(unet_skip_copy, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s, (size_t)npx, 1, B,
                       l0.cin, w.bw_x + Ly.sc_off_px[k]);
    if (b > 0) {
      const size_t nc = (size_t)(H / 2) * (W / 2);
      hipLaunchKernelGGL(unet_up_bw, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, H / 2, W / 2, 1, B,
                         l0.cin, 2, (const float*)nullptr, w.bw_t + Ly.sc_off_px[k + 1]);
    }
  }
  hipLaunchKernelGGL(pn_x_combine, dim3((nx * ny + 255) / 256), dim3(256), 0, s, nx, ny,
                     w.bw_x + Ly.sc_off_px[0], w.bw_x + Ly.sc_off_px[1], w.bw_x + Ly.sc_off_px[2]);
  return hipGetLastError();
}

hipError_t run_backward(const NetShape& net, const WsLayout& Ly, int nx, int ny, double dx,
                        int sweeps, float omega, double scale, bool accumulate,
                        const float* params, float* du, float* dv, float* dparams,
                        double* loss_out, const Ws& w, hipStream_t s) {
  const int n = nx * ny, nb = (n + 255) / 256;
  if ((size_t)nb > w.blockpart_n) return hipErrorInvalidValue;
  float* lamA = w.bw_cells;
  float* lamB = w.bw_cells + n;
  float* lamD = w.bw_cells + 2 * (size_t)n;
  const float inv_dx2 = (float)(1.0 / (dx * dx));
  bw_init<<<nb, 256, 0, s>>>(nx, ny, inv_dx2, (float)(2.0 * scale), w.cell, w.d, w.phi, lamA, lamD,
                             w.blockpart);
  bw_loss_finish<<<1, 256, 0, s>>>(nb, w.blockpart, scale, w.sc, loss_out);
  bw_neglap<<<nb, 256, 0, s>>>(nx, ny, inv_dx2, w.cell, lamA, lamB);
  float* cur = lamB;
  float* nxt = lamA;
  const float wdx2 = (float)(omega * dx * dx);
  for (int k = 0; k < sweeps; ++k) {
    bw_jacobi<<<nb, 256, 0, s>>>(nx, ny, omega, wdx2, w.cell, cur, nxt, lamD);
    float* t = cur; cur = nxt; nxt = t;
  }
  // CNN (the paper networks' output y is the full-resolution map phi0 = dx^2 s y)
  const bool unet = net.arch != HYP_ARCH_PARALLEL;
  bw_phi0<<<nb, 256, 0, s>>>(n, (float)(dx * dx), w.cell, cur, unet ? w.cnn_y : w.cnn_t, w.bw_t,
                             w.blockpart, w.sc);
  bw_lams_set<<<1, 256, 0, s>>>(nb, w.blockpart, dx * dx, w.sc);
  for (int k = 0; !unet && k + 1 < net.scales; ++k) {
    const int Hc = Ly.sc_h[k + 1], Wc = Ly.sc_w[k + 1];
    bw_up2T<<<(Hc * Wc + 255) / 256, 256, 0, s>>>(Hc, Wc, w.bw_t + Ly.sc_off_px[k],
                                                  w.bw_t + Ly.sc_off_px[k + 1]);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int acc = accumulate ? 1 : 0;
  if (unet) {
    if (net.precision != HYP_PREC_FP32) return hipErrorInvalidValue;
    e = net.arch == HYP_ARCH_UNET ? unet_backward(nx, ny, params, dparams, acc, w, s)
                                  : cascade_backward(net.arch, Ly, nx, ny, params, dparams, acc, w, s);
  } else if (net.precision == HYP_PREC_BF16) {
    switch (net.channels) {
      case 32: e = backward_cnn<uint16_t, 32>(net, Ly, nx, ny, params, dparams, acc, w, s); break;
      case 64: e = backward_cnn<uint16_t, 64>(net, Ly, nx, ny, params, dparams, acc, w, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (net.channels) {
      case 16: e = backward_cnn<float, 16>(net, Ly, nx, ny, params, dparams, acc, w, s); break;
      case 32: e = backward_cnn<float, 32>(net, Ly, nx, ny, params, dparams, acc, w, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  PyrT P{};
  P.nscales = unet ? 1 : net.scales;
  for (int k = 0; k < P.nscales; ++k) P.lx[k] = w.bw_x + Ly.sc_off_px[k];
  bw_pyr_sum<<<nb, 256, 0, s>>>(nx, ny, P, w.cell, w.d, w.blockpart);
  bw_lams_add<<<1, 256, 0, s>>>(nb, w.blockpart, w.sc);
  bw_dnorm<<<nb, 256, 0, s>>>(nx, ny, P, w.cell, w.d, lamD, w.sc);
  if (du || dv)
    bw_faces<<<nb, 256, 0, s>>>(nx, ny, (float)(1.0 / dx), w.cell, lamD, du, dv, acc);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t n, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

hipError_t run_adam(float* params, const float* grads, float* m, float* v, int64_t n, int step,
                    float lr, float b1, float b2, float eps, hipStream_t s) {
  const float bc1 = (float)(1.0 - pow((double)b1, step));
  const float bc2 = (float)(1.0 - pow((double)b2, step));
  adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(params, grads, m, v, n, lr, b1, b2, eps,
                                                         bc1, bc2);
  return hipGetLastError();
}

}  // namespace hyp
