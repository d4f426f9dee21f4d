// Batched projection: many plumes of uneven grid sizes, one persistent
// Jacobi launch for all of them.  The tiles of every instance form one
// global list; each work-group walks its share of the list once per block
// of B sweeps: it loads a 64 x 4R extended tile (interior + halo of width
// B + 1) from the instance's exchange plane, runs B sweeps in registers
// (the same DPP/LDS scheme as the single-grid kernel), and writes the
// interior back with its FP64 sum of |r|.  The working set does not fit on
// chip, so the temporal blocking is what cuts the HBM traffic: one read and
// one write of the tile per B sweeps.  After each block a grid barrier,
// per-instance E_1 sums (fixed order, one work-group per instance) and stop
// decisions, and a second barrier; converged instances drop out of the list.
#include "../../include/hyproj.h"
#include "common.h"
#include "internal.h"
#include "jacobi_rows.h"

namespace hyp {

struct BatchInstDev {
  int nx, ny, ntx, tile0, ntiles, max_iters;
  float inv_dx2, wfac, omega;
  double thr;
  const uint8_t* cell;
  const float* d;
  float* phi;
  float* exch;       // two planes
  Scalars* sc;
};

struct BatchState {  // per instance, device
  int status, iters, fpar, pad;
  double E;
};

struct BatchParams {
  const BatchInstDev* inst;
  const int* tile_inst;  // instance of each global tile
  int ninst, ntiles, H;
  double* tile_part;     // [2][ntiles]
  BatchState* st;
  unsigned* sync;
};

template <int R>
__device__ __forceinline__ double batch_tile(const BatchInstDev& I, int lt, int H, int B,
                                             const float* src, float* dst, bool from_phi,
                                             float (*edge)[2][4][64], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int TW = 64 - 2 * H, TH = 4 * R - 2 * H;
  const int bx = lt % I.ntx, by = lt / I.ntx;
  const int gx = bx * TW - H + lane;
  const int gy0 = by * TH - H + wave * R;
  const bool col_in = gx >= 0 && gx < I.nx;
  const bool lane_int = lane >= H && lane < H + TW && col_in;
  unsigned imask = 0, fmask = 0;
  // scaled form of the update (jac_rows_scaled): a = omega / k, b = -omega dx^2 d / k
  float ph[R], aa[R], bb[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int er = wave * R + r, gy = gy0 + r;
    float a_ = 0.f, b_ = 0.f, p_ = 0.f;
    if (col_in && gy >= 0 && gy < I.ny) {
      // the three loads are independent (masked afterwards): one round trip
      const int g = gy * I.nx + gx;
      const uint8_t ci = I.cell[g];
      const float dv = I.d[g];
      const float pv = from_phi ? I.phi[g] : ld_agent(src + g);
      if (!(ci & C_SOLID)) {
        const float k = (float)cell_k(ci);
        a_ = I.omega / k;
        b_ = -(I.wfac / k) * dv;
        p_ = pv;
      }
      if (lane_int && er >= H && er < H + TH) {
        imask |= 1u << r;
        if (!(ci & C_SOLID)) fmask |= 1u << r;
      }
    }
    ph[r] = p_; aa[r] = a_; bb[r] = b_;
  }
  int q = 0;
  float below, above;
  auto edges_of = [&](const float (&v)[R]) {
    edge[q][0][wave][lane] = v[0];
    edge[q][1][wave][lane] = v[R - 1];
    __syncthreads();
    below = wave > 0 ? edge[q][1][wave - 1][lane] : 0.f;
    above = wave < 3 ? edge[q][0][wave + 1][lane] : 0.f;
    q ^= 1;
  };
  // sweeps in pairs (ph -> tmp -> ph: no register copies between sweeps)
  const float om1 = 1.f - I.omega;
  float tmp[R];
  int s = 0;
  for (; s + 2 <= B; s += 2) {
    edges_of(ph);
    jac_rows_scaled<R, false>(ph, tmp, aa, bb, below, above, om1);
    edges_of(tmp);
    jac_rows_scaled<R, false>(tmp, ph, aa, bb, below, above, om1);
  }
  for (; s < B; ++s) {
    edges_of(ph);
    jac_rows_scaled<R, false>(ph, tmp, aa, bb, below, above, om1);
#pragma unroll
    for (int r = 0; r < R; ++r) ph[r] = tmp[r];
  }
  edges_of(ph);
  const double acc = jac_resid_scaled<R>(ph, aa, bb, below, above, I.omega, I.inv_dx2, fmask, false);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if ((imask >> r) & 1u) st_agent(dst + (size_t)(gy0 + r) * I.nx + gx, ph[r]);
  const double t = block_sum(acc, red);
  __syncthreads();  // edge[] and red[] are reused by the next tile
  return t;
}

// at most 128 VGPRs: four work-groups per CU, so that one work-group's
// loads overlap the others' sweeps (with 3 the 8192^2 DRAM case runs 15 %
// slower)
template <int R>
__global__ __launch_bounds__(256, 4) void jacobi_batch(BatchParams P) {
  __shared__ float edge[2][2][4][64];
  __shared__ double red[4];
  const int G = gridDim.x;
  const int B = P.H - 1;
  unsigned nbar = 0;
  int par = 0;  // plane read this block (written by the previous one)
  for (int nb = 0;; ++nb) {
    // phase A: sweep every tile of a running instance
    for (int t = blockIdx.x; t < P.ntiles; t += G) {
      const int i = P.tile_inst[t];
      const BatchInstDev& I = P.inst[i];
      const int sti = __hip_atomic_load(&P.st[i].status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (sti >= 0) continue;
      const int k = __hip_atomic_load(&P.st[i].iters, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int b = nb == 0 ? 0 : min(B, I.max_iters - k);
      const double s = batch_tile<R>(I, t - I.tile0, P.H, b, I.exch + (size_t)par * I.nx * I.ny,
                                     I.exch + (size_t)(par ^ 1) * I.nx * I.ny, nb == 0, edge, red);
      if (threadIdx.x == 0) st_agent(P.tile_part + (size_t)(par ^ 1) * P.ntiles + t, s);
    }
    ++nbar;
    grid_barrier(P.sync, nbar, (unsigned)G);
    // phase B: one work-group per instance sums its tiles in order and decides
    for (int i = blockIdx.x; i < P.ninst; i += G) {
      const BatchInstDev& I = P.inst[i];
      if (__hip_atomic_load(&P.st[i].status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) continue;
      const double tot = sum_partials(P.tile_part + (size_t)(par ^ 1) * P.ntiles + I.tile0, I.ntiles, red);
      if (threadIdx.x == 0) {
        int k = P.st[i].iters;
        if (nb > 0) k += min(B, I.max_iters - k);
        const int nF = I.sc->nF;
        const double E = nF > 0 ? tot / nF : 0.0;
        int st = -1;
        if (!isfinite(E)) st = HYP_STATUS_NONFINITE;
        else if (E < I.thr) st = HYP_STATUS_OK;
        else if (k >= I.max_iters) st = HYP_STATUS_MAXITER;
        if (nb == 0) I.sc->e1_cnn = E;
        P.st[i].E = E;
        __hip_atomic_store(&P.st[i].fpar, par ^ 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&P.st[i].iters, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&P.st[i].status, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (st >= 0) {
          I.sc->iters = k;
          I.sc->status = st;
          I.sc->e1_solve = E;
        }
      }
      __syncthreads();
    }
    ++nbar;
    grid_barrier(P.sync, nbar, (unsigned)G);
    int running = 0;
    for (int i = threadIdx.x; i < P.ninst; i += blockDim.x)
      running += __hip_atomic_load(&P.st[i].status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 0;
    running = (int)block_sum((double)running, red);
    par ^= 1;
    if (running == 0) break;
  }
  // epilogue: the returned iterate of every tile into the instance's phi
  for (int t = blockIdx.x; t < P.ntiles; t += G) {
    const int i = P.tile_inst[t];
    const BatchInstDev& I = P.inst[i];
    const int fp = __hip_atomic_load(&P.st[i].fpar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float* src = I.exch + (size_t)fp * I.nx * I.ny;
    const int H = P.H, TW = 64 - 2 * H, TH = 4 * R - 2 * H;
    const int lt = t - I.tile0, bx = lt % I.ntx, by = lt / I.ntx;
    for (int e = threadIdx.x; e < TW * TH; e += blockDim.x) {
      const int gx = bx * TW + e % TW, gy = by * TH + e / TW;
      if (gx < I.nx && gy < I.ny) I.phi[gy * I.nx + gx] = ld_agent(src + gy * I.nx + gx);
    }
  }
}

__global__ void batch_reset(BatchState* st, int n, unsigned* sync) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  sync_clear(sync, i);
  if (i < n) {
    st[i].status = kStatusRunning;
    st[i].iters = 0;
    st[i].fpar = 0;
    st[i].E = 0.0;
  }
}

int batch_rows() { return 16; }

// Host view of the batch area and the launch.
struct BatchArea {
  BatchInstDev* inst;
  int* tile_inst;
  double* tile_part;
  BatchState* st;
  unsigned* sync;
};

// The one layout of the batch area: carve() places every table, and the
// area size is what carve() takes from a null base.
static BatchArea carve(void* base, int ninst, int ntiles, size_t* bytes = nullptr) {
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  size_t o = 0;
  auto take = [&](size_t n) {
    const size_t at = o;
    o = (o + n + 255) & ~(size_t)255;
    return reinterpret_cast<char*>(b + at);
  };
  BatchArea A;
  A.sync = (unsigned*)take(kSyncBytes);
  A.inst = (BatchInstDev*)take(sizeof(BatchInstDev) * ninst);
  A.tile_inst = (int*)take(sizeof(int) * ntiles);
  A.tile_part = (double*)take(sizeof(double) * 2 * ntiles);
  A.st = (BatchState*)take(sizeof(BatchState) * ninst);
  if (bytes) *bytes = o;
  return A;
}

size_t batch_area_bytes(int ninst, int ntiles) {
  size_t n = 0;
  (void)carve(nullptr, ninst, ntiles, &n);
  return n;
}

int batch_tiles_of(int nx, int ny) {
  const int H = 9, R = batch_rows();
  const int TW = 64 - 2 * H, TH = 4 * R - 2 * H;
  return ((nx + TW - 1) / TW) * ((ny + TH - 1) / TH);
}

// Upload the instance and tile tables (synchronous; done once per batch).
hipError_t batch_setup(void* area, int ninst, const int* nx, const int* ny, const double* dx,
                       const double* thr, int max_iters, float omega, const Ws* ws) {
  int ntiles = 0;
  for (int i = 0; i < ninst; ++i) ntiles += batch_tiles_of(nx[i], ny[i]);
  BatchArea A = carve(area, ninst, ntiles);
  const int H = 9, R = batch_rows(), TW = 64 - 2 * H;
  (void)R;
  BatchInstDev* hi = new BatchInstDev[ninst];
  int* ht = new int[ntiles];
  int t0 = 0;
  for (int i = 0; i < ninst; ++i) {
    BatchInstDev& I = hi[i];
    I.nx = nx[i]; I.ny = ny[i];
    I.ntx = (nx[i] + TW - 1) / TW;
    I.tile0 = t0;
    I.ntiles = batch_tiles_of(nx[i], ny[i]);
    I.max_iters = max_iters;
    I.inv_dx2 = (float)(1.0 / (dx[i] * dx[i]));
    I.wfac = (float)(omega * dx[i] * dx[i]);
    I.omega = omega;
    I.thr = thr[i];
    I.cell = ws[i].cell; I.d = ws[i].d; I.phi = ws[i].phi; I.exch = ws[i].exch; I.sc = ws[i].sc;
    for (int t = 0; t < I.ntiles; ++t) ht[t0 + t] = i;
    t0 += I.ntiles;
  }
  hipError_t e = hipMemcpy(A.inst, hi, sizeof(BatchInstDev) * ninst, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(A.tile_inst, ht, sizeof(int) * ntiles, hipMemcpyHostToDevice);
  delete[] hi;
  delete[] ht;
  return e;
}

hipError_t run_jacobi_batch(const Device& dev, void* area, int ninst, int ntiles, bool cooperative,
                            hipStream_t s) {
  BatchArea A = carve(area, ninst, ntiles);
  batch_reset<<<(ninst + 63) / 64 + 1, 64, 0, s>>>(A.st, ninst, A.sync);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchParams P{};
  P.inst = A.inst; P.tile_inst = A.tile_inst; P.ninst = ninst; P.ntiles = ntiles; P.H = 9;
  P.tile_part = A.tile_part; P.st = A.st; P.sync = A.sync;
  // as many work-groups per CU as fit (up to 4), so that one work-group's
  // loads overlap another's sweeps; every one of them is resident (the
  // occupancy query accounts for registers and LDS), which the grid barrier
  // needs, also for the plain launch used inside stream capture
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)jacobi_batch<16>, 256, 0) !=
          hipSuccess || per_cu < 1)
    per_cu = 1;
  per_cu = per_cu > 4 ? 4 : per_cu;
  int G = dev.cu * per_cu;
  G = G < kMaxCoopBlocks ? G : kMaxCoopBlocks;
  void* args[] = {&P};
  if (cooperative)
    return hipLaunchCooperativeKernel((const void*)jacobi_batch<16>, dim3(G), dim3(256), args, 0, s);
  hipLaunchKernelGGL(jacobi_batch<16>, dim3(G), dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace hyp
