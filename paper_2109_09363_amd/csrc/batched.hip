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
//
// The tile height R is chosen per instance (the tuned table of the batch
// for its grid side, or forced for tuning), and an instance may use the
// variable-density operator (face weights beta = rho0 / rho_face, R = 8).
// Every wait is bounded: a work-group that gives up marks every running
// instance ABORTED and the launch ends.
#include <vector>

#include "../../include/hyproj.h"
#include "batch.h"
#include "common.h"
#include "internal.h"
#include "jacobi_rows.h"
#include "batch_tile_table.h"

namespace hyp {

constexpr int kBatchH = kBatchSweeps + 1;  // halo of a pass

struct BatchInstDev {
  int nx, ny, ntx, tile0, ntiles, max_iters, R, var;
  float inv_dx2, wfac, omega;
  double thr;
  const uint8_t* cell;
  const float* d;
  float* phi;
  float* exch;       // two planes
  Scalars* sc;
  const float* ce;   // variable density: beta of each cell's east face
  const float* cn;   // ... north face
};

struct BatchState {  // per instance, device
  int status, iters, fpar, pad;
  double E;
};

struct BatchParams {
  const BatchInstDev* inst;
  const int* tile_inst;  // instance of each global tile
  int ninst, ntiles;
  double* tile_part;     // [2][ntiles]
  BatchState* st;
  unsigned* sync;
  int test_passes;       // E_1 tested every test_passes passes of B sweeps,
  int max_iters;         // on the first pass and once B * pass >= max_iters
};

template <int R, bool VAR>
__device__ __forceinline__ double batch_tile(const BatchInstDev& I, int lt, int B, const float* src,
                                             float* dst, bool from_phi, bool test,
                                             BandEdges* edge, double* red) {
  constexpr int H = kBatchH;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // tile bx, by covers columns bx TW .. bx TW + 63 and rows by TH .. by TH +
  // 4R - 1, its interior H cells short of each side with a neighbouring
  // tile (none at the grid's edges, where the cells outside stay zero)
  const int TW = 64 - 2 * H, TH = 4 * R - 2 * H;
  const int bx = lt % I.ntx, by = lt / I.ntx, nty = I.ntiles / I.ntx;
  const int gx = bx * TW + lane;
  const int gy0 = by * TH + wave * R;
  const bool col_in = gx < I.nx;
  const bool lane_int = lane >= (bx == 0 ? 0 : H) && lane < (bx == I.ntx - 1 ? 64 : 64 - H) && col_in;
  const int row_lo = by == 0 ? 0 : H, row_hi = by == nty - 1 ? 4 * R : 4 * R - H;
  unsigned imask = 0, fmask = 0;
  // scaled forms of the update (jacobi_rows.h): constant coefficients keep
  // aa = omega / k and bb = -omega dx^2 d / k; VAR keeps aa = k, bb and the
  // face weights beta' = omega beta / k
  float ph[R], aa[R], bb[R];
  float be[VAR ? R : 1], bw[VAR ? R : 1], bn[VAR ? R : 1], bs[VAR ? R : 1];
  // every load of the tile is issued before the first is used (one round
  // trip; with the uses in the same loop the compiler waited row by row):
  // flags, d and phi of the in-domain rows, then the face coefficients of
  // the variable-density operator (a second round trip, they depend on the
  // flags)
  // (out-of-domain rows load cell 0 and are masked, so that no branch
  // separates the loads)
  unsigned dmask = 0;
  uint8_t ci[R];
  float dv[R];
  const float* sp = from_phi ? I.phi : src;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = gy0 + r;
    const bool in = col_in && gy >= 0 && gy < I.ny;
    const int g = in ? gy * I.nx + gx : 0;
    dmask |= in ? 1u << r : 0u;
    const uint8_t c_ = gld(I.cell + g);
    const float d_ = gld(I.d + g), p_ = ld_agent(sp + g);
    ci[r] = in ? c_ : (uint8_t)C_SOLID;
    dv[r] = d_;
    ph[r] = p_;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int er = wave * R + r, g = (gy0 + r) * I.nx + gx;
    const bool fl = !(ci[r] & C_SOLID);
    float a_ = 0.f, b_ = 0.f;
    if constexpr (VAR) {
      be[r] = bw[r] = bn[r] = bs[r] = 0.f;
      if (fl) {
        be[r] = (ci[r] & C_E) ? gld(I.ce + g) : 0.f;
        bw[r] = (ci[r] & C_W) ? gld(I.ce + g - 1) : 0.f;
        bn[r] = (ci[r] & C_N) ? gld(I.cn + g) : 0.f;
        bs[r] = (ci[r] & C_S) ? gld(I.cn + g - I.nx) : 0.f;
      }
    }
    if (fl) {
      if constexpr (VAR) {
        const float k = (be[r] + bw[r]) + (bn[r] + bs[r]);
        const float sc = I.omega / k;
        be[r] *= sc; bw[r] *= sc; bn[r] *= sc; bs[r] *= sc;
        a_ = k;
        b_ = -(I.wfac / k) * dv[r];
      } else {
        const float k = (float)cell_k(ci[r]);
        a_ = I.omega / k;
        b_ = -(I.wfac / k) * dv[r];
      }
    } else {
      ph[r] = 0.f;
    }
    if (((dmask >> r) & 1u) && lane_int && er >= row_lo && er < row_hi) {
      imask |= 1u << r;
      if (fl) fmask |= 1u << r;
    }
    aa[r] = a_; bb[r] = b_;
  }
  int q = 0;
  float below, above;
  auto edges_of = [&](const float (&v)[R]) { band_exchange<R>(v, edge, q, wave, lane, below, above); };
  auto rows = [&](const float (&s_)[R], float (&d_)[R], float om1) {
    if constexpr (VAR) jac_rows_var_scaled<R, false>(s_, d_, be, bw, bn, bs, bb, below, above, om1);
    else jac_rows_scaled<R, false>(s_, d_, aa, bb, below, above, om1);
  };
  // sweeps in pairs (ph -> tmp -> ph: no register copies between sweeps)
  const float om1 = 1.f - I.omega;
  float tmp[R];
  int s = 0;
  for (; s + 2 <= B; s += 2) {
    edges_of(ph);
    rows(ph, tmp, om1);
    edges_of(tmp);
    rows(tmp, ph, om1);
  }
  for (; s < B; ++s) {
    edges_of(ph);
    rows(ph, tmp, om1);
#pragma unroll
    for (int r = 0; r < R; ++r) ph[r] = tmp[r];
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if ((imask >> r) & 1u) st_agent(dst + (size_t)(gy0 + r) * I.nx + gx, ph[r]);
  double t = 0.0;
  if (test) {
    edges_of(ph);
    double acc;
    if constexpr (VAR)
      acc = jac_resid_var_scaled<R>(ph, aa, be, bw, bn, bs, bb, below, above, I.omega, I.inv_dx2,
                                    fmask, false);
    else
      acc = jac_resid_scaled<R>(ph, aa, bb, below, above, I.omega, I.inv_dx2, fmask, false);
    t = block_sum(acc, red);
  }
  __syncthreads();  // edge[] and red[] are reused by the next tile
  return t;
}

// every running instance ends with ABORTED (a work-group gave up waiting)
__device__ void batch_abort(const BatchParams& P) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < P.ninst; ++i)
    __hip_atomic_fetch_max(&P.inst[i].sc->status, (int32_t)HYP_STATUS_ABORTED, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Tile variants present in a launch (bits): constant-coefficient R = 16,
// constant-coefficient R = 8, variable density (R = 8).  Each combination
// is its own instance of the kernel, so that a launch carries only the
// register footprint of the variants its instances use.
constexpr int kTileR16 = 1, kTileR8 = 2, kTileVar = 4;

template <int MODE>
__device__ __forceinline__ double batch_tile_any(const BatchInstDev& I, int lt, int B,
                                                 const float* src, float* dst, bool from_phi,
                                                 bool test, BandEdges* edge, double* red) {
  if constexpr ((MODE & kTileVar) != 0) {
    if (I.var) return batch_tile<8, true>(I, lt, B, src, dst, from_phi, test, edge, red);
  }
  if constexpr ((MODE & kTileR8) != 0) {
    if ((MODE & kTileR16) == 0 || I.R == 8)
      return batch_tile<8, false>(I, lt, B, src, dst, from_phi, test, edge, red);
  }
  if constexpr ((MODE & kTileR16) != 0)
    return batch_tile<16, false>(I, lt, B, src, dst, from_phi, test, edge, red);
  return 0.0;
}

// at most 128 VGPRs: four work-groups per CU, so that one work-group's
// loads overlap the others' sweeps (with 3 the 8192^2 DRAM case runs 15 %
// slower)
template <int MODE>
__global__ __launch_bounds__(256, 4) void jacobi_batch(BatchParams P) {
  __shared__ BandEdges edge[2];
  __shared__ double red[4];
  band_edges_clear(edge, threadIdx.x >> 6, threadIdx.x & 63);
  const int G = gridDim.x;
  const int B = kBatchH - 1;
  unsigned nbar = 0;
  int par = 0;  // plane read this block (written by the previous one)
  for (int nb = 0;; ++nb) {
    // an instance still running has swept on every pass so far: before
    // pass nb > 0 it holds min(B (nb - 1), max_iters) sweeps.  Statuses
    // change only on test passes; the others sweep and pass one barrier.
    const bool test = nb == 0 || nb % P.test_passes == 0 || B * nb >= P.max_iters;
    // phase A: sweep every tile of a running instance
    for (int t = blockIdx.x; t < P.ntiles; t += G) {
      const int i = cld_int(P.tile_inst + t);
      const BatchInstDev I = cld(P.inst, i);
      const int sti = ld_agent(&P.st[i].status);
      if (sti >= 0) continue;
      const int k = nb == 0 ? 0 : min(B * (nb - 1), I.max_iters);
      const int b = nb == 0 ? 0 : min(B, I.max_iters - k);
      const float* src = I.exch + (size_t)par * I.nx * I.ny;
      float* dst = I.exch + (size_t)(par ^ 1) * I.nx * I.ny;
      const int lt = t - I.tile0;
      const double s = batch_tile_any<MODE>(I, lt, b, src, dst, nb == 0, test, edge, red);
      if (test && threadIdx.x == 0) st_agent(P.tile_part + (size_t)(par ^ 1) * P.ntiles + t, s);
    }
    if (!grid_barrier_bounded(P.sync, ++nbar, (unsigned)G)) {
      batch_abort(P);
      return;
    }
    if (!test) {
      par ^= 1;
      continue;
    }
    // phase B: one work-group per instance sums its tiles in order and decides
    for (int i = blockIdx.x; i < P.ninst; i += G) {
      const BatchInstDev I = cld(P.inst, i);
      if (ld_agent(&P.st[i].status) >= 0) continue;
      const double tot = sum_partials(P.tile_part + (size_t)(par ^ 1) * P.ntiles + I.tile0, I.ntiles, red);
      if (threadIdx.x == 0) {
        const int k = nb == 0 ? 0 : min(B * nb, I.max_iters);
        const int nF = I.sc->nF;
        const double E = nF > 0 ? tot / nF : 0.0;
        int st = -1;
        if (!isfinite(E)) st = HYP_STATUS_NONFINITE;
        else if (E < I.thr) st = HYP_STATUS_OK;
        else if (k >= I.max_iters) st = HYP_STATUS_MAXITER;
        if (nb == 0) I.sc->e1_cnn = E;
        P.st[i].E = E;
        st_agent(&P.st[i].fpar, par ^ 1);
        st_agent(&P.st[i].iters, k);
        st_agent(&P.st[i].status, st);
        if (st >= 0) {
          I.sc->iters = k;
          I.sc->status = st;
          I.sc->e1_solve = E;
        }
      }
      __syncthreads();
    }
    if (!grid_barrier_bounded(P.sync, ++nbar, (unsigned)G)) {
      batch_abort(P);
      return;
    }
    int running = 0;
    for (int i = threadIdx.x; i < P.ninst; i += blockDim.x)
      running += ld_agent(&P.st[i].status) < 0;
    running = (int)block_sum((double)running, red);
    par ^= 1;
    if (running == 0) break;
  }
  // epilogue: the returned iterate of every tile into the instance's phi
  for (int t = blockIdx.x; t < P.ntiles; t += G) {
    const int i = cld_int(P.tile_inst + t);
    const BatchInstDev I = cld(P.inst, i);
    const int fp = ld_agent(&P.st[i].fpar);
    const float* src = I.exch + (size_t)fp * I.nx * I.ny;
    const int H = kBatchH, TW = 64 - 2 * H, TH = 4 * I.R - 2 * H;
    const int lt = t - I.tile0, bx = lt % I.ntx, by = lt / I.ntx, nty = I.ntiles / I.ntx;
    // the tile's interior (as in batch_tile)
    const int c0 = bx == 0 ? 0 : bx * TW + H, r0 = by == 0 ? 0 : by * TH + H;
    const int c1 = min(I.nx, bx * TW + (bx == I.ntx - 1 ? 64 : 64 - H));
    const int r1 = min(I.ny, by * TH + (by == nty - 1 ? 4 * I.R : 4 * I.R - H));
    const int w = c1 - c0;
    for (int e = threadIdx.x; e < w * (r1 - r0); e += blockDim.x) {
      const int gx = c0 + e % w, gy = r0 + e / w;
      gst(I.phi + gy * I.nx + gx, ld_agent(src + gy * I.nx + gx));
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

// Tile rows of an instance: VAR tiles keep four face weights per row in
// registers, so they use R = 8; otherwise the forced R, else the tuned one
// for the grid side, else 16.
int batch_rows_of(int nx, int ny, bool var, int forced) {
  if (var) return 8;
  if (forced == 8 || forced == 16) return forced;
  for (int i = 0; i < kBatchTileTableSize; ++i)
    if (kBatchTileTable[i].nx == nx && kBatchTileTable[i].ny == ny) return kBatchTileTable[i].R;
  return 16;
}

int batch_tile_mode(int n, const int* rows, bool var) {
  if (var) return kTileVar;
  int m = 0;
  for (int i = 0; i < n; ++i) m |= rows[i] == 8 ? kTileR8 : kTileR16;
  return m;
}

// tiles across a row of nx cells: tile t starts at column t TW, the last
// reaches the grid's edge
static int batch_tiles_x(int nx) {
  const int TW = 64 - 2 * kBatchH;
  return 1 + (nx > 64 ? (nx - 64 + TW - 1) / TW : 0);
}

int batch_tiles_of(int nx, int ny, int R) {
  const int TW = 64 - 2 * kBatchH, TH = 4 * R - 2 * kBatchH;
  return batch_tiles_x(nx) * (1 + (ny > 4 * R ? (ny - 4 * R + TH - 1) / TH : 0));
}

// ---------------------------------------------------------------------------
// Host side: the one layout of the batch area.  carve() places every table,
// and the area size is what carve() takes from a null base.
// ---------------------------------------------------------------------------
struct BatchArea {
  unsigned* sync;
  BInst* binst;
  hyp_result* results;
  int* ranges;           // RK_COUNT x (n + 1)
  BatchInstDev* inst;
  int* tile_inst;
  double* tile_part;
  BatchState* st;
  void* cnn;             // network descriptor tables
};

static BatchArea carve(void* base, int n, int ntiles, size_t cnn_bytes, size_t* bytes = nullptr) {
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  size_t o = 0;
  auto take = [&](size_t k) {
    const size_t at = o;
    o = (o + k + 255) & ~(size_t)255;
    return reinterpret_cast<char*>(b + at);
  };
  BatchArea A;
  A.sync = (unsigned*)take(kSyncBytes);
  A.binst = (BInst*)take(sizeof(BInst) * n);
  A.results = (hyp_result*)take(sizeof(hyp_result) * n);
  A.ranges = (int*)take(sizeof(int) * RK_COUNT * (n + 1));
  A.inst = (BatchInstDev*)take(sizeof(BatchInstDev) * n);
  A.tile_inst = (int*)take(sizeof(int) * ntiles);
  A.tile_part = (double*)take(sizeof(double) * 2 * ntiles);
  A.st = (BatchState*)take(sizeof(BatchState) * n);
  A.cnn = cnn_bytes ? (void*)take(cnn_bytes) : nullptr;
  if (bytes) *bytes = o;
  return A;
}

size_t batch_area_bytes(int n, int ntiles, size_t cnn_bytes) {
  size_t k = 0;
  (void)carve(nullptr, n, ntiles, cnn_bytes, &k);
  return k;
}

BatchDevice batch_device(void* area, int n, int ntiles, size_t cnn_bytes) {
  const BatchArea A = carve(area, n, ntiles, cnn_bytes);
  BatchDevice D;
  D.binst = A.binst;
  D.results = A.results;
  D.cnn_tables = A.cnn;
  D.ranges.first = A.ranges;
  D.ranges.n = n;
  for (int r = 0; r < RK_COUNT; ++r) D.ranges.total[r] = 0;
  return D;
}

// Upload the instance, range and tile tables (synchronous; once per batch).
hipError_t batch_setup(void* area, int n, int ntiles, size_t cnn_bytes, const BInst* binst,
                       const int* rows, const double* thr, int max_iters, float omega,
                       BatchDevice* out) {
  BatchArea A = carve(area, n, ntiles, cnn_bytes);
  std::vector<BatchInstDev> hi(n);
  std::vector<int> ht(ntiles);
  std::vector<int> hr((size_t)RK_COUNT * (n + 1), 0);
  int t0 = 0;
  for (int i = 0; i < n; ++i) {
    const BInst& B = binst[i];
    BatchInstDev& I = hi[i];
    I.nx = B.nx; I.ny = B.ny;
    I.R = rows[i];
    I.var = B.var;
    I.ntx = batch_tiles_x(B.nx);
    I.tile0 = t0;
    I.ntiles = batch_tiles_of(B.nx, B.ny, I.R);
    I.max_iters = max_iters;
    I.inv_dx2 = (float)(1.0 / (B.dx * B.dx));
    I.wfac = (float)(omega * B.dx * B.dx);
    I.omega = omega;
    I.thr = thr[i];
    I.cell = B.w.cell; I.d = B.w.d; I.phi = B.w.phi; I.exch = B.w.exch; I.sc = B.w.sc;
    I.ce = B.w.coef_e; I.cn = B.w.coef_n;
    for (int t = 0; t < I.ntiles; ++t) ht[t0 + t] = i;
    t0 += I.ntiles;
    // work-groups of each launch shape
    const int nc = B.nx * B.ny, nu = B.ny * (B.nx + 1), nv = (B.ny + 1) * B.nx;
    int cnt[RK_COUNT] = {0};
    // the cell kernels stride over their instance's cells: a bounded grid
    // keeps each instance's FP64 block partials few (as the single-grid launches)
    cnt[RK_CELL] = (nc + 255) / 256 < kStreamGrid ? (nc + 255) / 256 : kStreamGrid;
    cnt[RK_FACE] = (nu + nv + 255) / 256;
    cnt[RK_ADV] = (nc + nu + nv + 255) / 256;
    cnt[RK_REG] = B.S > 0 ? ((B.nx + 31) / 32) * ((B.ny + 31) / 32) : 0;
    for (int k = 0; k < B.S && k < kBatchMaxScales; ++k)
      cnt[RK_LVL0 + k] = (B.sc_h[k] * B.sc_w[k] + 255) / 256;
    for (int r = 0; r < RK_COUNT; ++r)
      hr[(size_t)r * (n + 1) + i + 1] = hr[(size_t)r * (n + 1) + i] + cnt[r];
  }
  if (t0 != ntiles) return hipErrorInvalidValue;
  hipError_t e = hipMemcpy(A.inst, hi.data(), sizeof(BatchInstDev) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(A.tile_inst, ht.data(), sizeof(int) * ntiles, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(A.binst, binst, sizeof(BInst) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(A.ranges, hr.data(), sizeof(int) * hr.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  *out = batch_device(area, n, ntiles, cnn_bytes);
  for (int r = 0; r < RK_COUNT; ++r) out->ranges.total[r] = hr[(size_t)r * (n + 1) + n];
  return hipSuccess;
}

static const void* jacobi_batch_kernel(int mode) {
  switch (mode) {
    case kTileR16: return (const void*)jacobi_batch<kTileR16>;
    case kTileR8: return (const void*)jacobi_batch<kTileR8>;
    case kTileR8 | kTileR16: return (const void*)jacobi_batch<kTileR8 | kTileR16>;
    case kTileVar: return (const void*)jacobi_batch<kTileVar>;
    default: return nullptr;
  }
}

hipError_t run_jacobi_batch(const Device& dev, void* area, int n, int ntiles, size_t cnn_bytes,
                            int mode, int test_passes, int max_iters, bool cooperative,
                            hipStream_t s) {
  const void* kern = jacobi_batch_kernel(mode);
  if (!kern) return hipErrorInvalidValue;
  BatchArea A = carve(area, n, ntiles, cnn_bytes);
  batch_reset<<<(n + 63) / 64 + kSyncSlots / 64 + 1, 64, 0, s>>>(A.st, n, A.sync);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchParams P{};
  P.inst = A.inst; P.tile_inst = A.tile_inst; P.ninst = n; P.ntiles = ntiles;
  P.tile_part = A.tile_part; P.st = A.st; P.sync = A.sync;
  P.test_passes = test_passes > 0 ? test_passes : 1;
  P.max_iters = max_iters;
  // as many work-groups per CU as fit (up to 4), so that one work-group's
  // loads overlap another's sweeps; the occupancy query accounts for
  // registers and LDS, so all of them are resident when the GPU runs
  // nothing else, which the grid barrier needs (inside stream capture the
  // launch is a plain one; a barrier that is not reached within its bound
  // ends the launch with ABORTED instead of hanging)
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  per_cu = per_cu > 4 ? 4 : per_cu;
  int G = dev.cu * per_cu;
  G = G < kMaxCoopBlocks ? G : kMaxCoopBlocks;
  void* args[] = {&P};
  if (cooperative) return hipLaunchCooperativeKernel(kern, dim3(G), dim3(256), args, 0, s);
  return hipLaunchKernel(kern, dim3(G), dim3(256), args, 0, s);
}

}  // namespace hyp
