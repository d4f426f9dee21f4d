// Streaming stencil kernels of the projection: planner (pocket fill and
// neighbour bits), boundary faces + divergence, initial guess, gradient
// correction (Eq. 2) and the final divergence check.
#include "../../include/hyproj.h"
#include "batch.h"
#include "common.h"
#include "internal.h"

namespace hyp {

// ---------------------------------------------------------------------------
// Planner: the fluid cells linked to the open top by 4-connected fluid
// paths (the others are enclosed pockets and become solid), neighbour bits
// and the fluid count.
//
// The sets are bit words: for row j and tile column t (64 cells), word
// j * ntx + t of `fbits` holds the fluid cells (static) and of `rbits` the
// cells linked so far, seeded with the fluid cells of the top row.  A
// cooperative flood fill over 64x64 tiles, one wave per tile (lane l owns
// row y0 + l), repeats rounds until no tile links a cell in a whole round.
// In a row, every run of fluid cells that holds a linked cell is linked
// whole at once: adding R to F sends a carry from each linked bit up through
// the rest of its run (the bits the add flips inside F), and the same on the
// bit-reversed words spreads it down.  Columns likewise, on the transposed
// tile; rows and columns alternate until neither adds a cell, so a path
// crosses a tile in as many alternations as it has turns.
// ---------------------------------------------------------------------------
constexpr int PT = 64;

__device__ __forceinline__ uint64_t run_fill_up(uint64_t r, uint64_t f) {
  return (((f + r) ^ f) & f) | r;
}
// every run of f (maximal set of adjacent bits) that meets r, r a subset of f
__device__ __forceinline__ uint64_t run_fill(uint64_t r, uint64_t f) {
  const uint64_t up = run_fill_up(r, f);
  const uint64_t dn = __builtin_bitreverse64(
      run_fill_up(__builtin_bitreverse64(r), __builtin_bitreverse64(f)));
  return up | dn;
}
// 64x64 bit transpose across the wave (bit c of lane r -> bit r of lane c):
// at stage k, lanes l and l ^ k swap the k-wide bit blocks that sit where
// bit k of the lane and of the bit index differ
__device__ __forceinline__ uint64_t transpose64(uint64_t m, int lane) {
  constexpr uint64_t keep[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                                0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int k = 32 >> s;
    const uint64_t y = __shfl_xor(m, k);
    m = (lane & k) ? ((m & ~keep[s]) | ((y >> k) & keep[s])) : ((m & keep[s]) | ((y << k) & ~keep[s]));
  }
  return m;
}

__host__ __device__ inline size_t plan_words(int nx, int ny) {
  return (size_t)ny * ((nx + PT - 1) / PT);
}

// one thread per word: the fluid bits of 64 cells of a row, and the seeds
__global__ __launch_bounds__(256) void plan_init(int nx, int ny, int ntx, const uint8_t* __restrict__ flags,
                                                 uint64_t* __restrict__ fbits, uint64_t* __restrict__ rbits,
                                                 Scalars* sc, unsigned* sync) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  sync_clear(sync, c);
  if (c == 0) {
    sc->bar = 0;
    sc->epoch = 0;
    sc->nF = 0;
    sc->plan_rounds = 0;
  }
  if (c >= ny * ntx) return;
  const int j = c / ntx, x0 = (c % ntx) * PT;
  const int w = min(PT, nx - x0);
  const uint8_t* row = flags + (size_t)j * nx + x0;
  uint64_t f = 0;
  for (int i = 0; i < w; ++i) f |= (uint64_t)((row[i] & 1) == 0) << i;
  fbits[c] = f;
  rbits[c] = j == ny - 1 ? f : 0;
}

// One tile: its linked words, seeds across its four borders (the adjacent
// tiles' edge bits, the rows below and above), closure under row and column
// runs, the grown words stored back; returns how many cells this lane linked.
__device__ __forceinline__ int flood_tile(int ny, int ntx, int nty, const uint64_t* __restrict__ fbits,
                                          uint64_t* rbits, int t, int lane) {
  const int tx = t % ntx, y0 = (t / ntx) * PT;
  const int gy = y0 + lane;
  const bool row_in = gy < ny;
  const size_t wi = (size_t)gy * ntx + tx;
  const uint64_t F = row_in ? fbits[wi] : 0;
  const uint64_t R0 = row_in ? ld_agent(rbits + wi) : 0;
  uint64_t R = R0;
  if (row_in && tx > 0) R |= F & (ld_agent(rbits + wi - 1) >> 63);
  if (row_in && tx + 1 < ntx) R |= F & (ld_agent(rbits + wi + 1) << 63);
  if (lane == 0 && y0 > 0) R |= F & ld_agent(rbits + (size_t)(y0 - 1) * ntx + tx);
  if (lane == PT - 1 && y0 + PT < ny) R |= F & ld_agent(rbits + (size_t)(y0 + PT) * ntx + tx);
  const uint64_t Fc = transpose64(F, lane);
  for (int it = 0; it < PT * PT; ++it) {  // each alternation links >= 1 cell or ends
    const uint64_t C = run_fill(transpose64(run_fill(R, F), lane), Fc);
    const uint64_t R2 = transpose64(C, lane);
    const bool grew = __ballot(R2 != R) != 0;
    R = R2;
    if (!grew) break;
  }
  if (R != R0) st_agent(rbits + wi, R);
  return __builtin_popcountll(R & ~R0);
}

__global__ __launch_bounds__(256) void plan_flood(int ny, int ntx, int nty, const uint64_t* fbits,
                                                  uint64_t* rbits, double* partial, Scalars* sc,
                                                  unsigned* sync, unsigned max_rounds) {
  __shared__ double red[4];
  const int G = gridDim.x;
  const int ntiles = ntx * nty;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned round = 0;
  for (;;) {
    double my_changes = 0.0;
    for (int t = blockIdx.x * 4 + wave; t < ntiles; t += 4 * G)
      my_changes += flood_tile(ny, ntx, nty, fbits, rbits, t, lane);
    const double tot_local = block_sum(my_changes, red);
    double* part = partial + (round & 1) * kMaxCoopBlocks;
    if (threadIdx.x == 0) st_agent(part + blockIdx.x, tot_local);
    ++round;
    if (!grid_barrier_bounded(sync, round, (unsigned)G)) {
      if (threadIdx.x == 0) sc->plan_rounds = -1;  // a work-group never arrived
      return;
    }
    const double tot = sum_partials(part, G, red);
    if (tot == 0.0 || round >= max_rounds) break;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->plan_rounds = (int)round;
}

__global__ __launch_bounds__(256) void plan_finalize(int nx, int ny, int ntx, const uint8_t* __restrict__ flags,
                                                     const uint64_t* __restrict__ rbits,
                                                     uint8_t* __restrict__ cell, Scalars* sc) {
  __shared__ double red[4];
  auto linked = [&](int i, int j) {
    return (rbits[(size_t)j * ntx + i / PT] >> (i % PT)) & 1ull;
  };
  // grid-stride over a bounded grid: one count per work-group
  double fl_count = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nx * ny; c += gridDim.x * blockDim.x) {
    const int i = c % nx, j = c / nx;
    const bool fl = linked(i, j);
    uint8_t out = fl ? 0 : C_SOLID;
    if (fl) {
      if (i + 1 < nx && linked(i + 1, j)) out |= C_E;
      if (i > 0 && linked(i - 1, j)) out |= C_W;
      if (j + 1 >= ny || linked(i, j + 1)) out |= C_N;
      if (j > 0 && linked(i, j - 1)) out |= C_S;
      if (j == 0 && (flags[c] & 2)) out |= C_INFLOW;
      fl_count += 1.0;
    }
    cell[c] = out;
  }
  const double n = block_sum(fl_count, red);
  if (threadIdx.x == 0 && n > 0.0) atomicAdd(&sc->nF, (int)n);
}

size_t plan_bytes(int nx, int ny) { return 2 * sizeof(uint64_t) * plan_words(nx, ny); }

hipError_t run_plan(const Device& dev, int nx, int ny, const uint8_t* flags, const Ws& w,
                    hipStream_t s) {
  const int n = nx * ny;
  const int ntx = (nx + PT - 1) / PT, nty = (ny + PT - 1) / PT;
  const size_t words = plan_words(nx, ny);
  uint64_t* fbits = w.reach;
  uint64_t* rbits = w.reach + words;
  const int nbw = (int)((words > (size_t)kSyncSlots ? words : (size_t)kSyncSlots) + 255) / 256;
  plan_init<<<nbw, 256, 0, s>>>(nx, ny, ntx, flags, fbits, rbits, w.sc, w.sync);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int G = (ntx * nty + 3) / 4;  // four tiles (waves) per work-group
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, plan_flood, 256, 0);
  if (e != hipSuccess) return e;
  const int cap = per_cu * dev.cu;
  if (G > cap) G = cap;
  if (G > kMaxCoopBlocks) G = kMaxCoopBlocks;
  unsigned max_rounds = (unsigned)n + 2u;
  int ny_ = ny, ntx_ = ntx, nty_ = nty;
  const uint64_t* fb = fbits;
  double* partial = w.partial;
  Scalars* sc = w.sc;
  unsigned* sync = w.sync;
  void* args[] = {&ny_, &ntx_, &nty_, &fb, &rbits, &partial, &sc, &sync, &max_rounds};
  e = hipLaunchCooperativeKernel((const void*)plan_flood, dim3(G), dim3(256), args, 0, s);
  if (e != hipSuccess) return e;
  plan_finalize<<<min((n + 255) / 256, 2048), 256, 0, s>>>(nx, ny, ntx, flags, rbits, w.cell, w.sc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Boundary faces + divergence (forward differences) + FP64 sums of |d| and
// d^2 over fluid cells.  Each thread owns one cell and writes its west and
// south faces (plus the east wall face of the last column and the open top
// face of the last row).  A cell reads its east/north faces, which their
// owners may rewrite concurrently with the identical masked value.
// The kernel bodies take the work-group's index within its grid (lb of nb)
// so that the single-grid launches and the batched ones (one launch over
// all instances, batch.h) share them.
// ---------------------------------------------------------------------------
// Grid-stride walk over the cells of an nx-wide grid that keeps the column
// and row incrementally: one division per thread instead of one per cell.
struct CellWalk {
  int c, i, j, di, dj, stride;
  __device__ CellWalk(int c0, int stride_, int nx)
      : c(c0), i(c0 % nx), j(c0 / nx), di(stride_ % nx), dj(stride_ / nx), stride(stride_) {}
  __device__ void next(int nx) {
    c += stride;
    i += di;
    j += dj;
    if (i >= nx) {
      i -= nx;
      ++j;
    }
  }
};

__device__ __forceinline__ void div_body(int lb, int nb, int nx, int ny, float inv_dx,
                                         const uint8_t* __restrict__ cell, float* u, float* v,
                                         float* __restrict__ d, double* __restrict__ blockpart,
                                         Scalars* sc, unsigned* sync, float* __restrict__ phi_acc,
                                         double* red) {
  const int c0 = lb * blockDim.x + threadIdx.x;
  const int stride = nb * blockDim.x;
  for (int i = c0; i < kSyncSlots; i += stride) sync_clear(sync, i);
  if (c0 == 0) sc->bar = 0;
  double a = 0.0, q = 0.0;
  // grid-stride: a bounded grid keeps the per-block reduction cheap at
  // DRAM-resident sizes; faces are written back only where masking changed them
#pragma unroll 4
  for (CellWalk w(c0, stride, nx); w.c < nx * ny; w.next(nx)) {
    const int c = w.c, i = w.i, j = w.j, U = nx + 1;
    phi_acc[c] = 0.f;
    const uint8_t ci = cell[c];
    const bool fl = !(ci & C_SOLID);
    const float uw0 = u[j * U + i], ue = u[j * U + i + 1];
    const float vs0 = v[j * nx + i], vn0 = v[(j + 1) * nx + i];
    const float uw = (fl && (ci & C_W)) ? uw0 : 0.f;
    const float uem = (fl && (ci & C_E)) ? ue : 0.f;
    const float vn = (fl && (ci & C_N)) ? vn0 : 0.f;
    const float vs = (j == 0) ? ((fl && (ci & C_INFLOW)) ? vs0 : 0.f) : ((fl && (ci & C_S)) ? vs0 : 0.f);
    if (uw != uw0) u[j * U + i] = uw;
    if (vs != vs0) v[j * nx + i] = vs;
    if (i == nx - 1 && ue != 0.f) u[j * U + nx] = 0.f;
    if (j == ny - 1 && vn != vn0) v[ny * nx + i] = vn;
    const float dv = fl ? ((uem - uw) + (vn - vs)) * inv_dx : 0.f;
    d[c] = dv;
    a += fabs((double)dv);
    q += (double)dv * (double)dv;
  }
  a = block_sum(a, red);
  q = block_sum(q, red);
  if (threadIdx.x == 0) {
    blockpart[2 * lb] = a;
    blockpart[2 * lb + 1] = q;
  }
}

__device__ __forceinline__ void div_finish_body(int nblocks, const double* __restrict__ blockpart,
                                                Scalars* sc, double* red) {
  double a = 0.0, q = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    a += blockpart[2 * b];
    q += blockpart[2 * b + 1];
  }
  a = block_sum(a, red);
  q = block_sum(q, red);
  if (threadIdx.x == 0) {
    const int nF = sc->nF;
    sc->sum_abs_d = a;
    sc->sum_d2 = q;
    sc->e1_init = nF > 0 ? a / nF : 0.0;
    sc->s = nF > 0 ? sqrt(q / nF) : 0.0;
    sc->e1_cnn = sc->e1_init;
    sc->iters = 0;
    sc->status = kStatusRunning;
    sc->epoch = sc->epoch % kEpochs + 1;
  }
}

__global__ __launch_bounds__(256) void div_kernel(int nx, int ny, float inv_dx,
                                                  const uint8_t* __restrict__ cell, float* u,
                                                  float* v, float* __restrict__ d,
                                                  double* __restrict__ blockpart, Scalars* sc,
                                                  unsigned* sync, float* __restrict__ phi_acc) {
  __shared__ double red[4];
  div_body(blockIdx.x, gridDim.x, nx, ny, inv_dx, cell, u, v, d, blockpart, sc, sync, phi_acc, red);
}

__global__ __launch_bounds__(256) void div_finish(int nblocks, const double* __restrict__ blockpart,
                                                  Scalars* sc) {
  __shared__ double red[4];
  div_finish_body(nblocks, blockpart, sc, red);
}

hipError_t run_div(int nx, int ny, double dx, float* u, float* v, const Ws& w, int nblocks,
                   hipStream_t s) {
  if ((size_t)2 * nblocks > w.blockpart_n) return hipErrorInvalidValue;
  nblocks = nblocks < kStreamGrid ? nblocks : kStreamGrid;
  div_kernel<<<nblocks, 256, 0, s>>>(nx, ny, (float)(1.0 / dx), w.cell, u, v, w.d, w.blockpart,
                                     w.sc, w.sync, w.phi_acc);
  div_finish<<<1, 256, 0, s>>>(nblocks, w.blockpart, w.sc);
  return hipGetLastError();
}

// phi = scale * p_init on fluid cells (0 elsewhere), or phi = 0.
__global__ __launch_bounds__(256) void init_phi_kernel(int n, const float* __restrict__ p_init,
                                                       float scale, const uint8_t* __restrict__ cell,
                                                       float* __restrict__ phi) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const bool fl = !(cell[c] & C_SOLID);
  phi[c] = (fl && p_init) ? p_init[c] * scale : 0.f;
}

hipError_t run_init_phi(int nx, int ny, const float* p_init, double scale, const Ws& w,
                        hipStream_t s) {
  const int n = nx * ny;
  init_phi_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, p_init, (float)scale, w.cell, w.phi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient correction, Eq. (2): u -= beta grad phi on the open faces each
// cell owns (west, south, and the open top face with ghost phi = 0), so no
// face is read after another thread's update; p = rho0 (phi_acc + phi) / dt.
// beta = 1 for the constant-coefficient operator (VAR = false); for the
// variable-density one beta = rho0 / rho_face from the coefficient planes
// (ce: east face of each cell, cn: north face).
// ---------------------------------------------------------------------------
template <bool VAR>
__device__ __forceinline__ void grad_body(int lb, int nb, int nx, int ny, float inv_dx, float p_scale,
                                          const uint8_t* __restrict__ cell,
                                          const float* __restrict__ phi,
                                          const float* __restrict__ phi_acc, float* u, float* v,
                                          float* __restrict__ p, const float* __restrict__ ce,
                                          const float* __restrict__ cn) {
  // four cells per pass: all their loads (clamped neighbour indices) are
  // issued before any of their stores, so that they share one round trip;
  // each cell stores its own west and south faces unconditionally,
  // corrected or as they were (no other thread writes them), and the solid
  // cells' pressure is masked with a bit-and (selects and conditional stores
  // let the compiler move loads behind branches, one round trip per cell)
  constexpr int UN = 4;
  const int n = nx * ny, U = nx + 1;
  CellWalk w(lb * blockDim.x + threadIdx.x, nb * blockDim.x, nx);
  while (w.c < n) {
    int cc[UN], ii[UN], jj[UN];
    bool ok[UN];
#pragma unroll
    for (int k = 0; k < UN; ++k) {
      ok[k] = w.c < n;
      cc[k] = ok[k] ? w.c : 0;
      ii[k] = ok[k] ? w.i : 0;
      jj[k] = ok[k] ? w.j : 0;
      w.next(nx);
    }
    uint8_t ci[UN];
    float pc[UN], pw[UN], ps[UN], pa[UN], uw[UN], vs[UN], vt[UN], bw[UN], bs[UN], bn[UN];
#pragma unroll
    for (int k = 0; k < UN; ++k) {
      const int c = cc[k], cw = c > 0 ? c - 1 : 0, cs = c >= nx ? c - nx : 0;
      ci[k] = cell[c];
      pc[k] = phi[c];
      pw[k] = phi[cw];
      ps[k] = phi[cs];
      pa[k] = phi_acc[c];
      uw[k] = u[jj[k] * U + ii[k]];
      vs[k] = v[jj[k] * nx + ii[k]];
      vt[k] = v[ny * nx + ii[k]];
      bw[k] = bs[k] = bn[k] = 1.f;
      if constexpr (VAR) {
        bw[k] = ce[cw];
        bs[k] = cn[cs];
        bn[k] = cn[c];
      }
    }
#pragma unroll
    for (int k = 0; k < UN; ++k) {
      if (!ok[k]) continue;
      const int c = cc[k], i = ii[k], j = jj[k];
      const bool fl = !(ci[k] & C_SOLID);
      const bool cw_ = fl && (ci[k] & C_W), cs_ = fl && (ci[k] & C_S);
      u[j * U + i] = cw_ ? uw[k] - bw[k] * ((pc[k] - pw[k]) * inv_dx) : uw[k];
      v[j * nx + i] = cs_ ? vs[k] - bs[k] * ((pc[k] - ps[k]) * inv_dx) : vs[k];
      if (j == ny - 1 && fl && (ci[k] & C_N)) v[ny * nx + i] = vt[k] - bn[k] * ((0.f - pc[k]) * inv_dx);
      const int keep = -(int)fl;
      p[c] = __int_as_float(__float_as_int((pa[k] + pc[k]) * p_scale) & keep);
    }
  }
}

template <bool VAR>
__global__ __launch_bounds__(256) void grad_kernel(int nx, int ny, float inv_dx, double rho0,
                                                   double dt_host, int dt_dev,
                                                   const uint8_t* __restrict__ cell,
                                                   const float* __restrict__ phi,
                                                   const float* __restrict__ phi_acc, float* u,
                                                   float* v, float* __restrict__ p,
                                                   const Scalars* sc, const float* __restrict__ ce,
                                                   const float* __restrict__ cn) {
  const float p_scale = (float)(rho0 / (dt_dev ? sc->dt : dt_host));
  grad_body<VAR>(blockIdx.x, gridDim.x, nx, ny, inv_dx, p_scale, cell, phi, phi_acc, u, v, p, ce, cn);
}

// Face coefficients of the variable-density operator: beta = rho0 / rho_f on
// the east and north faces of every non-solid cell, rho_f the mean of the
// two cells (the cell itself on the open top face), 0 on closed faces.
__device__ __forceinline__ void coef_body(int c, int nx, int ny, double rho0,
                                          const uint8_t* __restrict__ cell,
                                          const float* __restrict__ rho, float* __restrict__ ce,
                                          float* __restrict__ cn) {
  if (c >= nx * ny) return;
  const int j = c / nx;
  const uint8_t ci = cell[c];
  float e = 0.f, n = 0.f;
  if (!(ci & C_SOLID)) {
    const double rc = rho[c];
    if (ci & C_E) e = (float)(rho0 / (0.5 * (rc + (double)rho[c + 1])));
    if (ci & C_N) n = (float)(j == ny - 1 ? rho0 / rc : rho0 / (0.5 * (rc + (double)rho[c + nx])));
  }
  ce[c] = e;
  cn[c] = n;
}

__global__ __launch_bounds__(256) void coef_kernel(int nx, int ny, double rho0,
                                                   const uint8_t* __restrict__ cell,
                                                   const float* __restrict__ rho,
                                                   float* __restrict__ ce, float* __restrict__ cn) {
  coef_body(blockIdx.x * blockDim.x + threadIdx.x, nx, ny, rho0, cell, rho, ce, cn);
}

hipError_t run_coef(int nx, int ny, double rho0, const float* rho, const Ws& w, hipStream_t s) {
  const int n = nx * ny;
  coef_kernel<<<(n + 255) / 256, 256, 0, s>>>(nx, ny, rho0, w.cell, rho, w.coef_e, w.coef_n);
  return hipGetLastError();
}

// Divergence of the returned faces: FP64 sum of |div| and max |div|.
__device__ __forceinline__ void check_body(int lb, int nb, int nx, int ny, float inv_dx,
                                           const uint8_t* __restrict__ cell,
                                           const float* __restrict__ u, const float* __restrict__ v,
                                           double* __restrict__ blockpart, double* red) {
  double a = 0.0, m = 0.0;
#pragma unroll 4
  for (CellWalk w(lb * blockDim.x + threadIdx.x, nb * blockDim.x, nx); w.c < nx * ny; w.next(nx)) {
    const int c = w.c, i = w.i, j = w.j, U = nx + 1;
    // loads issued before the flags decide: the solid cells' value is masked
    // with a bit-and (a select would be turned into a branch around the
    // loads, and every unrolled cell would wait for its own)
    const uint8_t ci = cell[c];
    const float dv = ((u[j * U + i + 1] - u[j * U + i]) + (v[(j + 1) * nx + i] - v[j * nx + i])) * inv_dx;
    const long long keep = -(long long)((ci & C_SOLID) == 0);
    const double ad = __longlong_as_double(__double_as_longlong(fabs((double)dv)) & keep);
    a += ad;
    m = fmax(m, ad);
  }
  const double sum = block_sum(a, red);
  const double mx = block_max(m, red);
  if (threadIdx.x == 0) {
    blockpart[2 * lb] = sum;
    blockpart[2 * lb + 1] = mx;
  }
}

__device__ __forceinline__ void finish_body(int nblocks, const double* __restrict__ blockpart,
                                            const Scalars* sc, hyp_result* res, double* red) {
  double a = 0.0, m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    a += blockpart[2 * b];
    m = fmax(m, blockpart[2 * b + 1]);
  }
  a = block_sum(a, red);
  m = block_max(m, red);
  if (threadIdx.x == 0) {
    hyp_result r;
    r.iters = sc->iters;
    r.status = sc->status;
    r.e1_init = sc->e1_init;
    r.e1_cnn = sc->e1_cnn;
    r.e1_final = sc->nF > 0 ? a / sc->nF : 0.0;
    r.einf_final = m;
    r.s = sc->s;
    r.n_fluid = sc->nF;
    r.reserved = 0;
    r.dt = sc->dt;
    *res = r;
  }
}

__global__ __launch_bounds__(256) void check_kernel(int nx, int ny, float inv_dx,
                                                    const uint8_t* __restrict__ cell,
                                                    const float* __restrict__ u,
                                                    const float* __restrict__ v,
                                                    double* __restrict__ blockpart) {
  __shared__ double red[4];
  check_body(blockIdx.x, gridDim.x, nx, ny, inv_dx, cell, u, v, blockpart, red);
}

__global__ __launch_bounds__(256) void finish_kernel(int nblocks, const double* __restrict__ blockpart,
                                                     const Scalars* sc, hyp_result* res) {
  __shared__ double red[4];
  finish_body(nblocks, blockpart, sc, res, red);
}

hipError_t run_grad_and_finish(int nx, int ny, double dx, double rho0, double dt, bool dt_dev,
                               float* u, float* v, float* p, const Ws& w, int nblocks, void* res,
                               bool var, hipStream_t s) {
  if ((size_t)2 * nblocks > w.blockpart_n) return hipErrorInvalidValue;
  const float inv_dx = (float)(1.0 / dx);
  const int ncheck = nblocks < kStreamGrid ? nblocks : kStreamGrid;
  if (var)
    grad_kernel<true><<<ncheck, 256, 0, s>>>(nx, ny, inv_dx, rho0, dt, dt_dev ? 1 : 0, w.cell, w.phi,
                                              w.phi_acc, u, v, p, w.sc, w.coef_e, w.coef_n);
  else
    grad_kernel<false><<<ncheck, 256, 0, s>>>(nx, ny, inv_dx, rho0, dt, dt_dev ? 1 : 0, w.cell, w.phi,
                                               w.phi_acc, u, v, p, w.sc, nullptr, nullptr);
  check_kernel<<<ncheck, 256, 0, s>>>(nx, ny, inv_dx, w.cell, u, v, w.blockpart);
  finish_kernel<<<1, 256, 0, s>>>(ncheck, w.blockpart, w.sc, (hyp_result*)res);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched launches (batch.h): one grid over all instances per phase; a
// work-group finds its instance in the prefix table of its range and runs
// the same body on that instance's arrays, one work-group per 256 cells.
// The per-instance reductions that follow run one work-group per instance.
// ---------------------------------------------------------------------------
struct BLoc {
  int i, lb, nb;
};
__device__ __forceinline__ BLoc batch_loc(const int* __restrict__ first, int n) {
  BLoc l;
  l.i = batch_find(first, n, blockIdx.x);
  l.lb = blockIdx.x - first[l.i];
  l.nb = first[l.i + 1] - first[l.i];
  return l;
}

__global__ __launch_bounds__(256) void div_batch(const BInst* __restrict__ I, const int* first, int n) {
  __shared__ double red[4];
  const BLoc l = batch_loc(first, n);
  const BInst& B = I[l.i];
  div_body(l.lb, l.nb, B.nx, B.ny, (float)(1.0 / B.dx), B.w.cell, B.u, B.v, B.w.d, B.w.blockpart,
           B.w.sc, B.w.sync, B.w.phi_acc, red);
}

__global__ __launch_bounds__(256) void div_finish_batch(const BInst* __restrict__ I, const int* first) {
  __shared__ double red[4];
  const BInst& B = I[blockIdx.x];
  div_finish_body(first[blockIdx.x + 1] - first[blockIdx.x], B.w.blockpart, B.w.sc, red);
}

hipError_t run_div_batch(const BInst* I, const BatchRanges& R, hipStream_t s) {
  if (R.total[RK_CELL] > 0)
    div_batch<<<R.total[RK_CELL], 256, 0, s>>>(I, R.of(RK_CELL), R.n);
  div_finish_batch<<<R.n, 256, 0, s>>>(I, R.of(RK_CELL));
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void coef_batch(const BInst* __restrict__ I, const int* first, int n) {
  const BLoc l = batch_loc(first, n);
  const BInst& B = I[l.i];
  if (!B.var) return;
  for (int c = l.lb * blockDim.x + threadIdx.x; c < B.nx * B.ny; c += l.nb * blockDim.x)
    coef_body(c, B.nx, B.ny, B.rho0, B.w.cell, B.rho, B.w.coef_e, B.w.coef_n);
}

hipError_t run_coef_batch(const BInst* I, const BatchRanges& R, hipStream_t s) {
  if (R.total[RK_CELL] > 0) coef_batch<<<R.total[RK_CELL], 256, 0, s>>>(I, R.of(RK_CELL), R.n);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void init_phi_batch(const BInst* __restrict__ I, const int* first,
                                                      int n) {
  const BLoc l = batch_loc(first, n);
  const BInst& B = I[l.i];
  for (int c = l.lb * blockDim.x + threadIdx.x; c < B.nx * B.ny; c += l.nb * blockDim.x) B.w.phi[c] = 0.f;
}

hipError_t run_init_phi_batch(const BInst* I, const BatchRanges& R, hipStream_t s) {
  if (R.total[RK_CELL] > 0) init_phi_batch<<<R.total[RK_CELL], 256, 0, s>>>(I, R.of(RK_CELL), R.n);
  return hipGetLastError();
}

template <bool VAR>
__global__ __launch_bounds__(256) void grad_batch(const BInst* __restrict__ I, const int* first, int n,
                                                  int dt_dev) {
  const BLoc l = batch_loc(first, n);
  const BInst& B = I[l.i];
  if (B.var != (VAR ? 1 : 0)) return;
  const float p_scale = (float)(B.rho0 / (dt_dev ? B.w.sc->dt : B.dt));
  grad_body<VAR>(l.lb, l.nb, B.nx, B.ny, (float)(1.0 / B.dx), p_scale, B.w.cell, B.w.phi,
                 B.w.phi_acc, B.u, B.v, B.p, B.w.coef_e, B.w.coef_n);
}

__global__ __launch_bounds__(256) void check_batch(const BInst* __restrict__ I, const int* first, int n) {
  __shared__ double red[4];
  const BLoc l = batch_loc(first, n);
  const BInst& B = I[l.i];
  check_body(l.lb, l.nb, B.nx, B.ny, (float)(1.0 / B.dx), B.w.cell, B.u, B.v, B.w.blockpart, red);
}

__global__ __launch_bounds__(256) void finish_batch(const BInst* __restrict__ I, const int* first) {
  __shared__ double red[4];
  const BInst& B = I[blockIdx.x];
  finish_body(first[blockIdx.x + 1] - first[blockIdx.x], B.w.blockpart, B.w.sc, B.res, red);
}

hipError_t run_grad_finish_batch(const BInst* I, const BatchRanges& R, bool dt_dev, bool var,
                                 hipStream_t s) {
  const int nb = R.total[RK_CELL];
  if (nb > 0) {
    grad_batch<false><<<nb, 256, 0, s>>>(I, R.of(RK_CELL), R.n, dt_dev ? 1 : 0);
    if (var) grad_batch<true><<<nb, 256, 0, s>>>(I, R.of(RK_CELL), R.n, dt_dev ? 1 : 0);
    check_batch<<<nb, 256, 0, s>>>(I, R.of(RK_CELL), R.n);
  }
  finish_batch<<<R.n, 256, 0, s>>>(I, R.of(RK_CELL));
  return hipGetLastError();
}

}  // namespace hyp
