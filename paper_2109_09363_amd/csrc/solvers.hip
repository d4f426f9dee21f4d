// Persistent iterative solvers of L phi = d (Eq. 3), one cooperative launch
// each (all work-groups co-resident, grid barrier of common.h):
//
//  * Jacobi (Sec. 2.2) in correction form phi <- phi - omega dx^2 r / k_c,
//    r = d - L phi.  Register-resident with temporal blocking: a work-group
//    owns a 64-column extended tile (interior + halo of width H on every
//    side), one lane per column; each of the 4 waves keeps R consecutive
//    rows of its lane's column in registers, together with d, k and the
//    update weight.  East/west neighbours move between lanes with DPP
//    wave shifts, north/south come from the same lane's registers (band
//    edges through LDS).  Every block of B <= H - 1 sweeps ends with the
//    FP64 sum of |r| over the interior, an exchange of the interior through
//    global memory and one grid barrier; the halo is then refreshed.
//    E_1 is tested at the block boundaries (every check_every sweeps and at
//    max_iters).
//  * Jacobi-preconditioned conjugate gradient with FP64 dot products: LDS
//    tiles with a one-cell halo for the search direction, three grid-wide
//    reductions per iteration, and a stop confirmed on the true residual.
// Every work-group sums the same partials in the same order, so all take
// the same stop decision at the same iteration.
#include "../../include/hyproj.h"
#include "common.h"
#include "internal.h"

namespace hyp {

__device__ __forceinline__ int decide(int k, double E, double thr, int max_iters,
                                      int check_every, int fixed_iters) {
  if (fixed_iters > 0) return k >= fixed_iters ? HYP_STATUS_OK : -1;
  if (k % check_every == 0 || k >= max_iters) {
    if (!isfinite(E)) return HYP_STATUS_NONFINITE;
    if (E < thr) return HYP_STATUS_OK;
    if (k >= max_iters) return HYP_STATUS_MAXITER;
  }
  return -1;
}

struct JacParams {
  int nx, ny, H, ntx;
  float inv_dx2, wfac;  // wfac = omega * dx^2
  double thr;
  int max_iters, check_every, fixed_iters;
  int fold_window;      // sweeps per stagnation window (0: no folds)
  int last_round;       // 1: this round may not end with a fold
  const uint8_t* cell;
  const float* d;
  float* phi;    // in: initial guess, out: returned iterate
  float* exch;   // 2 x nx*ny
  double* partial;
  Scalars* sc;
  unsigned* sync;
};

// One pass over the R rows of a lane: new value (or residual) of every cell.
// `below`/`above` are the rows just outside the band (from LDS).
template <int R, bool UPDATE>
__device__ __forceinline__ double jac_rows(float (&ph)[R], const float (&dd)[R], const float (&kk)[R],
                                           const float (&ww)[R], float below, float above,
                                           float inv_dx2, unsigned rmask) {
  float prev = below;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float c = ph[r];
    const float n = (r + 1 < R) ? ph[r + 1] : above;
    const float e = from_right(c);
    const float w = from_left(c);
    const float res = dd[r] - (((e + w) + (n + prev)) - kk[r] * c) * inv_dx2;
    prev = c;
    if (UPDATE) {
      ph[r] = c - ww[r] * res;
    } else if ((rmask >> r) & 1u) {
      acc += fabs((double)res);
    }
  }
  return acc;
}

template <int R>
__global__ __launch_bounds__(256) void jacobi_reg(JacParams p) {
  __shared__ float edge[2][2][4][64];  // [parity][low row / high row][wave][lane]
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int H = p.H, TW = 64 - 2 * H, TH = 4 * R - 2 * H;
  const int G = gridDim.x;
  const int bx = blockIdx.x % p.ntx, by = blockIdx.x / p.ntx;
  const int gx = bx * TW - H + lane;
  const int gy0 = by * TH - H + wave * R;
  const bool col_in = gx >= 0 && gx < p.nx;
  const bool lane_int = lane >= H && lane < H + TW && col_in;
  const int nF = p.sc->nF;
  if (p.sc->status >= 0) return;  // an earlier round finished the solve
  // rows of this thread inside the tile interior (and the domain): imask;
  // the fluid ones among them, which enter E_1: fmask
  unsigned imask = 0, fmask = 0;
  float ph[R], dd[R], kk[R], ww[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int er = wave * R + r, gy = gy0 + r;
    float d_ = 0.f, k_ = 0.f, w_ = 0.f, p_ = 0.f;
    if (col_in && gy >= 0 && gy < p.ny) {
      const int g = gy * p.nx + gx;
      const uint8_t ci = p.cell[g];
      if (!(ci & C_SOLID)) {
        const int k = cell_k(ci);
        k_ = (float)k;
        d_ = p.d[g];
        w_ = p.wfac / (float)k;
        p_ = p.phi[g];
      }
      if (lane_int && er >= H && er < H + TH) {
        imask |= 1u << r;
        if (!(ci & C_SOLID)) fmask |= 1u << r;
      }
    }
    ph[r] = p_; dd[r] = d_; kk[r] = k_; ww[r] = w_;
  }
  int k = p.sc->iters, par = 0, q = 0;
  unsigned nbar = 0;
  const int end = p.fixed_iters > 0 ? p.fixed_iters : p.max_iters;
  const size_t plane = (size_t)p.nx * p.ny;
  const int k_start = k;
  int k_ref = k;
  double E_ref = 0.0;
  auto edges = [&](float* below, float* above) {
    edge[q][0][wave][lane] = ph[0];
    edge[q][1][wave][lane] = ph[R - 1];
    __syncthreads();
    *below = wave > 0 ? edge[q][1][wave - 1][lane] : 0.f;
    *above = wave < 3 ? edge[q][0][wave + 1][lane] : 0.f;
    q ^= 1;
  };
  for (;;) {
    float below, above;
    edges(&below, &above);
    const double loc = jac_rows<R, false>(ph, dd, kk, ww, below, above, p.inv_dx2, fmask);
    float* ex = p.exch + par * plane;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if ((imask >> r) & 1u) st_agent(ex + (size_t)(gy0 + r) * p.nx + gx, ph[r]);
    const double tot_local = block_sum(loc, red);
    double* part = p.partial + par * kMaxCoopBlocks;
    if (threadIdx.x == 0) st_agent(part + blockIdx.x, tot_local);
    ++nbar;
    grid_barrier(p.sync, nbar, (unsigned)G);
    const double tot = sum_partials(part, G, red);
    const double E = nF > 0 ? tot / nF : 0.0;
    if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) p.sc->e1_cnn = E;
    int st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
    if (k == k_start) E_ref = E;
    if (st < 0 && !p.last_round && p.fold_window > 0 && k - k_ref >= p.fold_window) {
      // stagnation window: fold when E_1 fell by less than 1 % (always in
      // fixed-sweep mode, where folds only re-base the same iteration)
      if (p.fixed_iters > 0 || !(E < 0.99 * E_ref)) st = kStatusFold;
      k_ref = k;
      E_ref = E;
    }
    if (st != -1) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((imask >> r) & 1u) p.phi[(size_t)(gy0 + r) * p.nx + gx] = ph[r];
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.sc->iters = k;
        p.sc->status = st;
        p.sc->e1_solve = E;
      }
      return;
    }
    int B = min(H - 1, end - k);
    if (p.fixed_iters <= 0) B = min(B, p.check_every - k % p.check_every);
    // refresh every non-interior cell from the neighbours' interiors
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((imask >> r) & 1u) continue;
      if (kk[r] > 0.f) ph[r] = ld_agent(ex + (size_t)(gy0 + r) * p.nx + gx);
    }
    for (int s = 0; s < B; ++s) {
      edges(&below, &above);
      jac_rows<R, true>(ph, dd, kk, ww, below, above, p.inv_dx2, 0u);
    }
    k += B;
    par ^= 1;
  }
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned CG on A x = b, A = -dx^2 L (diagonal k_c, -1 per
// non-solid neighbour), b = -dx^2 d, M = diag(k_c).  LDS holds x, r, p (with
// a 1-wide halo for p) and k per tile; vectors are FP32, dot products FP64.
// ---------------------------------------------------------------------------
struct PcgParams {
  int nx, ny, T, TH, ntx;
  float dx2;
  double thr, inv_dx2;
  int max_iters, check_every, fixed_iters;
  int last_round;
  const uint8_t* cell;
  const float* d;
  float* phi;
  float* exch;
  double* partial;
  Scalars* sc;
  unsigned* sync;
};

#define REGION_LOOP(Y0, Y1, X0, X1)                              \
  for (int ly = (Y0) + ty; ly < (Y1); ly += 4)                  \
    for (int lx = (X0) + tx; lx < (X1); lx += 64)

__global__ __launch_bounds__(256) void pcg_persist(PcgParams p) {
  extern __shared__ float smem[];
  __shared__ double red[4];
  const int EX = p.T + 2, EY = p.TH + 2, NE = EX * EY;
  float* xl = smem;
  float* rl = xl + NE;
  float* pl = rl + NE;
  float* kl = pl + NE;
  const int G = gridDim.x;
  const int ox = (blockIdx.x % p.ntx) * p.T - 1;
  const int oy = (blockIdx.x / p.ntx) * p.TH - 1;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  unsigned nbar = 0;
  const int nF = p.sc->nF;
  if (p.sc->status >= 0) return;  // an earlier round finished the solve
  const int round0 = p.sc->iters == 0;
  double* part_rz = p.partial;
  double* part_ra = p.partial + kMaxCoopBlocks;
  double* part_pq = p.partial + 2 * kMaxCoopBlocks;
  const size_t plane = (size_t)p.nx * p.ny;
  float* pex = p.exch;          // search-direction halo exchange
  float* xex = p.exch + plane;  // iterate halo exchange (true-residual check)

  REGION_LOOP(0, EY, 0, EX) {
    const int gx = ox + lx, gy = oy + ly, l = ly * EX + lx;
    float kk = 0.f, xx = 0.f;
    if (gx >= 0 && gx < p.nx && gy >= 0 && gy < p.ny) {
      const int g = gy * p.nx + gx;
      const uint8_t ci = p.cell[g];
      if (!(ci & C_SOLID)) {
        kk = (float)cell_k(ci);
        xx = p.phi[g];
      }
    }
    xl[l] = xx;
    kl[l] = kk;
    pl[l] = 0.f;
    rl[l] = 0.f;
  }
  __syncthreads();
  // r = b - A x, p = z = r / k
  double rz = 0.0, ra = 0.0;
  REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
    const int l = ly * EX + lx;
    if (kl[l] > 0.f) {
      const int g = (oy + ly) * p.nx + (ox + lx);
      const float b = -p.dx2 * p.d[g];
      const float Ax = kl[l] * xl[l] - ((xl[l - 1] + xl[l + 1]) + (xl[l - EX] + xl[l + EX]));
      const float r = b - Ax;
      const float z = r / kl[l];
      rl[l] = r;
      pl[l] = z;
      rz += (double)r * (double)z;
      ra += fabs((double)r);
    }
  }
  rz = block_sum(rz, red);
  ra = block_sum(ra, red);
  if (threadIdx.x == 0) {
    st_agent(part_rz + blockIdx.x, rz);
    st_agent(part_ra + blockIdx.x, ra);
  }
  ++nbar;
  grid_barrier(p.sync, nbar, (unsigned)G);
  double rho = sum_partials(part_rz, G, red);
  double E = nF > 0 ? sum_partials(part_ra, G, red) / nF * p.inv_dx2 : 0.0;
  if (round0 && blockIdx.x == 0 && threadIdx.x == 0) p.sc->e1_cnn = E;
  int k = p.sc->iters;
  auto finish = [&](int st) {
    REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
      const int gx = ox + lx, gy = oy + ly;
      if (gx < p.nx && gy < p.ny) p.phi[gy * p.nx + gx] = xl[ly * EX + lx];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      p.sc->iters = k;
      p.sc->status = st;
      p.sc->e1_solve = E;
    }
  };
  for (;;) {
    int st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
    if (st < 0 && !(rho > 0.0)) st = HYP_STATUS_OK;  // r = 0 exactly
    if (st == HYP_STATUS_OK && p.fixed_iters <= 0) {
      // The updated residual drifts from b - A x in FP32: confirm the stop on
      // the true residual; if it fails, continue from it with p = z (restart).
      REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
        const int gx = ox + lx, gy = oy + ly;
        if (gx < p.nx && gy < p.ny) st_agent(xex + gy * p.nx + gx, xl[ly * EX + lx]);
      }
      ++nbar;
      grid_barrier(p.sync, nbar, (unsigned)G);
      REGION_LOOP(0, EY, 0, EX) {
        if (ly >= 1 && ly < 1 + p.TH && lx >= 1 && lx < 1 + p.T) continue;
        const int l = ly * EX + lx;
        xl[l] = kl[l] > 0.f ? ld_agent(xex + (oy + ly) * p.nx + (ox + lx)) : 0.f;
      }
      __syncthreads();
      double rzt = 0.0, rat = 0.0;
      REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
        const int l = ly * EX + lx;
        if (kl[l] > 0.f) {
          const int g = (oy + ly) * p.nx + (ox + lx);
          const float b = -p.dx2 * p.d[g];
          const float Ax = kl[l] * xl[l] - ((xl[l - 1] + xl[l + 1]) + (xl[l - EX] + xl[l + EX]));
          const float r = b - Ax;
          rl[l] = r;
          rzt += (double)r * (double)(r / kl[l]);
          rat += fabs((double)r);
        }
      }
      rzt = block_sum(rzt, red);
      rat = block_sum(rat, red);
      if (threadIdx.x == 0) {
        st_agent(part_rz + blockIdx.x, rzt);
        st_agent(part_ra + blockIdx.x, rat);
      }
      ++nbar;
      grid_barrier(p.sync, nbar, (unsigned)G);
      rho = sum_partials(part_rz, G, red);
      E = nF > 0 ? sum_partials(part_ra, G, red) / nF * p.inv_dx2 : 0.0;
      st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
      if (st < 0 && !(rho > 0.0)) st = HYP_STATUS_OK;
      if (st < 0 && !p.last_round) st = kStatusFold;  // fold, then CG on the new residual
      if (st < 0) {
        REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
          const int l = ly * EX + lx;
          pl[l] = kl[l] > 0.f ? rl[l] / kl[l] : 0.f;
        }
        __syncthreads();
      }
    }
    if (st != -1) {
      finish(st);
      return;
    }
    // exchange p
    REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
      const int gx = ox + lx, gy = oy + ly;
      if (gx < p.nx && gy < p.ny) st_agent(pex + gy * p.nx + gx, pl[ly * EX + lx]);
    }
    ++nbar;
    grid_barrier(p.sync, nbar, (unsigned)G);
    REGION_LOOP(0, EY, 0, EX) {
      if (ly >= 1 && ly < 1 + p.TH && lx >= 1 && lx < 1 + p.T) continue;
      const int l = ly * EX + lx;
      pl[l] = kl[l] > 0.f ? ld_agent(pex + (oy + ly) * p.nx + (ox + lx)) : 0.f;
    }
    __syncthreads();
    // q = A p kept in registers (each thread revisits the same cells)
    float qv[16];
    double pq = 0.0;
    int n = 0;
    REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
      const int l = ly * EX + lx;
      float q = 0.f;
      if (kl[l] > 0.f) {
        q = kl[l] * pl[l] - ((pl[l - 1] + pl[l + 1]) + (pl[l - EX] + pl[l + EX]));
        pq += (double)pl[l] * (double)q;
      }
      qv[n++ & 15] = q;
    }
    pq = block_sum(pq, red);
    if (threadIdx.x == 0) st_agent(part_pq + blockIdx.x, pq);
    ++nbar;
    grid_barrier(p.sync, nbar, (unsigned)G);
    const double pqt = sum_partials(part_pq, G, red);
    if (!(pqt > 0.0)) {  // breakdown or p = 0: return the current iterate
      finish(isfinite(pqt) ? HYP_STATUS_OK : HYP_STATUS_NONFINITE);
      return;
    }
    const float alpha = (float)(rho / pqt);
    double rz2 = 0.0, ra2 = 0.0;
    n = 0;
    REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
      const int l = ly * EX + lx;
      const float q = qv[n++ & 15];
      if (kl[l] > 0.f) {
        xl[l] += alpha * pl[l];
        const float r = rl[l] - alpha * q;
        rl[l] = r;
        const float z = r / kl[l];
        rz2 += (double)r * (double)z;
        ra2 += fabs((double)r);
      }
    }
    rz2 = block_sum(rz2, red);
    ra2 = block_sum(ra2, red);
    if (threadIdx.x == 0) {
      st_agent(part_rz + blockIdx.x, rz2);
      st_agent(part_ra + blockIdx.x, ra2);
    }
    ++nbar;
    grid_barrier(p.sync, nbar, (unsigned)G);
    const double rho_new = sum_partials(part_rz, G, red);
    E = nF > 0 ? sum_partials(part_ra, G, red) / nF * p.inv_dx2 : 0.0;
    const float beta = (float)(rho != 0.0 ? rho_new / rho : 0.0);
    REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
      const int l = ly * EX + lx;
      if (kl[l] > 0.f) pl[l] = rl[l] / kl[l] + beta * pl[l];
    }
    __syncthreads();
    rho = rho_new;
    ++k;
  }
}

// ---------------------------------------------------------------------------
// Launch geometry.  Jacobi: halo H = B + 1 with B = min(check_every, 8)
// sweeps per block (8 for fixed_iters), tile interior (64 - 2H) x (4R - 2H),
// the smallest R whose tile count fits one work-group per CU.
static int jacobi_block_len(int check_every, int fixed_iters) {
  const int kMaxBlock = 8;
  if (fixed_iters > 0) return kMaxBlock;
  return check_every < kMaxBlock ? check_every : kMaxBlock;
}

static const int kRows[] = {4, 8, 12, 16, 24, 32};

static bool jacobi_geom(const Device& dev, int nx, int ny, int check_every, int fixed_iters,
                        int* R, int* H, int* ntx, int* nty) {
  const int h = jacobi_block_len(check_every, fixed_iters) + 1;
  const int tw = 64 - 2 * h;
  const int tx = (nx + tw - 1) / tw;
  const int cap = dev.cu < kMaxCoopBlocks ? dev.cu : kMaxCoopBlocks;
  for (int r : kRows) {
    const int th = 4 * r - 2 * h;
    if (th < 1) continue;
    const int ty = (ny + th - 1) / th;
    if (tx * ty <= cap) {
      *R = r; *H = h; *ntx = tx; *nty = ty;
      return true;
    }
  }
  return false;
}

// PCG: the smallest square tile side (>= 16) whose tile count fits.
static bool pcg_geom(const Device& dev, int nx, int ny, int* T, int* ntx, int* nty, size_t* lds) {
  for (int t = 16; t <= 64; t *= 2) {
    const int tx = (nx + t - 1) / t, ty = (ny + t - 1) / t;
    const size_t bytes = (size_t)4 * (t + 2) * (t + 2) * sizeof(float);
    if (bytes + 1024 > (size_t)dev.max_lds) return false;
    if (tx * ty <= dev.cu && tx * ty <= kMaxCoopBlocks) {
      *T = t; *ntx = tx; *nty = ty; *lds = bytes;
      return true;
    }
  }
  return false;
}

bool solver_fits(const Device& dev, int nx, int ny, bool pcg, int check_every, int fixed_iters) {
  if (pcg) {
    int T, ntx, nty;
    size_t lds;
    return pcg_geom(dev, nx, ny, &T, &ntx, &nty, &lds);
  }
  int R, H, ntx, nty;
  return jacobi_geom(dev, nx, ny, check_every, fixed_iters, &R, &H, &ntx, &nty);
}

template <int R>
static hipError_t launch_jacobi(JacParams& p, int G, hipStream_t s) {
  void* args[] = {&p};
  return hipLaunchCooperativeKernel((const void*)jacobi_reg<R>, dim3(G), dim3(256), args, 0, s);
}

hipError_t run_jacobi(const Device& dev, int nx, int ny, double dx, double thr, float omega,
                      int max_iters, int check_every, int fixed_iters, int fold_window,
                      int round, const Ws& w, hipStream_t s) {
  JacParams p{};
  int R = 0, H = 0, ntx = 0, nty = 0;
  if (!jacobi_geom(dev, nx, ny, check_every, fixed_iters, &R, &H, &ntx, &nty))
    return hipErrorInvalidValue;
  p.nx = nx; p.ny = ny; p.H = H; p.ntx = ntx;
  p.inv_dx2 = (float)(1.0 / (dx * dx));
  p.wfac = (float)(omega * dx * dx);
  p.thr = thr;
  p.max_iters = max_iters; p.check_every = check_every; p.fixed_iters = fixed_iters;
  p.fold_window = fold_window > 0 ? fold_window : (fixed_iters > 0 ? 0 : 1024);
  p.last_round = round + 1 >= kSolveRounds;
  p.cell = w.cell; p.d = w.d; p.phi = w.phi; p.exch = w.exch; p.partial = w.partial; p.sc = w.sc;
  p.sync = w.sync;
  const int G = ntx * nty;
  switch (R) {
    case 4: return launch_jacobi<4>(p, G, s);
    case 8: return launch_jacobi<8>(p, G, s);
    case 12: return launch_jacobi<12>(p, G, s);
    case 16: return launch_jacobi<16>(p, G, s);
    case 24: return launch_jacobi<24>(p, G, s);
    case 32: return launch_jacobi<32>(p, G, s);
  }
  return hipErrorInvalidValue;
}

hipError_t run_pcg(const Device& dev, int nx, int ny, double dx, double thr, int max_iters,
                   int check_every, int fixed_iters, int round, const Ws& w, hipStream_t s) {
  PcgParams p{};
  p.nx = nx; p.ny = ny;
  int T = 0, ntx = 0, nty = 0;
  size_t lds = 0;
  if (!pcg_geom(dev, nx, ny, &T, &ntx, &nty, &lds)) return hipErrorInvalidValue;
  p.T = p.TH = T; p.ntx = ntx;
  p.dx2 = (float)(dx * dx);
  p.inv_dx2 = 1.0 / (dx * dx);
  p.thr = thr;
  p.max_iters = max_iters; p.check_every = check_every; p.fixed_iters = fixed_iters;
  p.last_round = round + 1 >= kSolveRounds;
  p.cell = w.cell; p.d = w.d; p.phi = w.phi; p.exch = w.exch; p.partial = w.partial; p.sc = w.sc;
  p.sync = w.sync;
  hipError_t e = hipFuncSetAttribute((const void*)pcg_persist,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&p};
  return hipLaunchCooperativeKernel((const void*)pcg_persist, dim3(ntx * nty), dim3(256), args,
                                    (unsigned)lds, s);
}

}  // namespace hyp
