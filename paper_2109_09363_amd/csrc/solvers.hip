// Persistent, LDS-resident iterative solvers of L phi = d (Eq. 3):
//  * Jacobi (Sec. 2.2) in correction form phi <- phi - omega dx^2 r / k_c,
//    with temporal blocking: each work-group keeps its tile of phi, d and
//    the stencil coefficients in LDS for the whole solve, exchanges a halo of
//    width H = B + 1 through global memory once per block of B sweeps, and
//    tests the mean |r| (FP64) at the block boundaries.
//  * Jacobi-preconditioned conjugate gradient with FP64 dot products, one
//    halo exchange and three grid-wide reductions per iteration.
// Both run as one cooperative launch (all work-groups co-resident) with a
// grid barrier; every work-group sums the same partials in the same order,
// so all of them take the same stop decision at the same iteration.
#include "common.h"
#include "internal.h"
#include "../../include/hyproj.h"

namespace hyp {

struct JacParams {
  int nx, ny, T, TH, ntx, H;
  float inv_dx2, wfac;  // wfac = omega * dx^2
  double thr;
  int max_iters, check_every, fixed_iters;
  const uint8_t* cell;
  const float* d;
  float* phi;   // in: initial guess, out: returned iterate
  float* exch;  // 2 x nx*ny
  double* partial;
  Scalars* sc;
};

// threads are laid out 64 (x) by 4 (y) over a tile region
#define REGION_LOOP(Y0, Y1, X0, X1)                              \
  for (int ly = (Y0) + ty; ly < (Y1); ly += 4)                  \
    for (int lx = (X0) + tx; lx < (X1); lx += 64)

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

__global__ __launch_bounds__(256) void jacobi_persist(JacParams p) {
  extern __shared__ float smem[];
  __shared__ double red[4];
  const int EX = p.T + 2 * p.H, EY = p.TH + 2 * p.H, NE = EX * EY;
  float* bufA = smem;
  float* bufB = bufA + NE;
  float* dl = bufB + NE;
  float* wl = dl + NE;
  float* kl = wl + NE;
  const int G = gridDim.x;
  const int ox = (blockIdx.x % p.ntx) * p.T - p.H;
  const int oy = (blockIdx.x / p.ntx) * p.TH - p.H;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int H = p.H;
  const int nF = p.sc->nF;

  REGION_LOOP(0, EY, 0, EX) {
    const int gx = ox + lx, gy = oy + ly, l = ly * EX + lx;
    float dd = 0.f, kk = 0.f, ww = 0.f, ph = 0.f;
    if (gx >= 0 && gx < p.nx && gy >= 0 && gy < p.ny) {
      const int g = gy * p.nx + gx;
      const uint8_t ci = p.cell[g];
      if (!(ci & C_SOLID)) {
        const int k = cell_k(ci);
        kk = (float)k;
        dd = p.d[g];
        ww = p.wfac / (float)k;
        ph = p.phi[g];
      }
    }
    bufA[l] = ph;
    bufB[l] = 0.f;
    dl[l] = dd;
    kl[l] = kk;
    wl[l] = ww;
  }
  __syncthreads();

  float* cur = bufA;
  float* nxt = bufB;
  int k = 0, par = 0;
  unsigned nbar = 0;
  const int end = p.fixed_iters > 0 ? p.fixed_iters : p.max_iters;
  const size_t plane = (size_t)p.nx * p.ny;
  for (;;) {
    // residual of the current iterate on the tile interior, FP64 sum of |r|
    double loc = 0.0;
    float* ex = p.exch + par * plane;
    REGION_LOOP(H, H + p.TH, H, H + p.T) {
      const int l = ly * EX + lx;
      const int gx = ox + lx, gy = oy + ly;
      const float c = cur[l];
      if (kl[l] > 0.f) {
        const float r = dl[l] - (((cur[l - 1] + cur[l + 1]) + (cur[l - EX] + cur[l + EX])) - kl[l] * c) * p.inv_dx2;
        loc += fabs((double)r);
      }
      if (gx < p.nx && gy < p.ny) ex[gy * p.nx + gx] = c;
    }
    const double tot_local = block_sum(loc, red);
    double* part = p.partial + par * kMaxCoopBlocks;
    if (threadIdx.x == 0) part[blockIdx.x] = tot_local;
    ++nbar;
    grid_barrier(&p.sc->bar, nbar * (unsigned)G);
    const double tot = sum_partials(part, G, red);
    const double E = nF > 0 ? tot / nF : 0.0;
    if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) p.sc->e1_cnn = E;
    const int st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
    if (st >= 0) {
      REGION_LOOP(H, H + p.TH, H, H + p.T) {
        const int gx = ox + lx, gy = oy + ly;
        if (gx < p.nx && gy < p.ny) p.phi[gy * p.nx + gx] = cur[ly * EX + lx];
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.sc->iters = k;
        p.sc->status = st;
        p.sc->e1_solve = E;
      }
      return;
    }
    int B = min(H - 1, end - k);
    if (p.fixed_iters <= 0) B = min(B, p.check_every - k % p.check_every);
    // refresh the halo ring from the neighbours' interiors
    REGION_LOOP(0, EY, 0, EX) {
      if (ly >= H && ly < H + p.TH && lx >= H && lx < H + p.T) continue;
      const int gx = ox + lx, gy = oy + ly, l = ly * EX + lx;
      float val = 0.f;
      if (kl[l] > 0.f) val = ex[gy * p.nx + gx];
      cur[l] = val;
    }
    __syncthreads();
    for (int s = 0; s < B; ++s) {
      const int e = H - 1 - s;
      REGION_LOOP(H - e, H + p.TH + e, H - e, H + p.T + e) {
        const int l = ly * EX + lx;
        const float c = cur[l];
        const float r = dl[l] - (((cur[l - 1] + cur[l + 1]) + (cur[l - EX] + cur[l + EX])) - kl[l] * c) * p.inv_dx2;
        nxt[l] = c - wl[l] * r;
      }
      __syncthreads();
      float* t = cur;
      cur = nxt;
      nxt = t;
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
  const uint8_t* cell;
  const float* d;
  float* phi;
  float* exch;
  double* partial;
  Scalars* sc;
};

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
  double* part_rz = p.partial;
  double* part_ra = p.partial + kMaxCoopBlocks;
  double* part_pq = p.partial + 2 * kMaxCoopBlocks;

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
    part_rz[blockIdx.x] = rz;
    part_ra[blockIdx.x] = ra;
  }
  ++nbar;
  grid_barrier(&p.sc->bar, nbar * (unsigned)G);
  double rho = sum_partials(part_rz, G, red);
  double E = nF > 0 ? sum_partials(part_ra, G, red) / nF * p.inv_dx2 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) p.sc->e1_cnn = E;
  int k = 0;
  float* xex = p.exch + (size_t)p.nx * p.ny;  // second plane: x halo exchange
  for (;;) {
    int st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
    if (st < 0 && !(rho > 0.0)) st = HYP_STATUS_OK;  // r = 0 exactly
    if (st == HYP_STATUS_OK && p.fixed_iters <= 0) {
      // The updated residual drifts from b - A x in FP32: confirm the stop on
      // the true residual; if it fails, continue from it with p = z (restart).
      REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
        const int gx = ox + lx, gy = oy + ly;
        if (gx < p.nx && gy < p.ny) xex[gy * p.nx + gx] = xl[ly * EX + lx];
      }
      ++nbar;
      grid_barrier(&p.sc->bar, nbar * (unsigned)G);
      REGION_LOOP(0, EY, 0, EX) {
        if (ly >= 1 && ly < 1 + p.TH && lx >= 1 && lx < 1 + p.T) continue;
        const int l = ly * EX + lx;
        xl[l] = kl[l] > 0.f ? xex[(oy + ly) * p.nx + (ox + lx)] : 0.f;
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
        part_rz[blockIdx.x] = rzt;
        part_ra[blockIdx.x] = rat;
      }
      ++nbar;
      grid_barrier(&p.sc->bar, nbar * (unsigned)G);
      rho = sum_partials(part_rz, G, red);
      E = nF > 0 ? sum_partials(part_ra, G, red) / nF * p.inv_dx2 : 0.0;
      st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
      if (st < 0 && !(rho > 0.0)) st = HYP_STATUS_OK;
      if (st < 0) {
        REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
          const int l = ly * EX + lx;
          pl[l] = kl[l] > 0.f ? rl[l] / kl[l] : 0.f;
        }
        __syncthreads();
      }
    }
    if (st >= 0) {
      REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
        const int gx = ox + lx, gy = oy + ly;
        if (gx < p.nx && gy < p.ny) p.phi[gy * p.nx + gx] = xl[ly * EX + lx];
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.sc->iters = k;
        p.sc->status = st;
        p.sc->e1_solve = E;
      }
      return;
    }
    // exchange p
    REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
      const int gx = ox + lx, gy = oy + ly;
      if (gx < p.nx && gy < p.ny) p.exch[gy * p.nx + gx] = pl[ly * EX + lx];
    }
    ++nbar;
    grid_barrier(&p.sc->bar, nbar * (unsigned)G);
    REGION_LOOP(0, EY, 0, EX) {
      if (ly >= 1 && ly < 1 + p.TH && lx >= 1 && lx < 1 + p.T) continue;
      const int l = ly * EX + lx;
      pl[l] = kl[l] > 0.f ? p.exch[(oy + ly) * p.nx + (ox + lx)] : 0.f;
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
    if (threadIdx.x == 0) part_pq[blockIdx.x] = pq;
    ++nbar;
    grid_barrier(&p.sc->bar, nbar * (unsigned)G);
    const double pqt = sum_partials(part_pq, G, red);
    if (!(pqt > 0.0)) {  // breakdown or p = 0: return the current iterate
      st = isfinite(pqt) ? HYP_STATUS_OK : HYP_STATUS_NONFINITE;
      REGION_LOOP(1, 1 + p.TH, 1, 1 + p.T) {
        const int gx = ox + lx, gy = oy + ly;
        if (gx < p.nx && gy < p.ny) p.phi[gy * p.nx + gx] = xl[ly * EX + lx];
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.sc->iters = k;
        p.sc->status = st;
        p.sc->e1_solve = E;
      }
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
      part_rz[blockIdx.x] = rz2;
      part_ra[blockIdx.x] = ra2;
    }
    ++nbar;
    grid_barrier(&p.sc->bar, nbar * (unsigned)G);
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

// Tile choice for the LDS-resident solvers: the smallest square tile side
// (>= 16) whose tile count fits the co-resident capacity.
static bool pick_tile(const Device& dev, int nx, int ny, int halo, int words, int per_cu_cap,
                      int* T, int* ntx, int* nty, size_t* lds) {
  for (int t = 16; t <= 128; t *= 2) {
    const int tx = (nx + t - 1) / t, ty = (ny + t - 1) / t;
    const size_t bytes = (size_t)words * (t + 2 * halo) * (t + 2 * halo) * sizeof(float);
    if (bytes + 1024 > (size_t)dev.max_lds) return false;
    if (tx * ty <= dev.cu * per_cu_cap && tx * ty <= kMaxCoopBlocks) {
      *T = t; *ntx = tx; *nty = ty; *lds = bytes;
      return true;
    }
  }
  return false;
}

static int jacobi_block_len(int check_every, int fixed_iters) {
  const int kMaxBlock = 8;
  if (fixed_iters > 0) return kMaxBlock;
  return check_every < kMaxBlock ? check_every : kMaxBlock;
}

bool solver_fits(const Device& dev, int nx, int ny, bool pcg, int check_every, int fixed_iters) {
  int T = 0, ntx = 0, nty = 0;
  size_t lds = 0;
  if (pcg) {
    if (!pick_tile(dev, nx, ny, 1, 4, 1, &T, &ntx, &nty, &lds)) return false;
    return T * T <= 16 * 256;
  }
  const int H = jacobi_block_len(check_every, fixed_iters) + 1;
  return pick_tile(dev, nx, ny, H, 5, 1, &T, &ntx, &nty, &lds);
}

hipError_t run_jacobi(const Device& dev, int nx, int ny, double dx, double thr, float omega,
                      int max_iters, int check_every, int fixed_iters, const Ws& w,
                      hipStream_t s) {
  JacParams p{};
  p.nx = nx; p.ny = ny;
  p.H = jacobi_block_len(check_every, fixed_iters) + 1;
  int T = 0, ntx = 0, nty = 0;
  size_t lds = 0;
  if (!pick_tile(dev, nx, ny, p.H, 5, 1, &T, &ntx, &nty, &lds)) return hipErrorInvalidValue;
  p.T = p.TH = T; p.ntx = ntx;
  p.inv_dx2 = (float)(1.0 / (dx * dx));
  p.wfac = (float)(omega * dx * dx);
  p.thr = thr;
  p.max_iters = max_iters; p.check_every = check_every; p.fixed_iters = fixed_iters;
  p.cell = w.cell; p.d = w.d; p.phi = w.phi; p.exch = w.exch; p.partial = w.partial; p.sc = w.sc;
  hipError_t e = hipFuncSetAttribute((const void*)jacobi_persist,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&p};
  return hipLaunchCooperativeKernel((const void*)jacobi_persist, dim3(ntx * nty), dim3(256), args,
                                    (unsigned)lds, s);
}

hipError_t run_pcg(const Device& dev, int nx, int ny, double dx, double thr, int max_iters,
                   int check_every, int fixed_iters, const Ws& w, hipStream_t s) {
  PcgParams p{};
  p.nx = nx; p.ny = ny;
  int T = 0, ntx = 0, nty = 0;
  size_t lds = 0;
  if (!pick_tile(dev, nx, ny, 1, 4, 1, &T, &ntx, &nty, &lds)) return hipErrorInvalidValue;
  if (T * T > 16 * 256) return hipErrorInvalidValue;  // q kept in 16 registers per thread
  p.T = p.TH = T; p.ntx = ntx;
  p.dx2 = (float)(dx * dx);
  p.inv_dx2 = 1.0 / (dx * dx);
  p.thr = thr;
  p.max_iters = max_iters; p.check_every = check_every; p.fixed_iters = fixed_iters;
  p.cell = w.cell; p.d = w.d; p.phi = w.phi; p.exch = w.exch; p.partial = w.partial; p.sc = w.sc;
  hipError_t e = hipFuncSetAttribute((const void*)pcg_persist,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&p};
  return hipLaunchCooperativeKernel((const void*)pcg_persist, dim3(ntx * nty), dim3(256), args,
                                    (unsigned)lds, s);
}

}  // namespace hyp
