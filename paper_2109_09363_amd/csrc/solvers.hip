// Persistent iterative solvers of L phi = d (Eq. 3), one cooperative launch
// each (all work-groups co-resident):
//
//  * Jacobi (Sec. 2.2) in correction form phi <- phi - omega dx^2 r / k_c,
//    r = d - L phi.  Register-resident with temporal blocking: a work-group
//    owns a 64-column extended tile (interior + halo of width H on every
//    side), one lane per column; each of the 4 waves keeps R consecutive
//    rows of its lane's column in registers, together with the scaled
//    update's per-cell factors (jacobi_rows.h).  East/west neighbours move
//    between lanes with DPP wave shifts, north/south come from the same
//    lane's registers (band edges through LDS).  A step of B <= H - 1 sweeps
//    ends with the interior written with agent-scope stores.  At a test
//    step the FP64 partial of sum|r| follows, then one grid barrier and one
//    round trip that brings back the halo and all partials together; any
//    other step waits only for the step words of the (up to) 8 adjacent
//    tiles, whose interiors hold its halo.  E_1 is tested at the steps that end on a multiple
//    of check_every (and at max_iters); every work-group sums the partials
//    in the same order, so all take the same decision at the same sweep.
//    Defect-correction folds (the velocity takes the increment, d is
//    recomputed from the faces, phi restarts at 0) run inside the launch.
//  * Jacobi-preconditioned conjugate gradient with FP64 dot products:
//    register tiles with a one-cell halo exchanged with the adjacent tiles,
//    one merged grid reduction per iteration, and a stop confirmed on the
//    true residual.
//
// Both come in a variable-density form (VAR): the operator weights every
// open face by beta = rho0 / rho_face (coefficient planes ce, cn), the
// diagonal is the sum of the four betas, and the fold corrects the faces by
// beta grad phi.  The constant-coefficient code is the VAR = false instance.
#include <atomic>
#include <type_traits>

#include "../../include/hyproj.h"
#include "common.h"
#include "internal.h"
#include "jacobi_rows.h"
#include "tile_table.h"

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
  int nx, ny, H, ntx, nty;
  float inv_dx2, wfac, inv_dx;  // wfac = omega * dx^2
  float omega, dx2;
  double thr;
  int max_iters, check_every, fixed_iters;
  int fold_window;      // sweeps per stagnation window (0: no folds)
  int einf;             // 1: stop on E_inf = max |r| instead of E_1 = mean |r|
  int nbsync;           // 1: steps without a test wait for the 8 adjacent tiles only
  int ckpt_every;       // > 0: write the interior iterate after every ckpt_every sweeps
  float* ckpt;          // ... into plane k / ckpt_every - 1 of this buffer
  const uint8_t* cell;
  float* d;             // recomputed on the interior at a fold
  float* phi;           // in: initial guess, out: returned iterate
  float* phi_acc;       // pressure folded into the faces
  float* u;             // faces, corrected at a fold
  float* v;
  uint64_t* exch64;     // 2 x nx*ny tagged halo words (steps between tests)
  float* exch;          // 2 x nx*ny halo planes (launches that test every step)
  double* partial;      // 4 x kMaxCoopBlocks partial sums (two parities each of the
                        // tests and of the lagged tests)
  unsigned* lagflag;    // 2 x kMaxCoopBlocks tags of the lagged partials
  int lag;              // 1: tests between the first and the last are lagged (below)
  Scalars* sc;
  unsigned* sync;       // grid barrier
  const float* ce;      // variable density: beta of each cell's east face
  const float* cn;      // ... north face
};

// The four face coefficients of cell g (flags ci): beta of the open faces,
// 0 on closed ones.
__device__ __forceinline__ void face_betas(const float* ce, const float* cn, int g, int nx,
                                           uint8_t ci, float& be, float& bw, float& bn, float& bs) {
  be = (ci & C_E) ? ce[g] : 0.f;
  bw = (ci & C_W) ? ce[g - 1] : 0.f;
  bn = (ci & C_N) ? cn[g] : 0.f;
  bs = (ci & C_S) ? cn[g - nx] : 0.f;
}

__device__ __forceinline__ void abort_solve(Scalars* sc) {
  __hip_atomic_fetch_max(&sc->status, (int32_t)HYP_STATUS_ABORTED, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// TAGGED: steps between E_1 tests exchange their halo through tagged words
// (below); otherwise every step ends at a test and crosses the grid barrier,
// after which the halo is read as plain FP32 values.
template <int R, bool VAR, bool TAGGED>
__global__ __launch_bounds__(256, (R <= 8 && (VAR || TAGGED) ? 2 : 1)) void jacobi_reg(JacParams p) {
  __shared__ BandEdges edge[2];
  __shared__ BandEdges2 edge2[2];  // two rows per edge: two sweeps per exchange
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  band_edges_clear(edge, wave, lane);
  band_edges2_clear(edge2, wave, lane);
  // Tile bx, by covers columns bx TW .. bx TW + 63 and rows by TH .. by TH +
  // 4R - 1; its interior leaves H cells to each side that has a neighbouring
  // tile and none at the grid's edges, where the cells outside stay zero
  // (so the first and last tiles of a row or column own H more cells)
  const int H = p.H, TW = 64 - 2 * H, TH = 4 * R - 2 * H;
  const int G = gridDim.x;
  const int bx = blockIdx.x % p.ntx, by = blockIdx.x / p.ntx;
  const int gx = bx * TW + lane;
  const int gy0 = by * TH + wave * R;
  const bool col_in = gx < p.nx;
  const bool lane_int = lane >= (bx == 0 ? 0 : H) && lane < (bx == p.ntx - 1 ? 64 : 64 - H) && col_in;
  const int row_lo = by == 0 ? 0 : H, row_hi = by == p.nty - 1 ? 4 * R : 4 * R - H;
  const int nF = p.sc->nF;
  if (p.sc->status >= 0) return;  // nothing to do (status already final)
  // rows of this thread inside the domain (dmask), inside the tile interior
  // (imask), and the fluid ones among the latter, which enter E_1 (fmask)
  unsigned dmask = 0, imask = 0, fmask = 0;
  // Scaled forms of the update (dd unused): the constant-coefficient instance
  // keeps kk = a = omega / k and ww = b = -omega dx^2 d / k; VAR keeps
  // kk = k (the sum of the betas), ww = b and the face weights
  // beta' = omega beta / k.  kk > 0 marks fluid cells in both.
  float ph[R], kk[R], ww[R];
  float be[R], bw[R], bn[R], bs[R];  // VAR only
  // every row's flags, d and phi are loaded before the first is used (one
  // round trip; out-of-domain rows load cell 0 and are masked), then the
  // coefficients; the face betas of the variable-density operator depend on
  // the flags (a second round trip)
  uint8_t ci[R];
  float dv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = gy0 + r;
    const bool in = col_in && gy >= 0 && gy < p.ny;
    const int g = in ? gy * p.nx + gx : 0;
    dmask |= in ? 1u << r : 0u;
    const uint8_t c_ = p.cell[g];
    dv[r] = p.d[g];
    ph[r] = p.phi[g];
    ci[r] = in ? c_ : (uint8_t)C_SOLID;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int er = wave * R + r, g = (gy0 + r) * p.nx + gx;
    const bool fl = !(ci[r] & C_SOLID);
    float k_ = 0.f, w_ = 0.f;
    be[r] = bw[r] = bn[r] = bs[r] = 0.f;
    if (fl) {
      if constexpr (VAR) {
        face_betas(p.ce, p.cn, g, p.nx, ci[r], be[r], bw[r], bn[r], bs[r]);
        k_ = (be[r] + bw[r]) + (bn[r] + bs[r]);
      } else {
        k_ = (float)cell_k(ci[r]);
      }
      w_ = -(p.wfac / k_) * dv[r];
      if constexpr (VAR) {
        const float sc = p.omega / k_;
        be[r] *= sc; bw[r] *= sc; bn[r] *= sc; bs[r] *= sc;
      } else {
        k_ = p.omega / k_;
      }
    } else {
      ph[r] = 0.f;
    }
    if (((dmask >> r) & 1u) && lane_int && er >= row_lo && er < row_hi) {
      imask |= 1u << r;
      if (fl) fmask |= 1u << r;
    }
    kk[r] = k_; ww[r] = w_;
  }
  // the tile's loads are complete before the loop (so that its publish
  // stores need not wait for them on every step)
  __builtin_amdgcn_s_waitcnt(0);
  const int k0 = p.sc->iters;
  const int end = p.fixed_iters > 0 ? p.fixed_iters : p.max_iters;
  const size_t plane = (size_t)p.nx * p.ny;
  int k = k0, q = 0, q2 = 0, k_ref = k0;
  unsigned j = 0, t = 0, nbar = 0;
  // Sweeps in pairs with one two-row band exchange (constant coefficients,
  // tagged form: there the waves drift apart between the tile exchanges,
  // and a block barrier per sweep costs more than the two extra rows that
  // the first sweep of a pair updates; in the plain form, every step behind
  // a grid barrier, it does not).  The coefficients of the rows next to the
  // band (the neighbouring waves' edge rows; zero beyond the tile):
  constexpr bool GHOST = !VAR && R <= 16 && TAGGED;
  float gk_b = 0.f, gw_b = 0.f, gk_a = 0.f, gw_a = 0.f;
  if constexpr (GHOST) {
    band_exchange<R>(kk, edge, q, wave, lane, gk_b, gk_a);
    band_exchange<R>(ww, edge, q, wave, lane, gw_b, gw_a);
  }
  double E_ref = 0.0;
  bool ref_set = false;
  auto edges_of = [&](const float (&v)[R], float* below, float* above) {
    band_exchange<R>(v, edge, q, wave, lane, *below, *above);
  };
  auto edges = [&](float* below, float* above) { edges_of(ph, below, above); };
  // kf: the sweep count of the returned iterate; a lagged stop returns the
  // iterate stored at its test, not the current one
  auto finish = [&](int st, double E, int kf, bool store) {
    if (store) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((imask >> r) & 1u) p.phi[(size_t)(gy0 + r) * p.nx + gx] = ph[r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      p.sc->iters = kf;
      p.sc->e1_solve = E;
      __hip_atomic_fetch_max(&p.sc->status, (int32_t)st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  auto barrier = [&]() -> bool {
    if (grid_barrier_bounded(p.sync, ++nbar, (unsigned)G)) return true;
    if (threadIdx.x == 0) abort_solve(p.sc);
    return false;
  };
  // Halo exchange through tagged words: each published value carries the
  // epoch of the launch and the step in its upper 32 bits, so a reader polls
  // the words it needs until their tags match instead of loading them after
  // a step flag, and a writer does not wait for its stores to complete before
  // raising that flag.  Flow control: every tile publishes all its
  // in-domain interior cells and reads all its in-domain halo cells, solid
  // ones included (they hold +0 on both sides), so a tile and each adjacent
  // tile read at least one word of each other's every step.  A tile
  // rewrites the plane of step j at step j + 2 only after reading its
  // neighbours' words of step j + 1, which they publish only after their
  // reads of step j have returned: no word is overwritten before it is read.
  // When the halo reaches beyond the adjacent tiles (nbsync 0) every step
  // also crosses the grid barrier.
  const unsigned epoch = p.sc->epoch;
  if (epoch == 1u) {
    // first launch after planning or an epoch wrap: no word may carry an
    // older tag of this epoch (whichever solver or exchange form the
    // projection at the wrap uses, it clears the words)
#pragma unroll
    for (int r = 0; r < R; ++r)
      if ((imask >> r) & 1u) {
        const size_t g = (size_t)(gy0 + r) * p.nx + gx;
        st_agent(p.exch64 + g, (uint64_t)0);
        st_agent(p.exch64 + plane + g, (uint64_t)0);
      }
    if (threadIdx.x == 0) {
      st_agent(p.lagflag + blockIdx.x, 0u);
      st_agent(p.lagflag + kMaxCoopBlocks + blockIdx.x, 0u);
    }
    if (!barrier()) return;
  }
  auto tag_of = [&](unsigned step) { return (epoch << 20) | (step & 0xFFFFFu); };
  // Lagged tests (tagged form, tests after the first and before max_iters
  // that cannot fold): a tile publishes its partial at step jL with a tag
  // word written after it and stores its interior as the candidate result,
  // then goes on without the grid barrier; one step later every tile reads
  // all partials (polling their tags), sums them in the same order and
  // takes the same decision: stop with the stored iterate and its sweep
  // count, or go on.  The host allows it only when tests are further apart
  // (in steps) than a tile can run ahead of any other (the neighbour
  // synchronisation bounds that by the tile grid's extent), so a partial is
  // read before its slot (two parities) is written again.
  bool pend = false;
  int kL = 0;
  unsigned jL = 0, nl = 0;
  for (;;) {
    // publish the interior of the state after j steps
    uint64_t* ex = p.exch64 + (size_t)(j & 1u) * plane;
    float* ex32 = p.exch + (size_t)(j & 1u) * plane;
    if (TAGGED && j > 0) {
      const uint64_t tag = (uint64_t)tag_of(j) << 32;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((imask >> r) & 1u) st_agent(ex + (size_t)(gy0 + r) * p.nx + gx, tag | __float_as_uint(ph[r]));
    } else if (j > 0) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (((imask >> r) & 1u) && kk[r] > 0.f) st_agent(ex32 + (size_t)(gy0 + r) * p.nx + gx, ph[r]);
    }
    // the decision of a lagged test, one step after it
    if (TAGGED && pend) {
      const unsigned want = tag_of(jL);
      const size_t sl = (size_t)(nl & 1u) * kMaxCoopBlocks;
      double a = 0.0;
      int ok = 1;
      const uint64_t t0 = (uint64_t)wall_clock64();
      for (int i = threadIdx.x; i < G; i += blockDim.x) {
        while (ld_agent(p.lagflag + sl + i) != want) {
          if ((uint64_t)wall_clock64() - t0 > kSpinTicks) {
            ok = 0;
            break;
          }
        }
        const double x = ld_agent(p.partial + 2 * kMaxCoopBlocks + sl + i);
        a = p.einf ? fmax(a, x) : a + x;
      }
      if (!__syncthreads_and(ok)) {
        if (threadIdx.x == 0) abort_solve(p.sc);
        return;
      }
      const double tot = p.einf ? block_max(a, red) : block_sum(a, red);
      const double EL = p.einf ? tot : (nF > 0 ? tot / nF : 0.0);
      const int stL = decide(kL, EL, p.thr, p.max_iters, p.check_every, p.fixed_iters);
      pend = false;
      if (stL != -1) {
        finish(stL, EL, kL, false);
        return;
      }
    }
    const bool at_test = k == k0 || (p.fixed_iters > 0 ? k >= end : (k % p.check_every == 0 || k >= end));
    const bool lagged = TAGGED && p.lag && at_test && k != k0 && k < end &&
                        !(p.fold_window > 0 && k - k_ref >= p.fold_window);
    const bool test = at_test && !lagged;
    // E_1 of the current state: the interior and the ring around it are
    // valid, so the residual needs no fresh halo
    double* part = p.partial + (size_t)((t + 1) & 1u) * kMaxCoopBlocks;
    if (lagged) {
      float below, above;
      edges(&below, &above);
      double part_loc;
      if constexpr (VAR)
        part_loc = jac_resid_var_scaled<R>(ph, kk, be, bw, bn, bs, ww, below, above, p.omega,
                                           p.inv_dx2, fmask, p.einf != 0);
      else
        part_loc = jac_resid_scaled<R>(ph, kk, ww, below, above, p.omega, p.inv_dx2, fmask,
                                       p.einf != 0);
      const double loc = p.einf ? block_max(part_loc, red) : block_sum(part_loc, red);
      ++nl;
      const size_t sl = (size_t)(nl & 1u) * kMaxCoopBlocks;
      if (threadIdx.x == 0) {
        st_agent(p.partial + 2 * kMaxCoopBlocks + sl + blockIdx.x, loc);
        __builtin_amdgcn_s_waitcnt(0);  // the partial is visible before its tag
        st_agent(p.lagflag + sl + blockIdx.x, tag_of(j));
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((imask >> r) & 1u) p.phi[(size_t)(gy0 + r) * p.nx + gx] = ph[r];
      pend = true;
      kL = k;
      jL = j;
    }
    if (test) {
      float below, above;
      edges(&below, &above);
      double part_loc;
      if constexpr (VAR)
        part_loc = jac_resid_var_scaled<R>(ph, kk, be, bw, bn, bs, ww, below, above, p.omega,
                                           p.inv_dx2, fmask, p.einf != 0);
      else
        part_loc = jac_resid_scaled<R>(ph, kk, ww, below, above, p.omega, p.inv_dx2, fmask,
                                       p.einf != 0);
      const double loc = p.einf ? block_max(part_loc, red) : block_sum(part_loc, red);
      ++t;
      if (threadIdx.x == 0) st_agent(part + blockIdx.x, loc);
    }
    // A step with a test (or, in fixed-sweep mode, a possible fold) crosses
    // the grid barrier; any other step only polls its halo words.
    const bool full = !TAGGED || test || !p.nbsync ||
                      (p.fixed_iters > 0 && p.fold_window > 0 && k - k_ref >= p.fold_window);
    if (full && !barrier()) return;
    // the halo of step j: every in-domain cell outside the interior, polled
    // until its tag is this step's (bounded like the barrier); without tags
    // the fluid halo cells after the barrier, in the same round trip as the
    // partials
    if (!TAGGED && j > 0) {
      // every row's load is issued before the first is used (at the lane's
      // own column and a row clamped into the grid), the halo's fluid cells
      // then taken by a bit mask: with the loads under the conditions the
      // compiler waited row by row
      const int gxc = gx < p.nx ? gx : p.nx - 1;
      float hv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int gy = gy0 + r, gyc = gy < 0 ? 0 : (gy < p.ny ? gy : p.ny - 1);
        hv[r] = ld_agent(ex32 + (size_t)gyc * p.nx + gxc);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const unsigned take = -(unsigned)((((imask >> r) & 1u) == 0u) & (kk[r] > 0.f));
        ph[r] = __uint_as_float((__float_as_uint(hv[r]) & take) | (__float_as_uint(ph[r]) & ~take));
      }
    } else if (j > 0) {
      const unsigned want = tag_of(j);
      unsigned need = dmask & ~imask;
      int ok = 1;
      const uint64_t t0 = (uint64_t)wall_clock64();
      for (;;) {
        // every load of a pass is issued before the first tag is compared
        uint64_t wd[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
          wd[r] = ((need >> r) & 1u) ? ld_agent(ex + (size_t)(gy0 + r) * p.nx + gx) : 0;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (((need >> r) & 1u) && (unsigned)(wd[r] >> 32) == want) {
            ph[r] = __uint_as_float((unsigned)wd[r]);
            need &= ~(1u << r);
          }
        if (__all(need == 0u)) break;
        if ((uint64_t)wall_clock64() - t0 > kSpinTicks) {
          ok = 0;
          break;
        }
      }
      if (!__syncthreads_and(ok)) {
        if (threadIdx.x == 0) abort_solve(p.sc);
        return;
      }
    }
    int st = -1;
    double E = 0.0;
    if (test) {
      double a = 0.0;
      for (int i = threadIdx.x; i < G; i += 256) {
        const double x = ld_agent(part + i);
        a = p.einf ? fmax(a, x) : a + x;
      }
      const double tot = p.einf ? block_max(a, red) : block_sum(a, red);
      E = p.einf ? tot : (nF > 0 ? tot / nF : 0.0);
      if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) p.sc->e1_cnn = E;
      st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
      if (!ref_set) { E_ref = E; ref_set = true; }
    }
    // stagnation window: fold when E_1 fell by less than 1 % over the window
    // (always in fixed-sweep mode, where folds only re-base the iteration)
    bool fold = false;
    if (st < 0 && p.fold_window > 0 && k - k_ref >= p.fold_window && (p.fixed_iters > 0 || test)) {
      fold = p.fixed_iters > 0 || !(E < 0.99 * E_ref);
      k_ref = k;
      E_ref = E;
    }
    if (st != -1) {
      finish(st, E, k, true);
      return;
    }
    if (fold) {
      // (1) the faces this tile owns (west and south of each interior cell,
      //     plus the open top face) take the increment; phi_acc keeps it.
      //     The refreshed halo holds the owners' values, bit-identical to
      //     the ring this tile computed itself.
      float below, above;
      edges(&below, &above);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float west = from_left(ph[r]);
        const float south = r > 0 ? ph[r - 1] : below;
        if (((imask >> r) & 1u) && kk[r] > 0.f) {
          const int gy = gy0 + r;
          const size_t c = (size_t)gy * p.nx + gx;
          const uint8_t ci = p.cell[c];
          const float pc = ph[r];
          // face weights: beta = beta' k / omega for the variable-density
          // operator, else 1
          const float bk = VAR ? kk[r] / p.omega : 0.f;
          const float fw = VAR ? bw[r] * bk : 1.f, fs = VAR ? bs[r] * bk : 1.f,
                      fn = VAR ? bn[r] * bk : 1.f;
          if (ci & C_W) {
            float* f = p.u + (size_t)gy * (p.nx + 1) + gx;
            st_agent(f, ld_agent(f) - fw * ((pc - west) * p.inv_dx));
          }
          if (ci & C_S) {
            float* f = p.v + c;
            st_agent(f, ld_agent(f) - fs * ((pc - south) * p.inv_dx));
          }
          if (gy == p.ny - 1 && (ci & C_N)) {
            float* f = p.v + plane + gx;
            st_agent(f, ld_agent(f) - fn * ((0.f - pc) * p.inv_dx));
          }
          p.phi_acc[c] += pc;
        }
      }
      (void)above;
      // (2) every tile's faces are in place
      if (!barrier()) return;
      // (3) d from the corrected faces on the whole extended tile; phi = 0
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (((dmask >> r) & 1u) && kk[r] > 0.f) {
          const int gy = gy0 + r;
          const size_t U = (size_t)p.nx + 1;
          const float uw = ld_agent(p.u + gy * U + gx), ue = ld_agent(p.u + gy * U + gx + 1);
          const float vs = ld_agent(p.v + (size_t)gy * p.nx + gx);
          const float vn = ld_agent(p.v + (size_t)(gy + 1) * p.nx + gx);
          const float dv = ((ue - uw) + (vn - vs)) * p.inv_dx;
          if constexpr (VAR) ww[r] = -(p.wfac / kk[r]) * dv;
          else ww[r] = -(kk[r] * p.dx2) * dv;
          if ((imask >> r) & 1u) p.d[(size_t)gy * p.nx + gx] = dv;
        }
        ph[r] = 0.f;
      }
      // the rows next to the band take the new right-hand sides too
      if constexpr (GHOST) band_exchange<R>(ww, edge, q, wave, lane, gw_b, gw_a);
    }
    // every load of the step (halo, partials, faces) is complete here: the
    // sweeps need the halo at once, and no path back to the publish stores
    // then carries a load in flight (which would make each of them wait)
    __builtin_amdgcn_s_waitcnt(0);
    int B = min(H - 1, end - k);
    if (p.fixed_iters <= 0) B = min(B, p.check_every - k % p.check_every);
    if (p.ckpt_every > 0) B = min(B, p.ckpt_every - k % p.ckpt_every);
    {
      // sweeps in pairs, ph -> tmp -> ph, so that no register copies are
      // needed between sweeps (up to R = 16; the larger tiles would spill);
      // omega = 1 drops one FMA per cell
      auto rows = [&](auto one, const float (&src)[R], float (&dst)[R], float below, float above,
                      float om1) {
        constexpr bool O1 = decltype(one)::value;
        if constexpr (VAR)
          jac_rows_var_scaled<R, O1>(src, dst, be, bw, bn, bs, ww, below, above, om1);
        else
          jac_rows_scaled<R, O1>(src, dst, kk, ww, below, above, om1);
      };
      auto sweeps = [&](auto one) {
        constexpr bool PAIRS = R <= 16;
        const float om1 = 1.f - p.omega;
        float tmp[R];
        int s = 0;
        if constexpr (GHOST) {
          // one exchange of two rows per pair of sweeps
          constexpr bool O1 = decltype(one)::value;
          for (; s + 2 <= B; s += 2) {
            float b0, b1, a0, a1;
            band_exchange2<R>(ph, edge2, q2, wave, lane, b0, b1, a0, a1);
            jac_pair_ghost<R, O1>(ph, tmp, kk, ww, gk_b, gw_b, gk_a, gw_a, b0, b1, a0, a1, om1);
          }
        }
        for (; PAIRS && s + 2 <= B; s += 2) {
          float below, above;
          edges_of(ph, &below, &above);
          rows(one, ph, tmp, below, above, om1);
          edges_of(tmp, &below, &above);
          rows(one, tmp, ph, below, above, om1);
        }
        for (; s < B; ++s) {
          float below, above;
          edges_of(ph, &below, &above);
          rows(one, ph, tmp, below, above, om1);
#pragma unroll
          for (int r = 0; r < R; ++r) ph[r] = tmp[r];
        }
      };
      if (R <= 16 && p.omega == 1.f) sweeps(std::true_type{});
      else sweeps(std::false_type{});
    }
    k += B;
    ++j;
    if (p.ckpt_every > 0 && k % p.ckpt_every == 0) {
      float* cp = p.ckpt + (size_t)(k / p.ckpt_every - 1) * plane;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((imask >> r) & 1u) cp[(size_t)(gy0 + r) * p.nx + gx] = ph[r];
    }
  }
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned CG on A x = b, A = -dx^2 L (diagonal k_c, -1 per
// non-solid neighbour), b = -dx^2 d, M = diag(k_c), in the single-reduction
// form of Chronopoulos and Gear: per iteration one halo exchange of the
// preconditioned residual u and one merged FP64 reduction of (r.u, w.u,
// sum|r|), w = A u.  Same tile layout as the Jacobi kernel with a one-cell
// halo; x, r, u, w, p, s live in registers.  A stop is confirmed on the true
// residual b - A x (FP32 drift of the updated residual).  When it fails, the
// velocity takes the increment (defect-correction fold: faces corrected, d
// recomputed from them, x restarts at 0) and CG restarts; after kMaxFolds
// folds a failed confirmation ends the solve with HYP_STATUS_FLOOR.
// ---------------------------------------------------------------------------
constexpr int kMaxFolds = 3;

struct PcgParams {
  int nx, ny, ntx, nty;
  float dx2, inv_dx;
  double thr, inv_dx2;
  int max_iters, check_every, fixed_iters;
  int einf;             // 1: stop on max |r| instead of the mean
  const uint8_t* cell;
  float* d;             // recomputed on the interior at a fold
  float* phi;           // in: initial guess, out: returned iterate
  float* phi_acc;       // pressure folded into the faces
  float* u;             // faces, corrected at a fold
  float* v;
  uint64_t* exch64;     // 2 x nx*ny tagged halo words (u, x)
  double* partial;      // 2 x 3 x kMaxCoopBlocks
  unsigned* lagflag;    // cleared with the halo words (the Jacobi kernel's lagged tags)
  Scalars* sc;
  unsigned* sync;
  const float* ce;      // variable density: beta of each cell's east face
  const float* cn;      // ... north face
};

// y = A v on the rows of a lane (k v - sum of the four neighbours; 0 where k = 0)
template <int R>
__device__ __forceinline__ void apply_A(const float (&v)[R], const float (&kk)[R], float below,
                                        float above, float (&y)[R]) {
  float prev = below;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float c = v[r];
    const float n = (r + 1 < R) ? v[r + 1] : above;
    const float e = from_right(c);
    const float w = from_left(c);
    y[r] = kk[r] > 0.f ? kk[r] * c - ((e + w) + (n + prev)) : 0.f;
    prev = c;
  }
}

// y = A v with face coefficients (diagonal kk = sum of the betas)
template <int R>
__device__ __forceinline__ void apply_A_var(const float (&v)[R], const float (&kk)[R],
                                            const float (&be)[R], const float (&bw)[R],
                                            const float (&bn)[R], const float (&bs)[R], float below,
                                            float above, float (&y)[R]) {
  float prev = below;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float c = v[r];
    const float n = (r + 1 < R) ? v[r + 1] : above;
    const float e = from_right(c);
    const float w = from_left(c);
    y[r] = kk[r] > 0.f ? kk[r] * c - ((be[r] * e + bw[r] * w) + (bn[r] * n + bs[r] * prev)) : 0.f;
    prev = c;
  }
}

// One tagged halo exchange of v (see pcg_reg): publish the interior fluid
// cells with tag `want`, poll the halo fluid cells until their tags match.
template <int R>
__device__ __forceinline__ bool pcg_exchange(float (&v)[R], uint64_t* ex, unsigned want,
                                                  unsigned imask, unsigned dmask, const float (&kk)[R],
                                                  int gy0, int gx, int nx) {
  const uint64_t tag = (uint64_t)want << 32;
#pragma unroll
  for (int i = 0; i < R; ++i)
    if ((imask >> i) & 1u) st_agent(ex + (size_t)(gy0 + i) * nx + gx, tag | __float_as_uint(v[i]));
  unsigned need = 0;
#pragma unroll
  for (int i = 0; i < R; ++i)
    if (((dmask >> i) & 1u) && !((imask >> i) & 1u) && kk[i] > 0.f) need |= 1u << i;
  int ok = 1;
  const uint64_t t0 = (uint64_t)wall_clock64();
  for (;;) {
    // every load of a pass is issued before the first tag is compared
    uint64_t wd[R];
#pragma unroll
    for (int i = 0; i < R; ++i)
      wd[i] = ((need >> i) & 1u) ? ld_agent(ex + (size_t)(gy0 + i) * nx + gx) : 0;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (((need >> i) & 1u) && (unsigned)(wd[i] >> 32) == want) {
        v[i] = __uint_as_float((unsigned)wd[i]);
        need &= ~(1u << i);
      }
    if (__all(need == 0u)) break;
    if ((uint64_t)wall_clock64() - t0 > kSpinTicks) {
      ok = 0;
      break;
    }
  }
  return __syncthreads_and(ok) != 0;
}
template <int R, bool VAR>
__global__ __launch_bounds__(256) void pcg_reg(PcgParams p) {
  __shared__ BandEdges edge[2];
  __shared__ double red3[12];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  band_edges_clear(edge, wave, lane);
  // tiles as in jacobi_reg with a one-cell halo: tile bx, by starts at
  // column 62 bx and row (4R - 2) by, no halo on the grid's sides
  const int TW = 62, TH = 4 * R - 2;
  const int G = gridDim.x;
  const int bx = blockIdx.x % p.ntx, by = blockIdx.x / p.ntx;
  const int gx = bx * TW + lane;
  const int gy0 = by * TH + wave * R;
  const bool col_in = gx < p.nx;
  const bool lane_int = lane >= (bx == 0 ? 0 : 1) && lane < (bx == p.ntx - 1 ? 64 : 63) && col_in;
  const int row_lo = by == 0 ? 0 : 1, row_hi = by == p.nty - 1 ? 4 * R : 4 * R - 1;
  const int nF = p.sc->nF;
  if (p.sc->status >= 0) return;
  unsigned dmask = 0, imask = 0;
  float x[R], r[R], u[R], w[R], pp[R], ss[R], kk[R], bb[R];
  float be[R], bw[R], bn[R], bs[R];  // VAR only
  // every row's flags, d and phi are loaded before the first is used (one
  // round trip; out-of-domain rows load cell 0 and are masked), then the
  // coefficients (face betas: a second round trip)
  uint8_t ci[R];
  float dv[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int gy = gy0 + i;
    const bool in = col_in && gy >= 0 && gy < p.ny;
    const int g = in ? gy * p.nx + gx : 0;
    dmask |= in ? 1u << i : 0u;
    const uint8_t c_ = p.cell[g];
    dv[i] = p.d[g];
    x[i] = p.phi[g];
    ci[i] = in ? c_ : (uint8_t)C_SOLID;
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int er = wave * R + i, g = (gy0 + i) * p.nx + gx;
    const bool fl = !(ci[i] & C_SOLID);
    float k_ = 0.f, b_ = 0.f;
    be[i] = bw[i] = bn[i] = bs[i] = 0.f;
    if (fl) {
      if constexpr (VAR) {
        face_betas(p.ce, p.cn, g, p.nx, ci[i], be[i], bw[i], bn[i], bs[i]);
        k_ = (be[i] + bw[i]) + (bn[i] + bs[i]);
      } else {
        k_ = (float)cell_k(ci[i]);
      }
      b_ = -p.dx2 * dv[i];
    } else {
      x[i] = 0.f;
    }
    if (((dmask >> i) & 1u) && lane_int && er >= row_lo && er < row_hi) imask |= 1u << i;
    kk[i] = k_; bb[i] = b_;
    r[i] = 0.f; u[i] = 0.f; w[i] = 0.f; pp[i] = 0.f; ss[i] = 0.f;
  }
  int q = 0, k = p.sc->iters, nfold = 0;
  const bool first = k == 0;
  unsigned nbar = 0;
  const size_t plane = (size_t)p.nx * p.ny;
  uint64_t* uex = p.exch64;
  uint64_t* xex = p.exch64 + plane;
  int par = 0;
  float below, above;

  auto barrier = [&]() -> bool {
    if (grid_barrier_bounded(p.sync, ++nbar, (unsigned)G)) return true;
    if (threadIdx.x == 0) abort_solve(p.sc);
    return false;
  };
  // refresh the halo of v from the neighbours' interiors: the words carry
  // the epoch and the exchange count in their upper 32 bits, and a tile polls
  // its halo words until their tags match (the writer does not wait for its
  // stores).  Every exchange is followed by the merged reduction's grid
  // barrier before its plane is written again, so no tile overwrites a word
  // that another has yet to read.
  const unsigned epoch = p.sc->epoch;
  if (epoch == 1u) {
    // first launch after planning or an epoch wrap: no word may carry an
    // older tag of this epoch
#pragma unroll
    for (int i = 0; i < R; ++i)
      if ((imask >> i) & 1u) {
        const size_t g = (size_t)(gy0 + i) * p.nx + gx;
        st_agent(uex + g, (uint64_t)0);
        st_agent(xex + g, (uint64_t)0);
      }
    if (threadIdx.x == 0) {  // the Jacobi kernel's lagged-test tags, too
      st_agent(p.lagflag + blockIdx.x, 0u);
      st_agent(p.lagflag + kMaxCoopBlocks + blockIdx.x, 0u);
    }
    if (!barrier()) return;
  }
  unsigned nex = 0;
  // up to R = 12 inlined; the larger tiles leave the call out of line, where
  // inlining would spill more of the kernel's register arrays
  auto exchange_call = [&](float (&v)[R], uint64_t* ex, unsigned want) __attribute__((noinline)) -> bool {
    return pcg_exchange<R>(v, ex, want, imask, dmask, kk, gy0, gx, p.nx);
  };
  auto exchange = [&](float (&v)[R], uint64_t* ex) __attribute__((always_inline)) -> bool {
    const unsigned want = (epoch << 20) | (++nex & 0xFFFFFu);
    bool ok;
    if constexpr (R <= 12) ok = pcg_exchange<R>(v, ex, want, imask, dmask, kk, gy0, gx, p.nx);
    else ok = exchange_call(v, ex, want);
    if (!ok && threadIdx.x == 0) abort_solve(p.sc);
    return ok;
  };
  // merged reduction of (r.u, w.u, sum|r| or max|r|) over the interior; forced
  // inline, since an out-of-line call takes r, u, w by reference and moves
  // them from registers to scratch memory (twice the time per iteration)
  double gam = 0.0, del = 0.0, E = 0.0;
  auto reduce3 = [&]() __attribute__((always_inline)) -> bool {
    double a = 0.0, c = 0.0, e = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if ((imask >> i) & 1u) {
        a += (double)r[i] * (double)u[i];
        c += (double)w[i] * (double)u[i];
        e = p.einf ? fmax(e, fabs((double)r[i])) : e + fabs((double)r[i]);
      }
    block_sum3(a, c, e, p.einf != 0, red3);
    double* pa = p.partial + par * 3 * kMaxCoopBlocks;
    if (threadIdx.x == 0) {
      st_agent(pa + blockIdx.x, a);
      st_agent(pa + kMaxCoopBlocks + blockIdx.x, c);
      st_agent(pa + 2 * kMaxCoopBlocks + blockIdx.x, e);
    }
    if (!barrier()) return false;
    // the three partial arrays come back in one round trip
    double sa = 0.0, sc_ = 0.0, se = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) {
      sa += ld_agent(pa + i);
      sc_ += ld_agent(pa + kMaxCoopBlocks + i);
      const double x = ld_agent(pa + 2 * kMaxCoopBlocks + i);
      se = p.einf ? fmax(se, x) : se + x;
    }
    block_sum3(sa, sc_, se, p.einf != 0, red3);
    gam = sa;
    del = sc_;
    if (p.einf)
      E = se * p.inv_dx2;
    else
      E = nF > 0 ? se / nF * p.inv_dx2 : 0.0;
    par ^= 1;
    return true;
  };
  // (re)start the recurrence from the current r: u = M^-1 r, w = A u, p = s = 0
  double alpha = 0.0, beta = 0.0;
  auto restart = [&]() -> bool {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      u[i] = kk[i] > 0.f ? r[i] / kk[i] : 0.f;
      pp[i] = 0.f;
      ss[i] = 0.f;
    }
    if (!exchange(u, uex)) return false;
    band_exchange<R>(u, edge, q, wave, lane, below, above);
    if constexpr (VAR) apply_A_var<R>(u, kk, be, bw, bn, bs, below, above, w);
    else apply_A<R>(u, kk, below, above, w);
    if (!reduce3()) return false;
    alpha = del > 0.0 ? gam / del : 0.0;
    beta = 0.0;
    return true;
  };
  // true residual r = b - A x (needs the halo of x)
  auto true_residual = [&]() -> bool {
    if (!exchange(x, xex)) return false;
    float ax[R];
    band_exchange<R>(x, edge, q, wave, lane, below, above);
    if constexpr (VAR) apply_A_var<R>(x, kk, be, bw, bn, bs, below, above, ax);
    else apply_A<R>(x, kk, below, above, ax);
#pragma unroll
    for (int i = 0; i < R; ++i) r[i] = kk[i] > 0.f ? bb[i] - ax[i] : 0.f;
    return true;
  };
  auto finish = [&](int st) {
#pragma unroll
    for (int i = 0; i < R; ++i)
      if ((imask >> i) & 1u) p.phi[(size_t)(gy0 + i) * p.nx + gx] = x[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      p.sc->iters = k;
      p.sc->e1_solve = E;
      __hip_atomic_fetch_max(&p.sc->status, (int32_t)st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  // defect-correction fold of the current x (its halo is fresh from the
  // true-residual exchange): faces, phi_acc, d recomputed from the faces
  auto fold = [&]() -> bool {
    band_exchange<R>(x, edge, q, wave, lane, below, above);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const float west = from_left(x[i]);
      const float south = i > 0 ? x[i - 1] : below;
      if (((imask >> i) & 1u) && kk[i] > 0.f) {
        const int gy = gy0 + i;
        const size_t c = (size_t)gy * p.nx + gx;
        const uint8_t ci = p.cell[c];
        const float pc = x[i];
        const float fw = VAR ? bw[i] : 1.f, fs = VAR ? bs[i] : 1.f, fn = VAR ? bn[i] : 1.f;
        if (ci & C_W) {
          float* f = p.u + (size_t)gy * (p.nx + 1) + gx;
          st_agent(f, ld_agent(f) - fw * ((pc - west) * p.inv_dx));
        }
        if (ci & C_S) {
          float* f = p.v + c;
          st_agent(f, ld_agent(f) - fs * ((pc - south) * p.inv_dx));
        }
        if (gy == p.ny - 1 && (ci & C_N)) {
          float* f = p.v + plane + gx;
          st_agent(f, ld_agent(f) - fn * ((0.f - pc) * p.inv_dx));
        }
        p.phi_acc[c] += pc;
      }
    }
    if (!barrier()) return false;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (((dmask >> i) & 1u) && kk[i] > 0.f) {
        const int gy = gy0 + i;
        const size_t U = (size_t)p.nx + 1;
        const float uw = ld_agent(p.u + gy * U + gx), ue = ld_agent(p.u + gy * U + gx + 1);
        const float vs = ld_agent(p.v + (size_t)gy * p.nx + gx);
        const float vn = ld_agent(p.v + (size_t)(gy + 1) * p.nx + gx);
        const float dv = ((ue - uw) + (vn - vs)) * p.inv_dx;
        bb[i] = -p.dx2 * dv;
        if ((imask >> i) & 1u) p.d[(size_t)gy * p.nx + gx] = dv;
      }
      x[i] = 0.f;
    }
    return true;
  };

  if (!true_residual() || !restart()) return;
  if (first && blockIdx.x == 0 && threadIdx.x == 0) p.sc->e1_cnn = E;
  for (;;) {
    int st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
    if (st < 0 && !(gam > 0.0)) st = HYP_STATUS_OK;  // r = 0 exactly
    if (st == HYP_STATUS_OK && p.fixed_iters <= 0) {
      // confirm on the true residual
      if (!true_residual() || !restart()) return;
      st = decide(k, E, p.thr, p.max_iters, p.check_every, p.fixed_iters);
      if (st < 0 && !(gam > 0.0)) st = HYP_STATUS_OK;
      if (st < 0) {
        if (nfold >= kMaxFolds) {
          st = HYP_STATUS_FLOOR;
        } else {
          ++nfold;
          if (!fold() || !true_residual() || !restart()) return;
          continue;
        }
      }
    }
    if (st != -1) {
      finish(st);
      return;
    }
    if (!(alpha == alpha) || !isfinite(alpha)) {
      finish(HYP_STATUS_NONFINITE);
      return;
    }
    const float a = (float)alpha, bt = (float)beta;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      pp[i] = u[i] + bt * pp[i];
      ss[i] = w[i] + bt * ss[i];
      x[i] += a * pp[i];
      r[i] -= a * ss[i];
      u[i] = kk[i] > 0.f ? r[i] / kk[i] : 0.f;
    }
    if (!exchange(u, uex)) return;
    band_exchange<R>(u, edge, q, wave, lane, below, above);
    if constexpr (VAR) apply_A_var<R>(u, kk, be, bw, bn, bs, below, above, w);
    else apply_A<R>(u, kk, below, above, w);
    const double gam_old = gam;
    if (!reduce3()) return;
    beta = gam_old != 0.0 ? gam / gam_old : 0.0;
    const double den = del - beta * gam / alpha;
    alpha = den != 0.0 ? gam / den : 0.0;
    ++k;
  }
}

// ---------------------------------------------------------------------------
// Launch geometry.  Jacobi: halo H = B + 1 for B sweeps per step, tile
// interior (64 - 2H) x (4R - 2H).  The tuned table gives (R, H) per grid
// (its tiles may fill two work-groups per CU when the kernel's registers
// allow it: one sweeps while the other waits for its halo); otherwise B =
// min(check_every, 8) (8 for fixed_iters) and the smallest R whose tile
// count fits one work-group per CU.  A caller's block length replaces B
// (clipped to check_every when a threshold decides).
static int jacobi_block_len(int check_every, int fixed_iters, int block) {
  const int b = block > 0 ? block : 8;
  if (fixed_iters > 0) return b;
  return check_every < b ? check_every : b;
}

static const int kRows[] = {4, 8, 12, 16, 24, 32};

// The persistent solvers need every work-group resident (grid barriers):
// a cooperative launch checks that.  Inside stream capture (a hipGraph of a
// projection or time step) the launch is a plain one of the same grid, whose
// size the occupancy query bounds, so that all its work-groups are resident
// when the graph runs alone on the GPU; a barrier that is not reached within
// its bound ends the solve with ABORTED instead of hanging.
static hipError_t launch_persistent(const void* k, int G, void** args, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return hipErrorInvalidValue;
  if (cs == hipStreamCaptureStatusActive) return hipLaunchKernel(k, dim3(G), dim3(256), args, 0, s);
  return hipLaunchCooperativeKernel(k, dim3(G), dim3(256), args, 0, s);
}

template <int R>
static const void* jacobi_kernel(bool var, bool tagged) {
  if (var) return tagged ? (const void*)jacobi_reg<R, true, true> : (const void*)jacobi_reg<R, true, false>;
  return tagged ? (const void*)jacobi_reg<R, false, true> : (const void*)jacobi_reg<R, false, false>;
}

// Work-groups of jacobi_reg<r> that one CU holds at once (registers, LDS),
// at most 2; every one of them must be resident for the grid barrier.
static int jacobi_per_cu(int r, bool var) {
  // queried once per instance; threads that race here store the same value
  static std::atomic<int> cache[2][6] = {};
  int i = 0;
  while (i < 6 && kRows[i] != r) ++i;
  if (i == 6) return 1;
  std::atomic<int>& slot = cache[var ? 1 : 0][i];
  int c = slot.load(std::memory_order_relaxed);
  if (c == 0) {
    // the smaller of the two exchange forms (they choose between them later)
    c = 2;
    for (int tagged = 0; tagged < 2; ++tagged) {
      const void* k = nullptr;
      switch (r) {
        case 4: k = jacobi_kernel<4>(var, tagged); break;
        case 8: k = jacobi_kernel<8>(var, tagged); break;
        case 12: k = jacobi_kernel<12>(var, tagged); break;
        case 16: k = jacobi_kernel<16>(var, tagged); break;
        case 24: k = jacobi_kernel<24>(var, tagged); break;
        default: k = jacobi_kernel<32>(var, tagged); break;
      }
      int n = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 256, 0) != hipSuccess || n < 1) n = 1;
      if (n < c) c = n;
    }
    slot.store(c, std::memory_order_relaxed);
  }
  return c;
}

// multi: allow as many work-groups per CU as are resident (tuned or chosen R)
static bool jacobi_fit(const Device& dev, int nx, int ny, int r, int h, bool var, bool multi,
                       int* ntx, int* nty) {
  const int tw = 64 - 2 * h, th = 4 * r - 2 * h;
  if (tw < 1 || th < 1) return false;
  int cap = dev.cu * (multi ? jacobi_per_cu(r, var) : 1);
  cap = cap < kMaxCoopBlocks ? cap : kMaxCoopBlocks;
  // tile t starts at t tw (columns) and t th (rows); the last one reaches
  // the grid's edge (the tile layout of jacobi_reg)
  const int tx = 1 + (nx > 64 ? (nx - 64 + tw - 1) / tw : 0);
  const int ty = 1 + (ny > 4 * r ? (ny - 4 * r + th - 1) / th : 0);
  if (tx * ty > cap) return false;
  *ntx = tx;
  *nty = ty;
  return true;
}

// rows = 0: the tuned table, else the smallest R that fits; rows > 0: that R.
// block = 0: the table's block when it fits check_every, else the default.
static bool jacobi_geom(const Device& dev, int nx, int ny, int check_every, int fixed_iters,
                        int rows, int block, bool var, int* R, int* H, int* ntx, int* nty) {
  if (rows == 0) {
    for (int i = 0; i < kTileTableSize; ++i) {
      const TileEntry& t = kTileTable[i];
      const int th = block > 0 ? jacobi_block_len(check_every, fixed_iters, block) + 1 : t.H;
      const bool fits_checks = fixed_iters > 0 || t.H - 1 <= check_every;
      if (t.nx == nx && t.ny == ny && th == t.H && fits_checks &&
          jacobi_fit(dev, nx, ny, t.R, t.H, var, true, ntx, nty)) {
        *R = t.R;
        *H = t.H;
        return true;
      }
    }
  }
  const int h = jacobi_block_len(check_every, fixed_iters, block) + 1;
  *H = h;
  if (rows > 0) {
    bool known = false;
    for (int r : kRows) known = known || r == rows;
    if (!known || !jacobi_fit(dev, nx, ny, rows, h, var, true, ntx, nty)) return false;
    *R = rows;
    return true;
  }
  for (int r : kRows) {
    if (jacobi_fit(dev, nx, ny, r, h, var, false, ntx, nty)) {
      *R = r;
      return true;
    }
  }
  return false;
}

// PCG: halo 1, tile interior 62 x (4R - 2), the smallest R that fits.
static bool pcg_geom(const Device& dev, int nx, int ny, int* R, int* ntx, int* nty) {
  const int tx = 1 + (nx > 64 ? (nx - 64 + 61) / 62 : 0);
  const int cap = dev.cu < kMaxCoopBlocks ? dev.cu : kMaxCoopBlocks;
  for (int r : kRows) {
    const int ty = 1 + (ny > 4 * r ? (ny - 4 * r + 4 * r - 3) / (4 * r - 2) : 0);
    if (tx * ty <= cap) {
      *R = r; *ntx = tx; *nty = ty;
      return true;
    }
  }
  return false;
}

bool solver_fits(const Device& dev, int nx, int ny, bool pcg, int check_every, int fixed_iters,
                 int tile_rows, int block, bool var) {
  if (pcg) {
    int R, ntx, nty;
    return pcg_geom(dev, nx, ny, &R, &ntx, &nty);
  }
  int R, H, ntx, nty;
  return jacobi_geom(dev, nx, ny, check_every, fixed_iters, tile_rows, block, var, &R, &H, &ntx, &nty);
}

// Tagged halo words pay off on steps between tests; a launch whose every
// step ends at a test (check_every up to the block length, or a halo that
// reaches beyond the adjacent tiles) crosses the grid barrier each step and
// reads plain FP32 halo values after it.
template <int R>
static hipError_t launch_jacobi(JacParams& p, int G, hipStream_t s) {
  void* args[] = {&p};
  const bool every_step_tested = p.fixed_iters <= 0 && p.check_every <= p.H - 1;
  const void* k = jacobi_kernel<R>(p.ce != nullptr, p.nbsync && !every_step_tested);
  return launch_persistent(k, G, args, s);
}

hipError_t run_jacobi(const Device& dev, int nx, int ny, double dx, double thr, float omega,
                      int max_iters, int check_every, int fixed_iters, int fold_window,
                      int checkpoint_every, float* phi_ckpt, int tile_rows, int block, bool var,
                      bool einf, float* u, float* v, const Ws& w, hipStream_t s) {
  JacParams p{};
  p.einf = einf ? 1 : 0;
  int R = 0, H = 0, ntx = 0, nty = 0;
  if (!jacobi_geom(dev, nx, ny, check_every, fixed_iters, tile_rows, block, var, &R, &H, &ntx, &nty))
    return hipErrorInvalidValue;
  p.nx = nx; p.ny = ny; p.H = H; p.ntx = ntx; p.nty = nty;
  p.nbsync = (H <= 64 - 2 * H && H <= 4 * R - 2 * H) ? 1 : 0;
  p.inv_dx2 = (float)(1.0 / (dx * dx));
  p.inv_dx = (float)(1.0 / dx);
  p.wfac = (float)(omega * dx * dx);
  p.omega = omega;
  p.dx2 = (float)(dx * dx);
  p.thr = thr;
  p.max_iters = max_iters; p.check_every = check_every; p.fixed_iters = fixed_iters;
  p.fold_window = fold_window > 0 ? fold_window : (fixed_iters > 0 ? 0 : 1024);
  p.ckpt_every = phi_ckpt ? checkpoint_every : 0;
  p.ckpt = phi_ckpt;
  p.cell = w.cell; p.d = w.d; p.phi = w.phi; p.phi_acc = w.phi_acc; p.u = u; p.v = v;
  p.exch64 = w.exch64; p.exch = w.exch; p.partial = w.partial; p.sc = w.sc; p.sync = w.sync;
  p.lagflag = w.lagflag;
  {
    // lagged tests: tagged form, and tests further apart in steps than the
    // tile grid's extent (the furthest one tile can run ahead of another)
    const bool tagged = p.nbsync && !(fixed_iters <= 0 && check_every <= H - 1);
    const int steps = (check_every + H - 2) / (H - 1);
    p.lag = (tagged && fixed_iters <= 0 && steps >= (ntx > nty ? ntx : nty) + 2) ? 1 : 0;
  }
  p.ce = var ? w.coef_e : nullptr;
  p.cn = var ? w.coef_n : nullptr;
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

template <int R>
static hipError_t launch_pcg(PcgParams& p, int G, hipStream_t s) {
  void* args[] = {&p};
  const void* k = p.ce ? (const void*)pcg_reg<R, true> : (const void*)pcg_reg<R, false>;
  return launch_persistent(k, G, args, s);
}

hipError_t run_pcg(const Device& dev, int nx, int ny, double dx, double thr, int max_iters,
                   int check_every, int fixed_iters, bool var, bool einf, float* u, float* v,
                   const Ws& w, hipStream_t s) {
  PcgParams p{};
  p.einf = einf ? 1 : 0;
  int R = 0, ntx = 0, nty = 0;
  if (!pcg_geom(dev, nx, ny, &R, &ntx, &nty)) return hipErrorInvalidValue;
  p.nx = nx; p.ny = ny; p.ntx = ntx; p.nty = nty;
  p.dx2 = (float)(dx * dx);
  p.inv_dx = (float)(1.0 / dx);
  p.inv_dx2 = 1.0 / (dx * dx);
  p.thr = thr;
  p.max_iters = max_iters; p.check_every = check_every; p.fixed_iters = fixed_iters;
  p.cell = w.cell; p.d = w.d; p.phi = w.phi; p.phi_acc = w.phi_acc; p.u = u; p.v = v;
  p.exch64 = w.exch64; p.partial = w.partial; p.lagflag = w.lagflag; p.sc = w.sc; p.sync = w.sync;
  p.ce = var ? w.coef_e : nullptr;
  p.cn = var ? w.coef_n : nullptr;
  const int G = ntx * nty;
  switch (R) {
    case 4: return launch_pcg<4>(p, G, s);
    case 8: return launch_pcg<8>(p, G, s);
    case 12: return launch_pcg<12>(p, G, s);
    case 16: return launch_pcg<16>(p, G, s);
    case 24: return launch_pcg<24>(p, G, s);
    case 32: return launch_pcg<32>(p, G, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace hyp
