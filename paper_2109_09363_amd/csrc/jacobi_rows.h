// Register-resident Jacobi rows shared by the single-grid and batched
// kernels: one lane per column, R consecutive rows of that column in
// registers, east/west neighbours by DPP wave shifts, the rows just outside
// the band (`below`, `above`) from the neighbouring waves through LDS.
#pragma once
#include "common.h"

namespace hyp {

// Band edges of a four-wave tile through LDS, edge[parity][low row / high
// row][wave + 1][lane]: a wave writes its first and last rows and reads the
// rows next to its band from slots wave and wave + 2.  Slot 0 of the high
// rows and slot 5 of the low rows stay zero (the rows beyond the first and
// last waves), so that every wave reads unconditionally: no branch splits
// a sweep, which lets the east/west shifts fold into the adds.
typedef float BandEdges[2][6][64];
__device__ __forceinline__ void band_edges_clear(BandEdges* edge, int wave, int lane) {
  if (wave == 0) edge[0][1][0][lane] = edge[1][1][0][lane] = 0.f;
  if (wave == 3) edge[0][0][5][lane] = edge[1][0][5][lane] = 0.f;
}
template <int R>
__device__ __forceinline__ void band_exchange(const float (&v)[R], BandEdges* edge, int& q, int wave,
                                              int lane, float& below, float& above) {
  edge[q][0][wave + 1][lane] = v[0];
  edge[q][1][wave + 1][lane] = v[R - 1];
  __syncthreads();
  below = edge[q][1][wave][lane];
  above = edge[q][0][wave + 2][lane];
  q ^= 1;
}

// Two rows per band edge, for two sweeps per exchange:
// edge[parity][low 0, low 1, high 0, high 1][wave + 1][lane]; the high rows
// of slot 0 and the low rows of slot 5 stay zero.
typedef float BandEdges2[4][6][64];
__device__ __forceinline__ void band_edges2_clear(BandEdges2* edge, int wave, int lane) {
  if (wave == 0) edge[0][2][0][lane] = edge[0][3][0][lane] = edge[1][2][0][lane] = edge[1][3][0][lane] = 0.f;
  if (wave == 3) edge[0][0][5][lane] = edge[0][1][5][lane] = edge[1][0][5][lane] = edge[1][1][5][lane] = 0.f;
}
// b0, b1: rows -2 and -1 of the band (the lower wave's last two); a0, a1:
// rows R and R + 1 (the upper wave's first two)
template <int R>
__device__ __forceinline__ void band_exchange2(const float (&v)[R], BandEdges2* edge, int& q, int wave,
                                               int lane, float& b0, float& b1, float& a0, float& a1) {
  edge[q][0][wave + 1][lane] = v[0];
  edge[q][1][wave + 1][lane] = v[1];
  edge[q][2][wave + 1][lane] = v[R - 2];
  edge[q][3][wave + 1][lane] = v[R - 1];
  __syncthreads();
  b0 = edge[q][2][wave][lane];
  b1 = edge[q][3][wave][lane];
  a0 = edge[q][0][wave + 2][lane];
  a1 = edge[q][1][wave + 2][lane];
  q ^= 1;
}

// Constant-coefficient sweep in scaled form.  With a = omega / k and
// b = -omega dx^2 d / k on fluid cells (0 elsewhere, so those cells stay 0),
// the weighted Jacobi update phi - omega dx^2 r / k, r = d - (S - k phi) / dx^2
// and S the sum of the four neighbours, is (1 - omega) phi + a S + b: one FMA
// after the neighbour sum (two when omega != 1, om1 = 1 - omega).  Reads src,
// writes dst (two register sets, so that two sweeps need no copies).
template <int R, bool OMEGA1>
__device__ __forceinline__ void jac_rows_scaled(const float (&src)[R], float (&dst)[R],
                                                const float (&aa)[R], const float (&bb)[R],
                                                float below, float above, float om1) {
  // each add takes at most one shifted operand, so that the shift folds
  // into it (v_add_f32 with a DPP source: four VALU operations per cell)
  auto cell = [&](int r, float s, float n) {
    const float c = src[r];
    const float S = from_right(c) + (from_left(c) + (n + s));
    const float y = fmaf(S, aa[r], bb[r]);
    return OMEGA1 ? y : fmaf(om1, c, y);
  };
#pragma unroll
  for (int r = 1; r + 1 < R; ++r) dst[r] = cell(r, src[r - 1], src[r + 1]);
  dst[0] = cell(0, below, src[1]);
  dst[R - 1] = cell(R - 1, src[R - 2], above);
}

// Two constant-coefficient sweeps from one band exchange (ph -> tmp -> ph):
// with rows -2, -1 and R, R + 1 of the neighbouring waves (b0, b1, a0, a1),
// the first sweep also updates rows -1 and R (their coefficients gk_b,
// gw_b and gk_a, gw_a; zero beyond the tile, so that those rows stay zero
// there), which is what the second sweep takes from the neighbours.  The
// neighbour rows are updated by the same operations as in their own wave,
// so the result equals two sweeps with an exchange each, bit for bit.
template <int R, bool OMEGA1>
__device__ __forceinline__ void jac_pair_ghost(float (&ph)[R], float (&tmp)[R], const float (&aa)[R],
                                               const float (&bb)[R], float gk_b, float gw_b,
                                               float gk_a, float gw_a, float b0, float b1, float a0,
                                               float a1, float om1) {
  auto upd = [&](float c, float s, float n, float a, float b) {
    const float S = from_right(c) + (from_left(c) + (n + s));
    const float y = fmaf(S, a, b);
    return OMEGA1 ? y : fmaf(om1, c, y);
  };
  const float tb = upd(b1, b0, ph[0], gk_b, gw_b);      // row -1 after the first sweep
  const float ta = upd(a0, ph[R - 1], a1, gk_a, gw_a);  // row R after the first sweep
  jac_rows_scaled<R, OMEGA1>(ph, tmp, aa, bb, b1, a0, om1);
  jac_rows_scaled<R, OMEGA1>(tmp, ph, aa, bb, tb, ta, om1);
}

// The residual r = d - (S - k phi) / dx^2 of the scaled form, from
// k = omega / a and d = -b / (a dx^2): r = (omega phi - a S - b) / (a dx^2),
// with the hardware reciprocal of a (1 ulp; r only enters E_1 or E_inf).
// Sum of |r| over the rows in rmask (fluid rows: a > 0), or their maximum.
template <int R>
__device__ __forceinline__ double jac_resid_scaled(const float (&ph)[R], const float (&aa)[R],
                                                   const float (&bb)[R], float below, float above,
                                                   float omega, float inv_dx2, unsigned rmask,
                                                   bool use_max) {
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float c = ph[r];
    const float s = r > 0 ? ph[r - 1] : below;
    const float n = (r + 1 < R) ? ph[r + 1] : above;
    const float S = from_right(c) + (from_left(c) + (n + s));
    const float num = fmaf(-aa[r], S, fmaf(omega, c, -bb[r]));
    if ((rmask >> r) & 1u) {
      const double res = fabsf(num * (__builtin_amdgcn_rcpf(aa[r]) * inv_dx2));
      acc = use_max ? fmax(acc, res) : acc + res;
    }
  }
  return acc;
}

// Variable-density sweep in scaled form: with the face weights
// beta'_f = omega beta_f / k (k the sum of the cell's betas) and
// b = -omega dx^2 d / k, the weighted Jacobi update is
// (1 - omega) phi + sum_f beta'_f phi_f + b: four FMAs after the east/west
// shifts (five when omega != 1).  Reads src, writes dst.
template <int R, bool OMEGA1>
__device__ __forceinline__ void jac_rows_var_scaled(const float (&src)[R], float (&dst)[R],
                                                    const float (&be)[R], const float (&bw)[R],
                                                    const float (&bn)[R], const float (&bs)[R],
                                                    const float (&bb)[R], float below, float above,
                                                    float om1) {
  auto cell = [&](int r, float s, float n) {
    const float c = src[r];
    float y = fmaf(be[r], from_right(c), bb[r]);
    y = fmaf(bw[r], from_left(c), y);
    y = fmaf(bn[r], n, y);
    y = fmaf(bs[r], s, y);
    return OMEGA1 ? y : fmaf(om1, c, y);
  };
#pragma unroll
  for (int r = 1; r + 1 < R; ++r) dst[r] = cell(r, src[r - 1], src[r + 1]);
  dst[0] = cell(0, below, src[1]);
  dst[R - 1] = cell(R - 1, src[R - 2], above);
}

// Its residual r = d - (sum_f beta_f phi_f - k phi) / dx^2 from the scaled
// quantities: r = (omega phi - sum_f beta'_f phi_f - b) k / (omega dx^2).
// Sum of |r| over the rows in rmask, or their maximum.
template <int R>
__device__ __forceinline__ double jac_resid_var_scaled(const float (&ph)[R], const float (&kk)[R],
                                                       const float (&be)[R], const float (&bw)[R],
                                                       const float (&bn)[R], const float (&bs)[R],
                                                       const float (&bb)[R], float below, float above,
                                                       float omega, float inv_dx2, unsigned rmask,
                                                       bool use_max) {
  const float scale = inv_dx2 / omega;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float c = ph[r];
    const float s = r > 0 ? ph[r - 1] : below;
    const float n = (r + 1 < R) ? ph[r + 1] : above;
    float y = fmaf(be[r], from_right(c), bb[r]);
    y = fmaf(bw[r], from_left(c), y);
    y = fmaf(bn[r], n, y);
    y = fmaf(bs[r], s, y);
    if ((rmask >> r) & 1u) {
      const double res = fabsf((omega * c - y) * (kk[r] * scale));
      acc = use_max ? fmax(acc, res) : acc + res;
    }
  }
  return acc;
}

}  // namespace hyp
