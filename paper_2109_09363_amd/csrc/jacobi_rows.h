// Register-resident Jacobi rows shared by the single-grid and batched
// kernels: one lane per column, R consecutive rows of that column in
// registers, east/west neighbours by DPP wave shifts, the rows just outside
// the band (`below`, `above`) from the neighbouring waves through LDS.
#pragma once
#include "common.h"

namespace hyp {

// One pass over the R rows of a lane: new value (or residual) of every cell.
// `below`/`above` are the rows just outside the band (from LDS).  The update
// computes the rows that need no band edge first, so that the LDS reads of
// the edges are in flight meanwhile.
template <int R>
__device__ __forceinline__ float jac_cell(float c, float s, float n, float d, float k, float w,
                                          float inv_dx2) {
  const float e = from_right(c);
  const float wv = from_left(c);
  const float res = d - (((e + wv) + (n + s)) - k * c) * inv_dx2;
  return c - w * res;
}

// Without UPDATE: the sum of |r| over the rows in rmask, or their maximum
// (use_max, the E_inf criterion).
template <int R, bool UPDATE>
__device__ __forceinline__ double jac_rows(float (&ph)[R], const float (&dd)[R], const float (&kk)[R],
                                           const float (&ww)[R], float below, float above,
                                           float inv_dx2, unsigned rmask, bool use_max = false) {
  if (UPDATE) {
    float nv[R];
#pragma unroll
    for (int r = 1; r + 1 < R; ++r)
      nv[r] = jac_cell<R>(ph[r], ph[r - 1], ph[r + 1], dd[r], kk[r], ww[r], inv_dx2);
    nv[0] = jac_cell<R>(ph[0], below, ph[1], dd[0], kk[0], ww[0], inv_dx2);
    nv[R - 1] = jac_cell<R>(ph[R - 1], ph[R - 2], above, dd[R - 1], kk[R - 1], ww[R - 1], inv_dx2);
#pragma unroll
    for (int r = 0; r < R; ++r) ph[r] = nv[r];
    return 0.0;
  }
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
    if ((rmask >> r) & 1u) acc = use_max ? fmax(acc, fabs((double)res)) : acc + fabs((double)res);
  }
  return acc;
}

// The variable-density operator: the four face coefficients of every cell
// (beta = rho0 / rho_face, 0 on closed faces) weight the neighbours, and
// kk holds their sum (the diagonal).  With every beta = 1 it is the
// constant-coefficient update of jac_rows.
template <int R, bool UPDATE>
__device__ __forceinline__ double jac_rows_var(float (&ph)[R], const float (&dd)[R],
                                               const float (&kk)[R], const float (&ww)[R],
                                               const float (&be)[R], const float (&bw)[R],
                                               const float (&bn)[R], const float (&bs)[R],
                                               float below, float above, float inv_dx2,
                                               unsigned rmask, bool use_max = false) {
  auto cell = [&](int r, float s, float n) {
    const float c = ph[r];
    const float e = from_right(c);
    const float w = from_left(c);
    return dd[r] - (((be[r] * e + bw[r] * w) + (bn[r] * n + bs[r] * s)) - kk[r] * c) * inv_dx2;
  };
  if (UPDATE) {
    float nv[R];
#pragma unroll
    for (int r = 1; r + 1 < R; ++r) nv[r] = ph[r] - ww[r] * cell(r, ph[r - 1], ph[r + 1]);
    nv[0] = ph[0] - ww[0] * cell(0, below, ph[1]);
    nv[R - 1] = ph[R - 1] - ww[R - 1] * cell(R - 1, ph[R - 2], above);
#pragma unroll
    for (int r = 0; r < R; ++r) ph[r] = nv[r];
    return 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float s = r > 0 ? ph[r - 1] : below;
    const float n = (r + 1 < R) ? ph[r + 1] : above;
    const float res = cell(r, s, n);
    if ((rmask >> r) & 1u) acc = use_max ? fmax(acc, fabs((double)res)) : acc + fabs((double)res);
  }
  return acc;
}

}  // namespace hyp
