// Advection + force half of a time step (Sec. 2.2): density and velocity
// advected by a MacCormack semi-Lagrangian scheme with the start-of-step
// velocity, buoyancy added by forward Euler, inflow faces and cells reset,
// faces touching solids or walls zeroed -> u*.
//
//   dt     = cfl dx / max(max|u|, max|v|, U_in)               (device FP64)
//   q_hat  = q sampled at x - dt vel(x)                       (pass 1)
//   q_til  = q_hat sampled at x + dt vel(x)                   (pass 2)
//   q_new  = clamp(q_hat + (q - q_til)/2, min4, max4)         (pass 2)
//   v     += dt g (rho0 - rho_face) / rho0, inflow, walls     (pass 3)
// min4/max4 are the extremes of the four samples of q that the backward
// trace of pass 1 interpolated.  Sampling is bilinear with positions clamped
// to the extent of the sampled grid.
#include "../../include/hyproj.h"
#include "batch.h"
#include "common.h"
#include "internal.h"

namespace hyp {

__device__ __forceinline__ float sample(const float* __restrict__ q, int H, int W, float X,
                                        float Y, float* mn, float* mx) {
  X = fminf(fmaxf(X, 0.f), (float)(W - 1));
  Y = fminf(fmaxf(Y, 0.f), (float)(H - 1));
  const int i0 = min((int)floorf(X), max(W - 2, 0));
  const int j0 = min((int)floorf(Y), max(H - 2, 0));
  const float fx = X - (float)i0, fy = Y - (float)j0;
  const int i1 = min(i0 + 1, W - 1), j1 = min(j0 + 1, H - 1);
  const float a = q[j0 * W + i0], b = q[j0 * W + i1], c = q[j1 * W + i0], d = q[j1 * W + i1];
  if (mn) {
    *mn = fminf(fminf(a, b), fminf(c, d));
    *mx = fmaxf(fmaxf(a, b), fmaxf(c, d));
  }
  return (1.f - fy) * ((1.f - fx) * a + fx * b) + fy * ((1.f - fx) * c + fx * d);
}

// velocity (in physical units) at sample point `idx` of grid `which`
// (0: cell centres, 1: u faces, 2: v faces)
__device__ __forceinline__ void vel_at(int which, int i, int j, int nx, int ny,
                                       const float* __restrict__ u, const float* __restrict__ v,
                                       float* vx, float* vy) {
  const int U = nx + 1;
  if (which == 0) {
    *vx = 0.5f * (u[j * U + i] + u[j * U + i + 1]);
    *vy = 0.5f * (v[j * nx + i] + v[(j + 1) * nx + i]);
  } else if (which == 1) {
    const int il = min(max(i - 1, 0), nx - 1), ir = min(i, nx - 1);
    *vx = u[j * U + i];
    *vy = 0.25f * (((v[j * nx + il] + v[j * nx + ir]) + v[(j + 1) * nx + il]) + v[(j + 1) * nx + ir]);
  } else {
    const int jb = min(max(j - 1, 0), ny - 1), jt = min(j, ny - 1);
    *vx = 0.25f * (((u[jb * U + i] + u[jb * U + i + 1]) + u[jt * U + i]) + u[jt * U + i + 1]);
    *vy = v[j * nx + i];
  }
}

struct AdvPtrs {
  const float* q[3];  // rho, u, v (start of step)
  float* hat[3];
  float* out[3];
  int H[3], W[3];
  int n0, n1, n2;     // sizes of the three sample grids
};

__device__ __forceinline__ void locate(const AdvPtrs& A, int gid, int* which, int* i, int* j) {
  int w = 0, l = gid;
  if (l >= A.n0) { l -= A.n0; w = 1; if (l >= A.n1) { l -= A.n1; w = 2; } }
  *which = w;
  *i = l % A.W[w];
  *j = l / A.W[w];
}

__device__ __forceinline__ void cfl_body(int gid, int nu, int nv, const float* __restrict__ u,
                                         const float* __restrict__ v, double* __restrict__ slot,
                                         double* red) {
  double m = 0.0;
  if (gid < nu) m = fabs((double)u[gid]);
  else if (gid < nu + nv) m = fabs((double)v[gid - nu]);
  m = block_max(m, red);
  if (threadIdx.x == 0) *slot = m;
}

__device__ __forceinline__ void cfl_finish_body(int nblocks, const double* __restrict__ blockpart,
                                                double dx, double cfl, double u_in, Scalars* sc,
                                                double* red) {
  double m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) m = fmax(m, blockpart[b]);
  m = block_max(m, red);
  if (threadIdx.x == 0) sc->dt = cfl * dx / fmax(m, u_in);
}

__global__ __launch_bounds__(256) void cfl_kernel(int nu, int nv, const float* __restrict__ u,
                                                  const float* __restrict__ v,
                                                  double* __restrict__ blockpart) {
  __shared__ double red[4];
  cfl_body(blockIdx.x * blockDim.x + threadIdx.x, nu, nv, u, v, blockpart + blockIdx.x, red);
}

__global__ __launch_bounds__(256) void cfl_finish(int nblocks, const double* __restrict__ blockpart,
                                                  double dx, double cfl, double u_in, Scalars* sc) {
  __shared__ double red[4];
  cfl_finish_body(nblocks, blockpart, dx, cfl, u_in, sc, red);
}

__device__ __forceinline__ void pass1_body(const AdvPtrs& A, int gid, int nx, int ny, float inv_dx,
                                           const float* __restrict__ u, const float* __restrict__ v,
                                           const Scalars* sc) {
  if (gid >= A.n0 + A.n1 + A.n2) return;
  int w, i, j;
  locate(A, gid, &w, &i, &j);
  const float r = (float)sc->dt * inv_dx;
  float vx, vy;
  vel_at(w, i, j, nx, ny, u, v, &vx, &vy);
  A.hat[w][j * A.W[w] + i] =
      sample(A.q[w], A.H[w], A.W[w], (float)i - r * vx, (float)j - r * vy, nullptr, nullptr);
}

__device__ __forceinline__ void pass2_body(const AdvPtrs& A, int gid, int nx, int ny, float inv_dx,
                                           const float* __restrict__ u, const float* __restrict__ v,
                                           const Scalars* sc) {
  if (gid >= A.n0 + A.n1 + A.n2) return;
  int w, i, j;
  locate(A, gid, &w, &i, &j);
  const float r = (float)sc->dt * inv_dx;
  float vx, vy;
  vel_at(w, i, j, nx, ny, u, v, &vx, &vy);
  const float ox = r * vx, oy = r * vy;
  float mn, mx;
  sample(A.q[w], A.H[w], A.W[w], (float)i - ox, (float)j - oy, &mn, &mx);
  const float qt = sample(A.hat[w], A.H[w], A.W[w], (float)i + ox, (float)j + oy, nullptr, nullptr);
  const int l = j * A.W[w] + i;
  const float qn = A.hat[w][l] + 0.5f * (A.q[w][l] - qt);
  A.out[w][l] = fminf(fmaxf(qn, mn), mx);
}

__global__ __launch_bounds__(256) void advect_pass1(AdvPtrs A, int nx, int ny, float inv_dx,
                                                    const float* __restrict__ u,
                                                    const float* __restrict__ v, const Scalars* sc) {
  pass1_body(A, blockIdx.x * blockDim.x + threadIdx.x, nx, ny, inv_dx, u, v, sc);
}

__global__ __launch_bounds__(256) void advect_pass2(AdvPtrs A, int nx, int ny, float inv_dx,
                                                    const float* __restrict__ u,
                                                    const float* __restrict__ v, const Scalars* sc) {
  pass2_body(A, blockIdx.x * blockDim.x + threadIdx.x, nx, ny, inv_dx, u, v, sc);
}

// buoyancy on interior/top v faces, inflow, boundary faces; writes the state
__device__ __forceinline__ void pass3_body(int gid, int nx, int ny, const float* __restrict__ rho_n,
                                           const float* __restrict__ u_n,
                                           const float* __restrict__ v_n,
                                           const uint8_t* __restrict__ cell,
                                           const float* __restrict__ xi, double g, double rho0,
                                           double drho, double u_in, float* __restrict__ rho,
                                           float* __restrict__ u, float* __restrict__ v,
                                           const Scalars* sc) {
  const int n = nx * ny, nu = ny * (nx + 1), nv = (ny + 1) * nx;
  if (gid < n) {
    const int j = gid / nx;
    const uint8_t ci = cell[gid];
    float val = rho_n[gid];
    if (j == 0 && (ci & C_INFLOW)) val = (float)(rho0 * (1.0 - drho));
    rho[gid] = val;
  } else if (gid < n + nu) {
    const int l = gid - n, U = nx + 1, i = l % U, j = l / U;
    bool open = false;
    if (i > 0 && i < nx) {
      const uint8_t c = cell[j * nx + i];
      open = !(c & C_SOLID) && (c & C_W);
    }
    u[l] = open ? u_n[l] : 0.f;
  } else if (gid < n + nu + nv) {
    const int l = gid - n - nu, i = l % nx, j = l / nx;
    float val;
    if (j == 0) {
      const uint8_t c = cell[i];
      const bool inflow = !(c & C_SOLID) && (c & C_INFLOW);
      val = inflow ? (float)(u_in * (1.0 + (double)xi[i])) : 0.f;
    } else {
      const float dt = (float)sc->dt;
      const float rf = j < ny ? 0.5f * (rho_n[(j - 1) * nx + i] + rho_n[j * nx + i]) : rho_n[(ny - 1) * nx + i];
      val = v_n[l] + dt * (float)g * ((float)rho0 - rf) / (float)rho0;
      bool open;
      if (j < ny) {
        const uint8_t c = cell[j * nx + i];
        open = !(c & C_SOLID) && (c & C_S);
      } else {
        open = !(cell[(ny - 1) * nx + i] & C_SOLID);
      }
      val = open ? val : 0.f;
    }
    v[l] = val;
  }
}

__global__ __launch_bounds__(256) void advect_pass3(int nx, int ny, const float* __restrict__ rho_n,
                                                    const float* __restrict__ u_n,
                                                    const float* __restrict__ v_n,
                                                    const uint8_t* __restrict__ cell,
                                                    const float* __restrict__ xi, double g,
                                                    double rho0, double drho, double u_in,
                                                    float* __restrict__ rho, float* __restrict__ u,
                                                    float* __restrict__ v, const Scalars* sc) {
  pass3_body(blockIdx.x * blockDim.x + threadIdx.x, nx, ny, rho_n, u_n, v_n, cell, xi, g, rho0,
             drho, u_in, rho, u, v, sc);
}

// the sample grids and temporaries of one instance (workspace adv area)
__host__ __device__ __forceinline__ AdvPtrs adv_ptrs(int nx, int ny, const float* rho, const float* u,
                                                     const float* v, float* adv) {
  const int n = nx * ny, nu = ny * (nx + 1), nv = (ny + 1) * nx;
  AdvPtrs A{};
  A.q[0] = rho; A.q[1] = u; A.q[2] = v;
  A.hat[0] = adv; A.hat[1] = adv + n; A.hat[2] = adv + n + nu;
  float* o = adv + n + nu + nv;
  A.out[0] = o; A.out[1] = o + n; A.out[2] = o + n + nu;
  A.H[0] = ny; A.W[0] = nx; A.H[1] = ny; A.W[1] = nx + 1; A.H[2] = ny + 1; A.W[2] = nx;
  A.n0 = n; A.n1 = nu; A.n2 = nv;
  return A;
}

hipError_t run_advect(int nx, int ny, double dx, double g, double rho0, double drho, double u_in,
                      double cfl, float* rho, float* u, float* v, const float* xi, const Ws& w,
                      hipStream_t s) {
  const int n = nx * ny, nu = ny * (nx + 1), nv = (ny + 1) * nx;
  const int nbf = (nu + nv + 255) / 256;
  if ((size_t)nbf > w.blockpart_n) return hipErrorInvalidValue;
  cfl_kernel<<<nbf, 256, 0, s>>>(nu, nv, u, v, w.blockpart);
  cfl_finish<<<1, 256, 0, s>>>(nbf, w.blockpart, dx, cfl, u_in, w.sc);
  const AdvPtrs A = adv_ptrs(nx, ny, rho, u, v, w.adv);
  const int tot = n + nu + nv, nb = (tot + 255) / 256;
  const float inv_dx = (float)(1.0 / dx);
  advect_pass1<<<nb, 256, 0, s>>>(A, nx, ny, inv_dx, u, v, w.sc);
  advect_pass2<<<nb, 256, 0, s>>>(A, nx, ny, inv_dx, u, v, w.sc);
  advect_pass3<<<nb, 256, 0, s>>>(nx, ny, A.out[0], A.out[1], A.out[2], w.cell, xi, g, rho0, drho,
                                  u_in, rho, u, v, w.sc);
  return hipGetLastError();
}

// ---- batched: one launch per pass over all instances (batch.h) ------------
__device__ __forceinline__ int adv_loc(const int* __restrict__ first, int n, int* lb) {
  const int i = batch_find(first, n, blockIdx.x);
  *lb = blockIdx.x - first[i];
  return i;
}

__global__ __launch_bounds__(256) void cfl_batch(const BInst* __restrict__ I, const int* first, int n) {
  __shared__ double red[4];
  int lb;
  const BInst& B = I[adv_loc(first, n, &lb)];
  const int nu = B.ny * (B.nx + 1), nv = (B.ny + 1) * B.nx;
  cfl_body(lb * blockDim.x + threadIdx.x, nu, nv, B.u, B.v, B.w.blockpart + lb, red);
}

__global__ __launch_bounds__(256) void cfl_finish_batch(const BInst* __restrict__ I, const int* first) {
  __shared__ double red[4];
  const BInst& B = I[blockIdx.x];
  cfl_finish_body(first[blockIdx.x + 1] - first[blockIdx.x], B.w.blockpart, B.dx, B.cfl, B.u_in,
                  B.w.sc, red);
}

template <int PASS>
__global__ __launch_bounds__(256) void advect_batch(const BInst* __restrict__ I, const int* first, int n) {
  int lb;
  const BInst& B = I[adv_loc(first, n, &lb)];
  const int gid = lb * blockDim.x + threadIdx.x;
  const AdvPtrs A = adv_ptrs(B.nx, B.ny, B.rho, B.u, B.v, B.w.adv);
  const float inv_dx = (float)(1.0 / B.dx);
  if constexpr (PASS == 1) pass1_body(A, gid, B.nx, B.ny, inv_dx, B.u, B.v, B.w.sc);
  else if constexpr (PASS == 2) pass2_body(A, gid, B.nx, B.ny, inv_dx, B.u, B.v, B.w.sc);
  else
    pass3_body(gid, B.nx, B.ny, A.out[0], A.out[1], A.out[2], B.w.cell, B.xi, B.g, B.rho0, B.drho,
               B.u_in, B.rho, B.u, B.v, B.w.sc);
}

hipError_t run_advect_batch(const BInst* I, const BatchRanges& R, hipStream_t s) {
  if (R.total[RK_FACE] > 0) cfl_batch<<<R.total[RK_FACE], 256, 0, s>>>(I, R.of(RK_FACE), R.n);
  cfl_finish_batch<<<R.n, 256, 0, s>>>(I, R.of(RK_FACE));
  const int nb = R.total[RK_ADV];
  if (nb > 0) {
    advect_batch<1><<<nb, 256, 0, s>>>(I, R.of(RK_ADV), R.n);
    advect_batch<2><<<nb, 256, 0, s>>>(I, R.of(RK_ADV), R.n);
    advect_batch<3><<<nb, 256, 0, s>>>(I, R.of(RK_ADV), R.n);
  }
  return hipGetLastError();
}

}  // namespace hyp
