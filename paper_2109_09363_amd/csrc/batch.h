// Device-side description of a batch of plumes of uneven sizes, shared by
// the batched launches of every phase of a time step (advection, boundary
// faces + divergence, network, Jacobi, gradient correction): each launch
// covers all instances at once, its work-groups mapped to (instance, local
// work-group) through a prefix table of per-instance work-group counts.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/hyproj.h"
#include "internal.h"

namespace hyp {

constexpr int kBatchMaxScales = 5;
constexpr int kBatchSweeps = 8;  // Jacobi sweeps of a tile between halo exchanges

// Work ranges: per instance, the number of work-groups of each launch shape.
enum BatchRange {
  RK_CELL = 0,   // 256 cells per work-group (divergence, gradient, check, init, coefficients)
  RK_FACE = 1,   // 256 faces per work-group (CFL maximum)
  RK_ADV = 2,    // 256 sample points (cells, u faces, v faces) per work-group (advection)
  RK_REG = 3,    // 32 x 32 regions (network input pyramid)
  RK_LVL0 = 4,   // 256 pixels of pyramid level k per work-group: RK_LVL0 + k (upsample-sum)
  RK_COUNT = RK_LVL0 + kBatchMaxScales
};

struct BInst {
  int nx, ny;
  double dx, rho0;
  double dt;                 // p = rho0 phi / dt when the step computed no dt
  double g, drho, u_in, cfl; // physics of this instance's time step
  int var;                   // variable-density operator
  int S;                     // network scales (0: none)
  float* u;
  float* v;
  float* rho;
  float* p;
  const float* xi;
  const uint8_t* flags;
  hyp_result* res;
  Ws w;                      // this instance's workspace
  int sc_h[kBatchMaxScales], sc_w[kBatchMaxScales];
  size_t sc_off_px[kBatchMaxScales];
};

// The instance of work-group b of a range: the largest i with first[i] <= b
// (first holds n + 1 prefix sums; instances with no work-groups are skipped).
__device__ __forceinline__ int batch_find(const int* __restrict__ first, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Host view of the range tables: first[r * (n + 1) + i], and the total
// work-groups of each range.
struct BatchRanges {
  const int* first;  // device, RK_COUNT x (n + 1)
  int total[RK_COUNT];
  int n;
  const int* of(int r) const { return first + (size_t)r * (n + 1); }
};

// Device tables of a batch (in its area) and the launch sizes.
struct BatchDevice {
  BInst* binst;
  void* cnn_tables;
  hyp_result* results;  // one per instance, copied to the caller's at the end
  BatchRanges ranges;
};

int batch_rows_of(int nx, int ny, bool var, int forced);
int batch_tiles_of(int nx, int ny, int R);
size_t batch_area_bytes(int n, int ntiles, size_t cnn_bytes);
BatchDevice batch_device(void* area, int n, int ntiles, size_t cnn_bytes);
hipError_t batch_setup(void* area, int n, int ntiles, size_t cnn_bytes, const BInst* binst,
                       const int* rows, const double* thr, int max_iters, float omega,
                       BatchDevice* out);
int batch_tile_mode(int n, const int* rows, bool var);
hipError_t run_jacobi_batch(const Device& dev, void* area, int n, int ntiles, size_t cnn_bytes,
                            int mode, int test_passes, int max_iters, bool cooperative,
                            hipStream_t s);
hipError_t run_div_batch(const BInst* I, const BatchRanges& R, hipStream_t s);
hipError_t run_coef_batch(const BInst* I, const BatchRanges& R, hipStream_t s);
hipError_t run_init_phi_batch(const BInst* I, const BatchRanges& R, hipStream_t s);
hipError_t run_grad_finish_batch(const BInst* I, const BatchRanges& R, bool dt_dev, bool var,
                                 hipStream_t s);
hipError_t run_advect_batch(const BInst* I, const BatchRanges& R, hipStream_t s);
size_t cnn_batch_bytes(const NetShape& net, int n);
hipError_t cnn_batch_setup(const NetShape& net, int n, const WsLayout* Ly, const Ws* ws,
                           const float* params, void* dev_tables, int* tiles);
hipError_t run_cnn_batch(const Device& dev, const NetShape& net, const BInst* I,
                         const BatchRanges& R, const void* tables, const int* tiles, const Ws& w0,
                         const float* params, hipStream_t s);

}  // namespace hyp
