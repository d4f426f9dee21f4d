// Internal device helpers shared by the hyproj kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hyp {

constexpr int kWave = 64;

// Planned cell byte (written by the planner, read by every stencil):
//   bit0 solid (after the pocket fill), bit1 inflow face below,
//   bit2 E, bit3 W, bit4 N, bit5 S: that neighbour is a non-solid cell
//   (N is also set on the top row: the open ghost row).
enum : uint8_t {
  C_SOLID = 1, C_INFLOW = 2, C_E = 4, C_W = 8, C_N = 16, C_S = 32
};

__device__ __forceinline__ int cell_k(uint8_t c) { return __popc((c >> 2) & 15u); }
__device__ __forceinline__ bool cell_fluid(uint8_t c) { return !(c & C_SOLID); }

// ---- wave / block reductions (fixed order, deterministic) ----------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, kWave));
  return v;
}

// Sum over the block; the result is valid in every thread.  `scratch` must
// hold blockDim.x/64 doubles of shared memory.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += scratch[i];
  return t;
}
__device__ __forceinline__ double block_max(double v, double* scratch) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double t = scratch[0];
  for (int i = 1; i < nw; ++i) t = fmax(t, scratch[i]);
  return t;
}

// ---- grid-wide barrier for cooperative (co-resident) launches ------------
// `counter` is zeroed before the launch; barrier number `n` (1, 2, ...) is
// passed when all `nblocks` work-groups have arrived `n` times.  Release and
// acquire fences at agent scope make every global write issued before the
// barrier visible to every work-group after it (across XCD L2s).
__device__ __forceinline__ void grid_barrier(unsigned* counter, unsigned target) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
  }
  __syncthreads();
}

// Sum of `n` doubles in global memory written by other work-groups, in a
// fixed order, so that every work-group obtains the bit-identical value.
__device__ __forceinline__ double sum_partials(const double* part, int n, double* scratch) {
  double v = 0.0;
  const unsigned long long* p = reinterpret_cast<const unsigned long long*>(part);
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    v += __longlong_as_double(static_cast<long long>(
        __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
  return block_sum(v, scratch);
}

}  // namespace hyp
