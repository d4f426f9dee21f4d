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
// Data that crosses work-groups is written and read with agent-scope atomic
// stores/loads (coherent across the XCD L2 caches), so the barrier needs no
// L2 write-back/invalidate fences: every wave waits for its own stores
// (workgroup-scope release fence), the work-group arrives on a counter, the
// last arriver raises a generation flag on its own cache line, and everyone
// polls the flag.  `sync[0]` (counter) and `sync[32]` (flag) are zeroed
// before the launch; barrier number n (1, 2, ...) passes when all `nblocks`
// work-groups have arrived n times.
__device__ __forceinline__ void grid_barrier(unsigned* sync, unsigned n, unsigned nblocks) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned old = __hip_atomic_fetch_add(sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == n * nblocks - 1)
      __hip_atomic_store(sync + 32, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (__hip_atomic_load(sync + 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n)
      __builtin_amdgcn_s_sleep(2);
  }
  __syncthreads();
}

__device__ __forceinline__ void st_agent(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float* p) {
  return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     static_cast<unsigned long long>(__double_as_longlong(v)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint8_t* p, uint8_t v) {
  // byte stores: go through a 32-bit atomic OR/AND pair on the containing word
  unsigned* w = reinterpret_cast<unsigned*>(reinterpret_cast<uintptr_t>(p) & ~(uintptr_t)3);
  const unsigned sh = (unsigned)(reinterpret_cast<uintptr_t>(p) & 3) * 8;
  __hip_atomic_fetch_and(w, ~(0xFFu << sh), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_or(w, (unsigned)v << sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint8_t ld_agent(const uint8_t* p) {
  const unsigned* w = reinterpret_cast<const unsigned*>(reinterpret_cast<uintptr_t>(p) & ~(uintptr_t)3);
  const unsigned sh = (unsigned)(reinterpret_cast<uintptr_t>(p) & 3) * 8;
  return (uint8_t)(__hip_atomic_load(const_cast<unsigned*>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> sh);
}

// lane l receives x from lane l-1 (lane 0 receives 0): DPP wave_shr:1
__device__ __forceinline__ float from_left(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xF, 0xF, false));
}
// lane l receives x from lane l+1 (lane 63 receives 0): DPP wave_shl:1
__device__ __forceinline__ float from_right(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xF, 0xF, false));
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
