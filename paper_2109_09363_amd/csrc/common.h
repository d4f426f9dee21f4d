// Internal device helpers shared by the hyproj kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace hyp {

constexpr int kWave = 64;

// Planned cell byte (written by the planner, read by every stencil):
//   bit0 solid (after the pocket fill), bit1 inflow face below,
//   bit2 E, bit3 W, bit4 N, bit5 S: that neighbour is a non-solid cell
//   (N is also set on the top row: the open ghost row).
enum : uint8_t {
  C_SOLID = 1, C_INFLOW = 2, C_E = 4, C_W = 8, C_N = 16, C_S = 32
};

// ---- global-memory access through pointers held in descriptors ------------
// A pointer read from memory (a descriptor table, a struct picked by a
// run-time index) is generic to the compiler, which then emits flat loads
// and stores.  Flat operations also count against the LDS wait counter, so
// every LDS wait of the kernel waits for them too: a prefetch issued before
// LDS-fed math stalls the first LDS read.  These accessors state that the
// memory is global.
template <typename T> using gmem = __attribute__((address_space(1))) T;
template <typename T> __device__ __forceinline__ T gld(const T* p) { return *(const gmem<T>*)p; }
template <typename T> __device__ __forceinline__ void gst(T* p, const T& v) { *(gmem<T>*)p = v; }
// Read-only data that every lane of a wave reads at one address (launch
// descriptors, also those indexed at run time): the constant address space
// gives scalar loads.
// Structs are copied word by word (a class copy cannot bind a reference in
// another address space).
template <typename T> using cmem = __attribute__((address_space(4))) T;
template <typename T> __device__ __forceinline__ T cld(const T* p) {
  static_assert(sizeof(T) % 4 == 0 && alignof(T) >= 4, "whole aligned words");
  T v;
  const cmem<uint32_t>* s = (const cmem<uint32_t>*)p;
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = s[i];
  return v;
}
template <typename T> __device__ __forceinline__ T cld(const T* p, int i) { return cld(p + i); }
__device__ __forceinline__ int cld_int(const int* p) { return *(const cmem<int>*)p; }

__device__ __forceinline__ int cell_k(uint8_t c) { return __popc((c >> 2) & 15u); }
__device__ __forceinline__ bool cell_fluid(uint8_t c) { return !(c & C_SOLID); }

// ---- wave / block reductions (fixed order, deterministic) ----------------
// Sums use DPP row shifts and row broadcasts (VALU rate; no LDS permutes).
// 64-bit DPP move of a double, lanes without a source (or in a disabled row)
// receive 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum over the 64 lanes of a wave with row shifts and row broadcasts (no LDS
// permutes); the result is valid in every lane.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0x111, 0xF>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xF>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xF>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xF>(v);  // row_shr:8  -> lane 15 of each row: the row sum
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3 -> lane 63: total
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
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
  v = wave_sum_dpp(v);
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += scratch[i];
  return t;
}
// Three block reductions in one exchange through shared memory: the sums of
// a and c, and the sum (or, with e_max, the maximum) of e, valid in every
// thread.  `scratch` must hold 3 * blockDim.x/64 doubles.
__device__ __forceinline__ void block_sum3(double& a, double& c, double& e, bool e_max,
                                           double* scratch) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  a = wave_sum_dpp(a);
  c = wave_sum_dpp(c);
  e = e_max ? wave_max(e) : wave_sum_dpp(e);
  __syncthreads();
  if (lane == 0) {
    scratch[3 * w] = a;
    scratch[3 * w + 1] = c;
    scratch[3 * w + 2] = e;
  }
  __syncthreads();
  a = 0.0;
  c = 0.0;
  e = e_max ? scratch[2] : 0.0;
  for (int i = 0; i < nw; ++i) {
    a += scratch[3 * i];
    c += scratch[3 * i + 1];
    e = e_max ? fmax(e, scratch[3 * i + 2]) : e + scratch[3 * i + 2];
  }
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
// L2 write-back/invalidate fences.  Every wave first waits until its own
// memory operations have completed (s_waitcnt 0: a workgroup-scope fence does
// not wait for stores on this target, and an arrival could otherwise overtake
// the data it announces).  Arrival is two-level: work-groups count on the
// counter of their group of kSyncGroup consecutive blocks (each counter on its
// own 128-byte line), the last of a group counts on the top counter, and the
// last of all raises the generation flag.  One thread per work-group polls
// that flag: agent-scope polling bypasses the L2, and more pollers (one per
// group counter, say) measurably slow every work-group's stores.  Barrier
// number n (1, 2, ...) passes when all `nblocks` work-groups have arrived n
// times.  Slot i of the sync area is the word sync[32 i]: 0 top counter,
// 1 flag, 2 + g group g; all are zeroed before a launch (sync_clear).
__device__ __forceinline__ void sync_clear(unsigned* sync, int i) {
  if (i >= 0 && i < kSyncSlots) sync[32 * i] = 0;
}

// Every wait is bounded (kSpinTicks of the constant 100 MHz wall clock):
// returns false in every thread of a work-group that gave up, so that a
// persistent kernel can end instead of hanging on a lost arrival.
constexpr uint64_t kSpinTicks = 200000000ull;  // 2 s

__device__ __forceinline__ bool grid_barrier_bounded(unsigned* sync, unsigned n, unsigned nblocks) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int ok = 1;
  if (threadIdx.x == 0) {
    const unsigned ng = (nblocks + kSyncGroup - 1) / kSyncGroup, g = blockIdx.x / kSyncGroup;
    const unsigned gs = (g == ng - 1) ? nblocks - kSyncGroup * (ng - 1) : kSyncGroup;
    const unsigned old = __hip_atomic_fetch_add(sync + 32 * (2 + g), 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old == n * gs - 1) {
      const unsigned top = __hip_atomic_fetch_add(sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (top == n * ng - 1) __hip_atomic_store(sync + 32, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint64_t t0 = (uint64_t)wall_clock64();
    while (__hip_atomic_load(sync + 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n) {
      if ((uint64_t)wall_clock64() - t0 > kSpinTicks) { ok = 0; break; }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  return __syncthreads_and(ok) != 0;
}

// The same barrier for kernels without an abort path (the bounded wait can
// only give up on a lost arrival, which a correct launch never has).
__device__ __forceinline__ void grid_barrier(unsigned* sync, unsigned n, unsigned nblocks) {
  (void)grid_barrier_bounded(sync, n, nblocks);
}

// Relaxed agent-scope loads and stores of global memory (data that other
// work-groups read or wrote), in the global address space like gld/gst.
__device__ __forceinline__ void st_agent(float* p, float v) {
  __hip_atomic_store((gmem<float>*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float* p) {
  return __hip_atomic_load((gmem<float>*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store((gmem<unsigned long long>*)p, static_cast<unsigned long long>(__double_as_longlong(v)),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __longlong_as_double(static_cast<long long>(
      __hip_atomic_load((gmem<unsigned long long>*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
}
__device__ __forceinline__ void st_agent(uint8_t* p, uint8_t v) {
  // byte stores: go through a 32-bit atomic OR/AND pair on the containing word
  gmem<unsigned>* w = (gmem<unsigned>*)(reinterpret_cast<uintptr_t>(p) & ~(uintptr_t)3);
  const unsigned sh = (unsigned)(reinterpret_cast<uintptr_t>(p) & 3) * 8;
  __hip_atomic_fetch_and(w, ~(0xFFu << sh), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_or(w, (unsigned)v << sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint8_t ld_agent(const uint8_t* p) {
  gmem<unsigned>* w = (gmem<unsigned>*)(reinterpret_cast<uintptr_t>(p) & ~(uintptr_t)3);
  const unsigned sh = (unsigned)(reinterpret_cast<uintptr_t>(p) & 3) * 8;
  return (uint8_t)(__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> sh);
}

__device__ __forceinline__ void st_agent(int* p, int v) {
  __hip_atomic_store((gmem<int>*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load((gmem<int>*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned* p, unsigned v) {
  __hip_atomic_store((gmem<unsigned>*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_agent(const unsigned* p) {
  return __hip_atomic_load((gmem<unsigned>*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store((gmem<uint64_t>*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load((gmem<uint64_t>*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// lane l receives x from lane l-1 (lane 0 receives 0): DPP wave_shr:1 with
// bound_ctrl, so the lane without a source reads 0 and no old value is needed
__device__ __forceinline__ float from_left(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xF, 0xF, true));
}
// lane l receives x from lane l+1 (lane 63 receives 0): DPP wave_shl:1
__device__ __forceinline__ float from_right(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xF, 0xF, true));
}

// Sum of `n` doubles in global memory written by other work-groups, in a
// fixed order, so that every work-group obtains the bit-identical value.
// Each thread adds its strided share in index order; the loads go out
// eight at a time before the adds, so that a long list costs n / (8 x
// threads) round trips instead of n / threads (same order, same result).
__device__ __forceinline__ double sum_partials(const double* part, int n, double* scratch) {
  double v = 0.0;
  const int T = blockDim.x;
  int i = threadIdx.x;
  for (; i + 7 * T < n; i += 8 * T) {
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = ld_agent(part + i + k * T);
#pragma unroll
    for (int k = 0; k < 8; ++k) v += t[k];
  }
  for (; i < n; i += T) v += ld_agent(part + i);
  return block_sum(v, scratch);
}

}  // namespace hyp
