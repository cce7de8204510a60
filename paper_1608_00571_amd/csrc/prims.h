// Wavefront (64-lane) and work-group primitives for CDNA4.
//
// These implement the co-operative side of the work-together principle
// (Section 3.2, Tenet 2): prefix sums by ballot + mbcnt inside a wavefront,
// wavefront totals combined through LDS, and a single device-scope atomic
// per work-group segment instead of one per task.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trees {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// popcount(mask & lanes-below-me): the mbcnt instruction pair.
__device__ __forceinline__ int mbcnt64(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return (uint64_t)__ballot(p); }

// Exclusive wavefront prefix of small non-negative values v < 2^BITS, one
// ballot per bit; *total receives the wavefront sum.
template <int BITS>
__device__ __forceinline__ int wave_prefix_small(int v, int *total) {
  int pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    uint64_t m = ballot64((v >> b) & 1);
    pre += mbcnt64(m) << b;
    tot += __popcll(m) << b;
  }
  *total = tot;
  return pre;
}

// Inclusive wavefront scan of arbitrary ints (shuffle-up ladder).
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive work-group scan of ints; returns the prefix and writes the
// work-group total to *total.  `tmp` holds WG/64 + 1 ints of LDS.  Must be
// called by every thread of the work-group.
template <int WG>
__device__ __forceinline__ int wg_excl_scan(int v, int *tmp, int *total) {
  constexpr int NW = WG / 64;
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  int inc = wave_incl_scan(v);
  if (lane == 63) tmp[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) { int t = tmp[w]; tmp[w] = s; s += t; }
    tmp[NW] = s;
  }
  __syncthreads();
  int r = tmp[wave] + inc - v;
  *total = tmp[NW];
  __syncthreads();
  return r;
}

// 64-bit variant of wg_excl_scan (`tmp` holds WG/64 + 1 int64 of LDS).
__device__ __forceinline__ int64_t wave_incl_scan64(int64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}
template <int WG>
__device__ __forceinline__ int64_t wg_excl_scan64(int64_t v, int64_t *tmp, int64_t *total) {
  constexpr int NW = WG / 64;
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  int64_t inc = wave_incl_scan64(v);
  if (lane == 63) tmp[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) { int64_t t = tmp[w]; tmp[w] = s; s += t; }
    tmp[NW] = s;
  }
  __syncthreads();
  int64_t r = tmp[wave] + inc - v;
  *total = tmp[NW];
  __syncthreads();
  return r;
}

// Device-scope loads/stores of words that other work-groups update with
// atomics (they bypass the non-coherent per-XCD L2).
template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T add_agent(T *p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T or_agent(T *p, T v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until this wavefront's vector memory operations (loads, stores,
// atomics) have completed: s_waitcnt vmcnt(0), leaving the other counters.
// Stores are then in the XCD's L2 and atomics performed, with no L2 write-back.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Release / acquire at agent scope.  On this chip a release writes back the
// XCD's L2 and an acquire invalidates it (the L2s of the 8 XCDs are not
// coherent with each other), so they are paid once per work-group per epoch
// at the epoch barrier (Tenet 1), never per task or per wavefront.
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ __forceinline__ int64_t realtime() { return (int64_t)wall_clock64(); }

}  // namespace trees
