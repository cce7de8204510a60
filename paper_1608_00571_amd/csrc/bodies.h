// Serial parts of the task bodies (one lane each).  The fork / join / emit
// side of every body lives in the epoch sweep, which does it co-operatively.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trees {

// Merge-sort leaf: insertion sort of keys[lo, hi) into the buffer of its
// depth d (d even: in place in keys; d odd: into tmp).
__device__ __forceinline__ void ms_leaf(uint32_t *keys, uint32_t *tmp, int32_t lo, int32_t hi,
                                        int32_t d) {
  uint32_t *dst = (d & 1) ? tmp : keys;
  if (d & 1)
    for (int32_t k = lo; k < hi; ++k) dst[k] = keys[k];
  for (int32_t k = lo + 1; k < hi; ++k) {
    uint32_t x = dst[k];
    int32_t j = k - 1;
    while (j >= lo) {
      uint32_t y = dst[j];
      if (y <= x) break;
      dst[j + 1] = y;
      --j;
    }
    dst[j + 1] = x;
  }
}

// Merge of the two sorted halves of [lo, hi) written by the children (depth
// d + 1) into the buffer of depth d.
__device__ __forceinline__ void ms_merge(uint32_t *keys, uint32_t *tmp, int32_t lo, int32_t hi,
                                         int32_t d) {
  const uint32_t *src = ((d + 1) & 1) ? tmp : keys;
  uint32_t *dst = (d & 1) ? tmp : keys;
  const int32_t mid = lo + (hi - lo) / 2;
  int32_t i = lo, j = mid, k = lo;
  if (i < mid && j < hi) {
    uint32_t x = src[i], y = src[j];
    while (true) {
      if (y < x) {
        dst[k++] = y;
        if (++j == hi) break;
        y = src[j];
      } else {
        dst[k++] = x;
        if (++i == mid) break;
        x = src[i];
      }
    }
  }
  while (i < mid) dst[k++] = src[i++];
  while (j < hi) dst[k++] = src[j++];
}

// Co-operative leaf sort (Tenet 2): the whole wavefront sorts one run of at
// most 64 keys, one key per lane, with a bitonic network of lane exchanges.
// Lanes beyond the run hold the largest key, so the first n lanes end up with
// the run's keys in order.  Must be called by all 64 lanes.
// B independent runs go through the network together, so the lane exchanges
// of different runs overlap instead of waiting on each other.
template <int B>
__device__ __forceinline__ void wave_bitonic64(uint32_t (&v)[B]) {
  const int lane = (int)__lane_id();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const bool up = (lane & k) == 0;          // this k-block sorts ascending
      const bool low = (lane & j) == 0;         // lower partner keeps the smaller key
      uint32_t w[B];
#pragma unroll
      for (int b = 0; b < B; ++b) w[b] = (uint32_t)__shfl_xor((int)v[b], j, 64);
#pragma unroll
      for (int b = 0; b < B; ++b) v[b] = (low == up) ? min(v[b], w[b]) : max(v[b], w[b]);
    }
  }
}

// Merge path: how many of the first q outputs of merging A (na keys) and B
// (nb keys) come from A, when equal keys are taken from A first.
__device__ __forceinline__ int64_t merge_path(const uint32_t *A, int64_t na, const uint32_t *B,
                                              int64_t nb, int64_t q) {
  int64_t lo = q > nb ? q - nb : 0;
  int64_t hi = q < na ? q : na;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (A[mid] <= B[q - mid - 1]) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

}  // namespace trees
