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

}  // namespace trees
