// Map phase of the merge-sort continuation (Section 4.2): device code shared
// by the standalone map kernels and the batched epoch kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bodies.h"
#include "prims.h"
#include "trees_dev.h"

namespace trees {

// ---------------------------------------------------------------------------
// Map phase: the merges registered in the last epoch, co-operatively, in two
// passes.  The jobs' outputs are laid end to end (a job of m keys owns m
// consecutive units) and cut into tiles of kMapTile units.
//  * partition: one wavefront per tile boundary finds the job holding the
//    boundary unit (64-ary search over the job offsets) and the merge-path
//    split there (k-ary search along the diagonal);
//  * merge: a work-group per tile stages the input runs of every job
//    portion the tile covers in LDS with coalesced loads, and each lane
//    merges its run of consecutive outputs out of LDS and stores it.
// ---------------------------------------------------------------------------
constexpr int kMaxPortions = 72;   // merge jobs exceed 64 keys, so a tile meets at most 65

struct MapLds {
  uint32_t in[kMapTile];
  int32_t pbase[kMaxPortions + 1];   // tile-relative first output of each portion
  int32_t pna[kMaxPortions];         // keys the portion takes from the job's first half
  int64_t pas[kMaxPortions], pbs[kMaxPortions];   // first key taken from each half
  int64_t pqs[kMaxPortions];         // job-relative first output of the portion
  int64_t plo[kMaxPortions], pmid[kMaxPortions];
  const uint32_t *psrc[kMaxPortions];
  uint32_t *pdst[kMaxPortions];
  int32_t P;
  uint32_t J;
  uint64_t U;
};

// k-ary merge-path search by one wavefront (all 64 lanes): the number of the
// first q outputs that come from A, equal keys taken from A first.  Wide
// ranges take 64 probes a round (each probe reads its own line anyway, and
// the early rounds are shared by neighbouring tiles in L2); once the probes
// would be closer than 64 keys, 8 probes a round read 8x fewer lines, and
// the last round scans the remaining <= 64 keys with every lane.
__device__ __forceinline__ int64_t wave_merge_path(const uint32_t *A, int64_t na, const uint32_t *B,
                                                   int64_t nb, int64_t q) {
  const int lane = lane_id();
  int64_t lo = q > nb ? q - nb : 0;
  int64_t hi = q < na ? q : na;
  while (lo < hi) {
    const int64_t r = hi - lo;
    const int ar = (r > 64 * 64 || r <= 64) ? 64 : 8;
    const int64_t step = (r + ar - 1) / ar;
    const int64_t pos = lo + (int64_t)lane * step;
    const bool t = lane < ar && pos < hi && A[pos] <= B[q - pos - 1];
    const int c = __popcll(ballot64(t));
    if (c == 0) {
      hi = lo;
    } else {
      const int64_t nlo = lo + (int64_t)(c - 1) * step + 1;
      hi = min(lo + (int64_t)c * step, hi);
      lo = nlo;
    }
  }
  return lo;
}

__device__ __forceinline__ int portion_of(const MapLds &M, int e) {
  int lo = 0, hi = M.P;   // last portion whose base is <= e
  while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (M.pbase[mid] <= e) lo = mid; else hi = mid; }
  return lo;
}

// Number of usable jobs and the unit count they cover.
__device__ __forceinline__ void map_extent(const DevCtx &C, uint32_t Jraw, uint32_t *J, uint64_t *U) {
  *J = min(Jraw, (uint32_t)C.mj_cap);
  *U = *J ? C.mj_off[*J - 1] + (uint64_t)(C.mj_hi[*J - 1] - C.mj_lo[*J - 1]) : 0;
  const uint64_t maxU = (uint64_t)(C.part_cap - 1) * kMapTile;
  if (*U > maxU) *U = maxU;   // (never for the sizes the arena admits)
}

// Pass 1: the split at every tile boundary.  `wid` / `nwaves` enumerate the
// wavefronts taking part.
__device__ void map_partition(const DevCtx &C, uint32_t J, uint64_t U, int64_t wid, int64_t nwaves) {
  const uint64_t nb = (U + kMapTile - 1) / kMapTile + 1;   // boundaries 0 .. ntiles
  const int lane = lane_id();
  // each wavefront takes a contiguous run of boundaries
  const uint64_t per = (nb + (uint64_t)nwaves - 1) / (uint64_t)nwaves;
  const uint64_t tb = (uint64_t)wid * per, te = min(tb + per, nb);
  for (uint64_t t = tb; t < te; ++t) {
    const uint64_t u = min(t * kMapTile, U);
    uint32_t lo = 0, hi = J;   // last job whose offset is <= u (u = U: the last job)
    while (hi - lo > 1) {
      const uint32_t step = (hi - lo + 63) >> 6;
      const uint32_t p = lo + (uint32_t)lane * step;
      const bool ok = p < hi && C.mj_off[p] <= u;
      const int j = __popcll(ballot64(ok)) - 1;
      lo = lo + (uint32_t)j * step;
      hi = min(lo + step, hi);
    }
    const int64_t jlo = C.mj_lo[lo], jhi = C.mj_hi[lo];
    const int64_t mid = jlo + (jhi - jlo) / 2;
    const uint32_t *src = C.mj_src[lo];
    const int64_t q = (int64_t)(u - C.mj_off[lo]);
    const int64_t ia = wave_merge_path(src + jlo, mid - jlo, src + mid, jhi - mid, q);
    if (lane == 0) { C.part_job[t] = lo; C.part_ia[t] = ia; }
  }
}

// Pass 2: merge tiles.  Every thread of the work-group takes part.
template <int WG>
__device__ void map_merge(const DevCtx &C, MapLds &M, uint32_t J, uint64_t U) {
  constexpr int K = kMapTile / WG;
  const uint64_t ntiles = (U + kMapTile - 1) / kMapTile;
  const int tid = threadIdx.x;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t u0 = tile * kMapTile;
    const uint64_t u1 = min(u0 + (uint64_t)kMapTile, U);
    const int tl = (int)(u1 - u0);
    const uint32_t j0 = C.part_job[tile], j1 = C.part_job[tile + 1];
    const int64_t ia0 = C.part_ia[tile], ia1 = C.part_ia[tile + 1];
    const int n = (int)(j1 - j0) + 1;   // jobs j0 .. j1 (j1 may start exactly at u1)
    if (tid < n && tid < kMaxPortions) {
      const uint32_t j = j0 + tid;
      const uint64_t off = C.mj_off[j];
      const int64_t lo = C.mj_lo[j], hi = C.mj_hi[j];
      const int64_t mid = lo + (hi - lo) / 2;
      const uint64_t ts0 = max(u0, off);
      const uint64_t te0 = min(u1, off + (uint64_t)(hi - lo));
      const int64_t qs = (int64_t)(ts0 - off), qe = (int64_t)(te0 - off);
      const int64_t as = (j == j0) ? ia0 : 0;
      const int64_t ae = (j == j1 && te0 == u1 && u1 - off == (uint64_t)qe) ? ia1 : (mid - lo);
      M.pbase[tid] = (int32_t)(ts0 - u0);
      M.pqs[tid] = qs;
      M.plo[tid] = lo;
      M.pmid[tid] = mid;
      M.pas[tid] = as;
      M.pbs[tid] = qs - as;
      M.pna[tid] = (int32_t)(ae - as);
      M.psrc[tid] = C.mj_src[j];
      M.pdst[tid] = C.mj_dst[j];
    }
    if (tid == 0) {
      // the job starting exactly at the tile's end contributes nothing
      const int P = (n > 1 && C.mj_off[j1] >= u1) ? n - 1 : n;
      M.P = min(P, kMaxPortions);
      M.pbase[M.P] = tl;
    }
    __syncthreads();
    // stage the inputs: portion k's first-half keys then its second-half keys
    for (int e = tid; e < tl; e += WG) {
      const int k = portion_of(M, e);
      const int r = e - M.pbase[k];
      const uint32_t *src = M.psrc[k];
      M.in[e] = (r < M.pna[k]) ? src[M.plo[k] + M.pas[k] + r] : src[M.pmid[k] + M.pbs[k] + (r - M.pna[k])];
    }
    __syncthreads();
    // every lane merges K consecutive outputs out of LDS
    {
      int e = tid * K;
      const int e1 = min(e + K, tl);
      while (e < e1) {
        const int k = portion_of(M, e);
        const int base = M.pbase[k];
        const int len = M.pbase[k + 1] - base;
        const int na = M.pna[k], nb = len - na;
        const uint32_t *A = M.in + base;
        const uint32_t *B = A + na;
        const int o = e - base;
        int lo = o > nb ? o - nb : 0, hi = o < na ? o : na;
        while (lo < hi) { const int mid = (lo + hi) >> 1; if (A[mid] <= B[o - mid - 1]) lo = mid + 1; else hi = mid; }
        int ia = lo, ib = o - lo;
        const int cnt = min(e1 - e, len - o);
        uint32_t *out = M.pdst[k] + M.plo[k] + M.pqs[k] + o;
        for (int t = 0; t < cnt; ++t) {
          const bool takeA = ib >= nb || (ia < na && A[ia] <= B[ib]);
          out[t] = takeA ? A[ia++] : B[ib++];
        }
        e += cnt;
      }
    }
    __syncthreads();
  }
}

}  // namespace trees
