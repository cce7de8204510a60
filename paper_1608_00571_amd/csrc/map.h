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
// consecutive units) and cut into tiles of TILE units.
//  * partition: one wavefront per tile boundary finds the job holding the
//    boundary unit (64-ary search over the job offsets) and the merge-path
//    split there (k-ary search along the diagonal);
//  * merge: a work-group per tile loads the input runs of every job portion
//    the tile covers into LDS (all of a lane's loads in flight together),
//    each lane merges a run of consecutive outputs into registers, the
//    outputs go back to the same LDS buffer, and the work-group stores them
//    with consecutive lanes on consecutive addresses.
// ---------------------------------------------------------------------------

// Global-address-space access through a generic pointer (the pointers kept
// in LDS are generic; these make the loads and stores global ones).
__device__ __forceinline__ uint32_t gld32(const uint32_t *p) {
  return *(const __attribute__((address_space(1))) uint32_t *)p;
}
__device__ __forceinline__ void gst32(uint32_t *p, uint32_t v) {
  *(__attribute__((address_space(1))) uint32_t *)p = v;
}

__device__ __forceinline__ int lds_pad(int e) { return e + (e >> 6); }

// What the merge pass reads of the context.
struct MapView {
  const uint32_t *part_job;
  const int64_t *part_ia;
  const uint64_t *mj_off;
  const int32_t *mj_lo, *mj_hi;
  const uint32_t *const *mj_src;
  uint32_t *const *mj_dst;
};

__device__ __forceinline__ MapView map_view(const DevCtx &C) {
  return MapView{C.part_job, C.part_ia, C.mj_off, C.mj_lo, C.mj_hi, C.mj_src, C.mj_dst};
}

template <int TILE>
struct MapLds {
  // A tile meets at most two partial jobs (its first and last portion); the
  // ones between are whole merge jobs, which exceed kLeaf keys.
  static constexpr int kPort = TILE / (kLeaf + 1) + 3;
  static constexpr int kBlk = TILE / 64;
  // input runs, portion by portion, then the merged outputs; key e sits at
  // lds_pad(e): one spare word after every 64 keys keeps lanes K keys apart
  // on different banks, and a wavefront's 64 consecutive keys contiguous
  uint32_t in[TILE + TILE / 64];
  const uint32_t *pa[kPort];   // first key a portion takes from its job's first half
  const uint32_t *pb[kPort];   // first key it takes from the second half
  uint32_t *po[kPort];         // destination of its first output
  int32_t pbase[kPort + 1];    // tile-relative first output of each portion; pbase[P] = tile length
  int32_t pna[kPort];          // keys it takes from the first half
  uint16_t first[kBlk];        // portion that holds tile output 64 b
  int32_t P;
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

// Portion holding tile output e (the block table gives the portion of the
// block's first output; at most two portions start inside a block).
template <int TILE>
__device__ __forceinline__ int portion_of(const MapLds<TILE> &M, int e) {
  int p = M.first[e >> 6];
  while (M.pbase[p + 1] <= e) ++p;
  return p;
}

// Number of usable jobs and the unit count they cover.
template <int TILE>
__device__ __forceinline__ void map_extent(const DevCtx &C, uint32_t Jraw, uint32_t *J, uint64_t *U) {
  *J = min(Jraw, (uint32_t)C.mj_cap);
  *U = *J ? C.mj_off[*J - 1] + (uint64_t)(C.mj_hi[*J - 1] - C.mj_lo[*J - 1]) : 0;
  const uint64_t maxU = (uint64_t)(C.part_cap - 1) * TILE;
  if (*U > maxU) *U = maxU;   // (never for the sizes the arena admits)
}

// Pass 1: the split at every tile boundary.  `wid` / `nwaves` enumerate the
// wavefronts taking part.
template <int TILE>
__device__ __forceinline__ void map_partition(const DevCtx &C, uint32_t J, uint64_t U, int64_t wid, int64_t nwaves) {
  const uint64_t nb = (U + TILE - 1) / TILE + 1;   // boundaries 0 .. ntiles
  const int lane = lane_id();
  // each wavefront takes a contiguous run of boundaries
  const uint64_t per = (nb + (uint64_t)nwaves - 1) / (uint64_t)nwaves;
  const uint64_t tb = (uint64_t)wid * per, te = min(tb + per, nb);
  for (uint64_t t = tb; t < te; ++t) {
    const uint64_t u = min(t * TILE, U);
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

// Merge-path split inside LDS for one lane: the number of the first o
// outputs of the merge of A = in[base, base + na) and B = in[base + na,
// base + na + nb) that come from A (equal keys from A first).
__device__ __forceinline__ int merge_split_lds(const uint32_t *in, int base, int na, int nb, int o) {
  int lo = o > nb ? o - nb : 0, hi = o < na ? o : na;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (in[lds_pad(base + mid)] <= in[lds_pad(base + na + o - mid - 1)]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One output of a lane's serial merge: portion p of the tile, ia / ib keys
// of its halves taken so far, av / bv the next key of each half.  Moves on to
// the next portion where one ends.
template <int TILE>
__device__ __forceinline__ uint32_t merge_step(const MapLds<TILE> &M, int &p, int &base, int &len, int &na,
                                               int &nb, int &ia, int &ib, uint32_t &av, uint32_t &bv) {
  while (ia + ib == len) {   // this portion is done: the next one starts here
    ++p;
    base = M.pbase[p];
    len = M.pbase[p + 1] - base;
    na = M.pna[p];
    nb = len - na;
    ia = ib = 0;
    av = na > 0 ? M.in[lds_pad(base)] : 0u;
    bv = nb > 0 ? M.in[lds_pad(base + na)] : 0u;
  }
  if (ib >= nb || (ia < na && av <= bv)) {
    const uint32_t x = av;
    ++ia;
    av = ia < na ? M.in[lds_pad(base + ia)] : 0u;
    return x;
  }
  const uint32_t x = bv;
  ++ib;
  bv = ib < nb ? M.in[lds_pad(base + na + ib)] : 0u;
  return x;
}

// ---- Pass 2 pieces ----------------------------------------------------------

// A tile's ends: the job and the first-half split at its first unit and at
// the unit after its last.
struct TileEnds {
  uint32_t j0, j1;
  int64_t ia0, ia1;
};

__device__ __forceinline__ TileEnds tile_ends(const MapView &C, uint64_t tile) {
  return TileEnds{C.part_job[tile], C.part_job[tile + 1], C.part_ia[tile], C.part_ia[tile + 1]};
}

// One merge job as the job table holds it.
struct JobRegs {
  uint64_t off;
  int32_t lo, hi;
  const uint32_t *src;
  uint32_t *dst;
};

__device__ __forceinline__ JobRegs load_job(const MapView &C, uint32_t j) {
  return JobRegs{C.mj_off[j], C.mj_lo[j], C.mj_hi[j], C.mj_src[j], C.mj_dst[j]};
}

// Jobs a tile meets (j0 .. j1; j1 may start exactly at the tile's end).
template <int TILE>
__device__ __forceinline__ int tile_jobs(const TileEnds &te) {
  return min((int)(te.j1 - te.j0) + 1, MapLds<TILE>::kPort);
}

// Portion k of the tile [u0, u1): the part of job j0 + k it covers.  The
// thread of the last job sets P and the end mark.
template <int TILE>
__device__ __forceinline__ void put_portion(MapLds<TILE> &M, int k, int n, const TileEnds &te, const JobRegs &jr,
                                            uint64_t u0, uint64_t u1) {
  const uint32_t j = te.j0 + k;
  const int64_t lo = jr.lo, hi = jr.hi;
  const int64_t mid = lo + (hi - lo) / 2;
  const uint64_t ts0 = max(u0, jr.off);
  const uint64_t te0 = min(u1, jr.off + (uint64_t)(hi - lo));
  const int64_t qs = (int64_t)(ts0 - jr.off);
  const int64_t as = (j == te.j0) ? te.ia0 : 0;
  const int64_t ae = (j == te.j1 && te0 == u1) ? te.ia1 : (mid - lo);
  M.pbase[k] = (int32_t)(ts0 - u0);
  M.pna[k] = (int32_t)(ae - as);
  M.pa[k] = jr.src + lo + as;
  M.pb[k] = jr.src + mid + (qs - as);
  M.po[k] = jr.dst + lo + qs;
  if (k == n - 1) {
    // the job starting exactly at the tile's end contributes nothing
    const int P = (ts0 < te0) ? n : n - 1;
    M.P = P;
    M.pbase[P] = (int32_t)(u1 - u0);
  }
}

// The portion of each 64-output block's first output (after put_portion and
// a barrier).
template <int WG, int TILE>
__device__ __forceinline__ void build_table(MapLds<TILE> &M, int tl) {
  const int P = M.P;
  for (int b = threadIdx.x; b < (tl + 63) / 64; b += WG) {
    const int e = b * 64;
    int lo = 0, hi = P;   // last portion whose base is <= e
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (M.pbase[mid] <= e) lo = mid; else hi = mid; }
    M.first[b] = (uint16_t)lo;
  }
}

// The lane's input keys (tile positions k * WG + lane), portion by portion:
// first-half keys then second-half keys; all loads in flight together.
template <int WG, int TILE>
__device__ __forceinline__ void stage_load(const MapLds<TILE> &M, int tl, uint32_t (&v)[TILE / WG]) {
#pragma unroll
  for (int k = 0; k < TILE / WG; ++k) {
    const int e = k * WG + threadIdx.x;
    v[k] = 0;
    if (e < tl) {
      const int p = portion_of(M, e);
      const int r = e - M.pbase[p];
      const int na = M.pna[p];
      v[k] = gld32(r < na ? M.pa[p] + r : M.pb[p] + (r - na));
    }
  }
}

template <int WG, int TILE>
__device__ __forceinline__ void stage_put(MapLds<TILE> &M, int tl, const uint32_t (&v)[TILE / WG]) {
#pragma unroll
  for (int k = 0; k < TILE / WG; ++k) {
    const int e = k * WG + threadIdx.x;
    if (e < tl) M.in[lds_pad(e)] = v[k];
  }
}

// Loads the tile's input keys straight into LDS, portion by portion: first-
// half keys then second-half keys.  Key e = k * WG + lane goes to lds_pad(e);
// a wavefront's 64 keys land contiguously from its first key's slot, as the
// direct-to-LDS load writes them.  The loads complete at the next wait for
// vector memory (wait_vmem), which must precede the barrier before their use.
template <int WG, int TILE>
__device__ __forceinline__ void stage_dma(MapLds<TILE> &M, int tl) {
  static_assert(WG % 64 == 0, "whole wavefronts");
  constexpr int K = TILE / WG;
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = k * WG + tid;
    if (e < tl) {
      const int p = portion_of(M, e);
      const int r = e - M.pbase[p];
      const int na = M.pna[p];
      const uint32_t *g = r < na ? M.pa[p] + r : M.pb[p] + (r - na);
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)g,
                                       (__attribute__((address_space(3))) void *)&M.in[lds_pad(e & ~63)],
                                       4, 0, 0);
    }
  }
}

// Stores a merged tile from LDS, consecutive lanes on consecutive addresses.
template <int WG, int TILE>
__device__ __forceinline__ void store_out(const MapLds<TILE> &M, int tl) {
  constexpr int K = TILE / WG;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = k * WG + threadIdx.x;
    if (e < tl) {
      const int q = portion_of(M, e);
      gst32(M.po[q] + (e - M.pbase[q]), M.in[lds_pad(e)]);
    }
  }
}

// Merges a staged tile (after a barrier) and stores it.  FAST: the lane's K
// outputs from one batch of LDS reads and a sorting network, back to LDS, and
// out with consecutive lanes on consecutive addresses (more registers);
// otherwise one key at a time, each stored as it is found.  Ends with a
// barrier.
template <int WG, int TILE, bool FAST>
__device__ __forceinline__ void merge_out(MapLds<TILE> &M, int tl) {
  constexpr int K = TILE / WG;   // outputs per lane
  static_assert(K * WG == TILE && K >= 1 && K <= 64 && (K & (K - 1)) == 0,
                "a power-of-two number of outputs per lane");
  constexpr int kLogK = K >= 32 ? 5 : K >= 16 ? 4 : K >= 8 ? 3 : K >= 4 ? 2 : K >= 2 ? 1 : 0;
  const int tid = threadIdx.x;
  const int e0 = tid * K;
  const bool live = e0 < tl;
  int p = 0, base = 0, len = 0, na = 0, nb = 0, ia = 0, ib = 0;
  if (live) {
    p = portion_of(M, e0);
    base = M.pbase[p];
    len = M.pbase[p + 1] - base;
    na = M.pna[p];
    nb = len - na;
    ia = merge_split_lds(M.in, base, na, nb, e0 - base);
    ib = e0 - base - ia;
  }
  if constexpr (FAST) {
    uint32_t out[K];
    if (live && min(e0 + K, tl) <= base + len) {
      // The lane's outputs are the K smallest keys of A[ia, ia + K) and
      // B[ib, ib + K) (keys past a half's end count as the largest key; only
      // key values are moved, so which of two equal keys goes first cannot
      // be seen).  The smaller key of each pair (A[ia + i], B[ib + K-1-i])
      // forms a bitonic sequence holding exactly those K keys; a bitonic
      // sorting network puts them in order.
      uint32_t a[K], b[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        a[i] = ia + i < na ? M.in[lds_pad(base + ia + i)] : 0xFFFFFFFFu;
        b[i] = ib + i < nb ? M.in[lds_pad(base + na + ib + i)] : 0xFFFFFFFFu;
      }
#pragma unroll
      for (int i = 0; i < K; ++i) out[i] = min(a[i], b[K - 1 - i]);
#pragma unroll
      for (int s = kLogK - 1; s >= 0; --s) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          if ((i & (1 << s)) == 0) {
            const uint32_t x = out[i], y = out[i + (1 << s)];
            out[i] = min(x, y);
            out[i + (1 << s)] = max(x, y);
          }
        }
      }
    } else {
      // outputs that run into the next portion (or none): one key at a time
      uint32_t av = 0, bv = 0;
      if (live) {
        av = ia < na ? M.in[lds_pad(base + ia)] : 0u;
        bv = ib < nb ? M.in[lds_pad(base + na + ib)] : 0u;
      }
#pragma unroll
      for (int t = 0; t < K; ++t) {
        out[t] = 0;
        if (e0 + t < tl) out[t] = merge_step(M, p, base, len, na, nb, ia, ib, av, bv);
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < K; ++t)
      if (e0 + t < tl) M.in[lds_pad(e0 + t)] = out[t];
    __syncthreads();
    store_out<WG>(M, tl);
  } else {
    uint32_t av = 0, bv = 0;
    if (live) {
      av = ia < na ? M.in[lds_pad(base + ia)] : 0u;
      bv = ib < nb ? M.in[lds_pad(base + na + ib)] : 0u;
    }
    for (int t = 0; t < K && e0 + t < tl; ++t) {
      const uint32_t x = merge_step(M, p, base, len, na, nb, ia, ib, av, bv);
      gst32(M.po[p] + (ia + ib - 1), x);
    }
  }
  __syncthreads();
}

// Pass 2: tiles go to work-groups blockIdx.x, blockIdx.x + gridDim.x, ...;
// every thread of the work-group takes part.  FAST as in merge_out, with all
// of a lane's input loads in registers in flight together; otherwise the
// inputs go straight to LDS (no registers held).  (The direct-to-LDS loads
// measured slower than register loads for the standalone pass, and a
// software pipeline over several tiles per work-group slower than one tile
// per work-group with many work-groups in flight.)
template <int WG, int TILE, bool FAST>
__device__ __forceinline__ void map_merge(const MapView &C, MapLds<TILE> &M, uint32_t /*jobs*/, uint64_t U) {
  const uint64_t ntiles = (U + TILE - 1) / TILE;
  const int tid = threadIdx.x;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t u0 = tile * TILE;
    const uint64_t u1 = min(u0 + (uint64_t)TILE, U);
    const int tl = (int)(u1 - u0);
    const TileEnds te = tile_ends(C, tile);
    const int n = tile_jobs<TILE>(te);
    for (int k = tid; k < n; k += WG) put_portion(M, k, n, te, load_job(C, te.j0 + k), u0, u1);
    __syncthreads();
    build_table<WG>(M, tl);
    __syncthreads();
    if constexpr (FAST) {
      uint32_t v[TILE / WG];
      stage_load<WG>(M, tl, v);
      stage_put<WG>(M, tl, v);
    } else {
      stage_dma<WG>(M, tl);
      wait_vmem();
    }
    __syncthreads();
    merge_out<WG, TILE, FAST>(M, tl);
  }
}

}  // namespace trees
