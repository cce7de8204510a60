// TREES epoch kernels for CDNA4 (gfx950).
//
// One launch of the sweep executes Phase 2 of an epoch (Section 5.2.3) for
// every work item: a work item is one task-vector entry of one tree's
// current range.  Each lane reads its entry, decodes epoch number and task
// type (Section 5.1.2 and its footnote: code = epoch * NTT + type, runnable
// iff CEN*NTT + 1 <= code <= (CEN+1)*NTT), runs the body of its type and
// performs fork / join / emit (Section 4.3.2):
//
//  * fork: children of a work-group are allocated together -- a wavefront
//    prefix sum by ballot + mbcnt, wavefront totals combined in LDS, and ONE
//    device-scope atomic add on the tree's nextFreeCore per work-group and
//    tree (the paper takes one atomic per wavefront through a local-memory
//    reduction, Section 5.2.3); children of one parent are contiguous, and
//    children are written with structure-of-arrays stores;
//  * join: the lane rewrites its own entry with the continuation at the same
//    epoch number and counts one join for its tree;
//  * emit: the lane stores its value in r[i] and marks the entry invalid.
//
// Phase 3 and Phase 1 (Sections 5.2.2 and 5.2.4) run on the device in the
// batched forms: the work-group that retires the last work item of a tree in
// an epoch pushes that tree's join and fork ranges, pops its next range and
// resets its counters; the last work-group to reach the epoch barrier turns
// the per-tree ranges into the next epoch's work list with one exclusive
// scan.  The plain form leaves Phases 1 and 3 to the host, one launch per
// epoch, as the paper does.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "bodies.h"
#include "map.h"
#include "prims.h"
#include "trees.h"
#include "trees_dev.h"

namespace trees {

enum : int { ACT_NONE = 0, ACT_EMIT = 1, ACT_JOIN = 2, ACT_FINISH = 3 };

// A chunk is the unit of work of one work-group: kChunk consecutive work
// items, IT = kChunk / WG per lane (item x of the chunk is handled by lane
// x % WG as its item x / WG, so each of a lane's items is a coalesced
// work-group-wide access).  All per-tree state a chunk needs is cached in LDS
// per segment (a run of the chunk's items that belong to one tree).
constexpr int kChunk = kChunkItems;

template <int WG, int NS = kChunk>   // NS: segments a chunk can touch (1 in the plain form)
struct Lds {
  int32_t kfirst;          // first work-list entry of the chunk
  int32_t nseg;            // entries (trees) the chunk touches
  uint32_t off0;           // wl_off[kfirst]
  int32_t flag;            // scratch broadcast
  int32_t flag2;
  uint32_t gen;
  int32_t sink;            // destination of atomics whose completion must be awaited
  int32_t tflag;
  int32_t sflag, scnt;     // work-list scan: broadcast and counter (adoption)
  uint32_t hdr[6];         // header of the next epoch (S, L, stop, mapJ, initN, wsel), for a solo epoch
  uint32_t jbase;          // first map job reserved by this work-group
  uint64_t ubase;          // first map unit reserved by this work-group
  int64_t tprof;           // debug: clock at the last phase boundary
  int64_t prof[8];         // debug: time per phase
  uint8_t op_tab[kMaxTypes + 1];   // global type id -> operation
  uint32_t win[NS];        // wl_off[kfirst + 1 + t]
  int32_t seg_slot[NS];   // tree slot of segment s
  int32_t seg_cen[NS];    // its epoch number
  int32_t seg_b[NS];      // arena-relative start of its range
  uint32_t seg_tb[NS];    // its arena base / 64
  uint32_t seg_tp[NS];    // first type id | parameter << 8
  int32_t seg_cnt[NS];    // children requested per segment (LDS atomics)
  int32_t seg_base[NS];   // arena-relative first child per segment (-1: overflow)
  int32_t seg_jv[NS];     // joins (low 16 bits) | valid tasks (high 16 bits) per segment
  int32_t scan_tmp[WG / 64 + 1];
  int64_t scan_tmp64[WG / 64 + 1];
};

// VISIT expansion state (only in kernels that run BFS).
constexpr int kClaimQ = 2048;
constexpr int kArcsPerLane = 4;   // arcs a lane probes per step of the expansion (at most)
// Arcs per lane per step for a work-group of WG lanes: one step claims at
// most WG * A vertices, and a flush leaves room for one more step.
template <int WG>
constexpr int arcs_per_lane() {
  return (kClaimQ / 2) / WG >= kArcsPerLane ? kArcsPerLane : ((kClaimQ / 2) / WG > 0 ? (kClaimQ / 2) / WG : 1);
}
struct VisitLds {
  int32_t row[kChunk];     // first arc of the item's vertex
  int32_t pre[kChunk];     // exclusive prefix of out-degrees, in (lane, item) order
  int32_t seg[kChunk];
  int32_t dv[kChunk];      // SSSP item: its vertex's distance when fetched; BFS item: -1
  int32_t qu[kClaimQ];     // claimed vertices waiting for their child entries
  int32_t qd[kClaimQ];     // SSSP claim: the distance it set (the child's a1); BFS: -1
  int16_t qs[kClaimQ];     // their segment (< kChunk)
  int16_t qo[kClaimQ];     // their offset inside the segment's block (< kClaimQ)
  int32_t qn;
};
struct NoVisitLds {};

// Debug phase clock: thread 0 charges the time since the last boundary to
// phase ph (only with TREES_F_DEBUG; the branch is uniform).
template <int WG, int NS>
__device__ __forceinline__ void phase_mark(const DevCtx &C, Lds<WG, NS> &L, int ph) {
  if (C.debug && threadIdx.x == 0) {
    const int64_t t = realtime();
    L.prof[ph] += t - L.tprof;
    L.tprof = t;
  }
}

// ---------------------------------------------------------------------------
// Segment helpers
// ---------------------------------------------------------------------------

// Adds two 0/1 flags per lane to a segment's packed counter: `lo` to the
// low 16 bits and `hi` to the high 16 bits (a segment retires at most
// kChunk items per chunk, so neither half carries).
__device__ __forceinline__ void seg_add_pair(int32_t *arr, int seg, bool lo, bool hi) {
  const uint64_t mlo = ballot64(lo), mhi = ballot64(hi);
  const uint64_t m = mlo | mhi;
  if (!m) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  const int s0 = __shfl(seg, leader, 64);
  if (__all(!(lo || hi) || seg == s0)) {
    if (lane_id() == leader) atomicAdd(&arr[s0], __popcll(mlo) + (__popcll(mhi) << 16));
  } else if (lo || hi) {
    atomicAdd(&arr[seg], (lo ? 1 : 0) + (hi ? 0x10000 : 0));
  }
}

// First half of the co-operative fork allocation (Tenet 2): the lane asks
// for nk (< 16) children of the tree of segment `seg` and gets its offset
// inside the work-group's block for that tree.  A wavefront whose requests
// all go to one tree takes its exclusive prefix from one ballot per bit and
// adds its total with a single LDS atomic.  All 64 lanes must call it.
__device__ __forceinline__ int lds_reserve(int32_t *seg_cnt, int seg, int nk) {
  int off = 0;
  const uint64_t m = ballot64(nk > 0);
  if (m) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int s0 = __shfl(seg, leader, 64);
    if (__all(nk == 0 || seg == s0)) {
      int tot;
      const int pre = wave_prefix_small<4>(nk, &tot);
      int wb = 0;
      if (lane_id() == leader) wb = atomicAdd(&seg_cnt[s0], tot);
      wb = __shfl(wb, leader, 64);
      off = wb + pre;
    } else if (nk > 0) {
      off = atomicAdd(&seg_cnt[seg], nk);
    }
  }
  return off;
}

// Second half: one device-scope atomic add on the tree's nextFreeCore per
// segment of the chunk (the plain form adds forks and joins of its single
// tree with one 64-bit atomic).  Every thread of the work-group calls it;
// afterwards L.seg_base[s] holds the arena-relative first child of segment s
// or -1 if the tree's arena overflowed.
template <int WG, bool MULTI, int NS>
__device__ __forceinline__ void seg_commit(const DevCtx &C, Lds<WG, NS> &L, const PlainArgs &P,
                                           bool with_joins) {
  __syncthreads();
  const int nseg = L.nseg;
  for (int s = threadIdx.x; s < nseg; s += WG) {
    const int c = L.seg_cnt[s];
    int b = 0;
    if (MULTI) {
      if (c > 0) {
        L.seg_cnt[s] = 0;
        const int slot = L.seg_slot[s];
        b = add_agent(&C.hot[slot].nfc, (int32_t)c);
        // (b < 0: the counter wrapped after an overflow earlier in the epoch,
        // possible only for programs whose task count has no exact bound)
        if (b < 0 || (int64_t)b + c > (int64_t)C.ts[slot].cap) {
          L.sink = or_agent(&C.hot[slot].flags, (int32_t)TF_OVERFLOW);
          b = -1;
        }
      }
    } else {
      const int j = with_joins ? (L.seg_jv[s] & 0xFFFF) : 0;
      if (with_joins) L.seg_jv[s] &= ~0xFFFF;
      if (c > 0 || j > 0) {
        L.seg_cnt[s] = 0;
        const uint64_t prev = add_agent(&C.plain->fj[P.par], ((uint64_t)(uint32_t)j << 32) | (uint32_t)c);
        b = (int32_t)(uint32_t)prev;
        if (b < 0 || (int64_t)P.nfc0 + b + c > (int64_t)C.ts[P.slot].cap) {
          L.sink = or_agent(&C.plain->flags[P.par], (int32_t)TF_OVERFLOW);
          b = -1;
        } else {
          b += P.nfc0;
        }
      }
    }
    L.seg_base[s] = b;
  }
  __syncthreads();
}

__device__ __forceinline__ int32_t child_base(const int32_t *seg_base, int seg, int nk, int off) {
  if (nk == 0) return 0;
  const int b = seg_base[seg];
  return b < 0 ? -1 : b + off;
}

// ---------------------------------------------------------------------------
// Phase 3 + Phase 1 of one tree (device form).  Run by one lane of the
// wavefront or work-group that retired the tree's last work item of the
// epoch.  Returns the tree's next range (len 0: the tree is complete), which
// the caller appends to the next epoch's work list.
// ---------------------------------------------------------------------------
struct NextRange {
  int32_t len = 0, cen = 0, b = 0;
  uint32_t tb = 0, tp = 0;
  int32_t nxt = 0;   // the work-list buffer the range goes to
};

__device__ NextRange tree_phase3(const DevCtx &C, int slot, uint32_t joins) {
  NextRange out;
  TreeState *T = &C.st[slot];
  TreeHot *H = &C.hot[slot];
  const int32_t nfc = ld_agent(&H->nfc);
  const int32_t flags = ld_agent(&H->flags);
  const int32_t cen = T->cen, b = T->b, e = T->e, old = T->old;
  int32_t sp = T->sp;
  const int32_t forks = nfc - old;
  const int32_t valid = ld_agent(&H->valid);   // tasks executed this epoch (its share of the work)
  const int32_t ep = T->epochs;
  out.nxt = ld_agent(&C.hdr->wsel) ^ 1;
  out.tb = (uint32_t)(C.ts[slot].base >> 6);
  out.tp = C.ts[slot].tp;
  T->epochs = ep + 1;
  T->launched += e - b;
  T->tasks += valid;
  if (nfc > T->peak) T->peak = nfc;
  if (C.trace_on && ep < kTraceMax) {
    TraceRec q;
    q.epoch = ep; q.cen = cen; q.b = b; q.e = e; q.launched = e - b;
    q.valid = valid; q.forks = forks; q.joins = (int32_t)joins; q.nfc = nfc;
    C.trace[(size_t)slot * kTraceMax + ep] = q;
    T->ntrace = ep + 1;
  }
  int4 *stk = C.stack + (size_t)slot * kStackMax;
  int err = 0;
  if (flags & TF_OVERFLOW) err = -3;        // TREES_E_OVERFLOW
  else if (flags & TF_ENCODING) err = -8;   // TREES_E_ENCODING
  int4 top;
  bool have = false;
  if (!err) {
    // Phase 3: the join range first, then the forked range on top (LIFO).
    if (joins) {
      if (sp >= kStackMax) err = -9;        // TREES_E_STACK
      else stk[sp++] = make_int4(cen, b, e, nfc);
    }
    if (!err) {
      if (forks) { top = make_int4(cen + 1, old, nfc, nfc); have = true; }
      else if (sp > 0) { top = stk[--sp]; have = true; }
    }
  }
  if (err || !have) {  // empty stack: the tree is complete (Section 4.3.3)
    T->status = TS_DONE;
    T->err = err;
    T->sp = sp;
    C.t_len[slot] = 0;
    int j = add_agent(&C.hdr->done_count, 1);
    C.done_list[j] = slot;
    return out;
  }
  // Phase 1 of the tree's next epoch: nextFreeCore returns to the value it
  // had when the popped range was pushed.
  T->cen = top.x; T->b = top.y; T->e = top.z; T->old = top.w; T->sp = sp;
  st_agent(&H->nfc, top.w);
  st_agent(&H->done, (uint64_t)0);
  st_agent(&H->valid, 0);
  C.t_len[slot] = top.z - top.y;
  C.t_cen[slot] = top.x;
  C.t_b[slot] = top.y;
  out.len = top.z - top.y;
  out.cen = top.x;
  out.b = top.y;
  return out;
}

// Entry k of work-list buffer n.nxt: the range n of tree `slot`, its items
// starting at `off`.
__device__ __forceinline__ void wl_put(const DevCtx &C, const NextRange &n, int slot, int k, uint32_t off) {
  const size_t i = (size_t)n.nxt * (size_t)(C.tmax + 1) + (size_t)k;
  C.wl_tree[i] = slot;
  C.wl_off[i] = off;
  C.wl_b[i] = n.b;
  C.wl_cen[i] = n.cen;
  C.wl_tb[i] = n.tb;
  C.wl_tp[i] = n.tp;
}

// Phase 3 of one tree from one lane, its next range appended on its own.
__device__ void tree_finish(const DevCtx &C, int slot, uint32_t joins) {
  const NextRange n = tree_phase3(C, slot, joins);
  if (n.len > 0) {
    const uint64_t prev = add_agent(&C.hdr->wl_next, ((uint64_t)1 << kWlShift) | (uint64_t)n.len);
    wl_put(C, n, slot, (int)(prev >> kWlShift), (uint32_t)(prev & kWlItemMask));
  }
}

// ---------------------------------------------------------------------------
// The body of one task by its operation (Section 4.3.2): what it forks (nk
// children, whose arguments follow from x0..x3), whether it joins or emits
// (val), and the co-operative work it hands on (a merge for the map phase, a
// leaf sort, an FFT leaf).  errf: the tree's error flags (an invalid node
// raises TF_ENCODING there); sink receives atomics' results.
// ---------------------------------------------------------------------------
template <uint32_t OPS>
__device__ __forceinline__ void task_body(const DevCtx &C, int op, int32_t a0v, int32_t a1v, int32_t a2v, int32_t a3v,
                                          int64_t tb, uint32_t tp, int slot, int32_t *errf, int32_t &sink, int &nk,
                                          int &act, int64_t &val, int32_t &x0, int32_t &x1, int32_t &x2, int32_t &x3,
                                          bool &want_map, bool &leaf, bool &fleaf) {
  nk = 0; act = ACT_NONE; val = 0;
  x0 = x1 = x2 = x3 = 0;
  want_map = false; leaf = false; fleaf = false;
  if (op == OP_NONE) return;
  switch (op) {
    case OP_FIB32:
    case OP_FIB64: {
      const int32_t n = a0v;
      if (n < 2) { act = ACT_EMIT; val = n; }
      else { act = ACT_JOIN; nk = 2; x0 = n; }
    } break;
    case OP_SUM32: {
    if constexpr ((OPS & opbit(OP_SUM32)) == 0) break;
      const int32_t c = a0v;
      const uint32_t sm = (uint32_t)C.r[tb + c] + (uint32_t)C.r[tb + c + 1];
      act = ACT_EMIT; val = (int64_t)(int32_t)sm;
    } break;
    case OP_SUM64: {
    if constexpr ((OPS & opbit(OP_SUM64)) == 0) break;
      const int32_t c = a0v;
      act = ACT_EMIT; val = C.r[tb + c] + C.r[tb + c + 1];
    } break;
    case OP_Q: {
    if constexpr ((OPS & opbit(OP_Q)) == 0) break;
      const int32_t n = (int32_t)(tp >> 8);
      const int32_t row = a0v;
      if (row == n) { act = ACT_EMIT; val = 1; break; }
      const uint32_t full = (1u << n) - 1u;
      const uint32_t cols = (uint32_t)a1v, ld = (uint32_t)a2v, rd = (uint32_t)a3v;
      const uint32_t avail = ~(cols | ld | rd) & full;
      if (!avail) { act = ACT_EMIT; val = 0; break; }
      act = ACT_JOIN; nk = __popc(avail);
      x0 = row; x1 = (int32_t)cols; x2 = (int32_t)ld; x3 = (int32_t)rd;
    } break;
    case OP_QSUM: {
    if constexpr ((OPS & opbit(OP_QSUM)) == 0) break;
      // the children's counts (kk <= 14), all loads issued before the sum
      const int32_t c = a0v, kk = a1v;
      const int64_t *rr = C.r + tb + c;
      int64_t part[14];
#pragma unroll
      for (int j = 0; j < 14; ++j) part[j] = j < kk ? rr[j] : 0;
      int64_t sm = 0;
#pragma unroll
      for (int j = 0; j < 14; ++j) sm += part[j];
      act = ACT_EMIT; val = sm;
    } break;
    case OP_MS: {
    if constexpr ((OPS & opbit(OP_MS)) == 0) break;
      const int32_t lo = a0v, hi = a1v, d = a2v;
      x0 = lo; x1 = hi; x2 = d;
      if (hi - lo <= kLeaf) { act = ACT_FINISH; leaf = true; }   // sorted co-operatively below
      else { act = ACT_JOIN; nk = 2; }
    } break;
    case OP_MERGE: {
    if constexpr ((OPS & opbit(OP_MERGE)) == 0) break;
      act = ACT_FINISH;
      x0 = a0v; x1 = a1v; x2 = a2v;
      if (C.mj_cap > 0) {
        want_map = true;   // the merge runs in the map phase
      } else {
        const TreeStatic *T = &C.ts[slot];
        ms_merge((uint32_t *)T->ptr0, (uint32_t *)T->ptr1, x0, x1, x2);
      }
    } break;
    case OP_VISIT:
    case OP_SVISIT:
      act = ACT_FINISH;   // its arcs are expanded co-operatively below
      break;
    case OP_POST: {
    if constexpr ((OPS & opbit(OP_POST)) == 0) break;
      // Figure 2: postorder(node) forks postorder(right), postorder(left)
      // and joins a visit of node; postorder(-1) ends.
      const int32_t node = a0v, n = (int32_t)(tp >> 8);
      act = ACT_FINISH;
      if (node < 0) break;
      if (node >= n) {   // not a node of this tree: an error of the tree
        sink = or_agent(errf, (int32_t)TF_ENCODING);
        break;
      }
      const TreeStatic *T = &C.ts[slot];
      act = ACT_JOIN; nk = 2;
      x0 = node;
      x1 = ((const int32_t *)T->ptr1)[node];   // right child, forked first
      x2 = ((const int32_t *)T->ptr0)[node];   // left child
    } break;
    case OP_PVISIT:
      act = ACT_FINISH;   // the visit: appended to the tree's log below
      break;
    case OP_FFT: {
    if constexpr ((OPS & opbit(OP_FFT)) == 0) break;
      // FFT(lo, o, ls): n = 2^(log2 N - ls) points; a leaf is transformed
      // by a wavefront below; otherwise fork the even and odd halves and
      // join the combine (which keeps lo, o, ls)
      const int lg = (int)(tp >> 8) - a2v;
      if (lg <= kFftLeafLog) { act = ACT_FINISH; fleaf = true; }
      else { act = ACT_JOIN; nk = 2; x0 = a0v; x1 = a1v; x2 = a2v; }
    } break;
    case OP_COMB:
      act = ACT_FINISH;   // its butterflies are expanded co-operatively below
      break;
    case OP_PRE: {
    if constexpr ((OPS & opbit(OP_PRE)) == 0) break;
      // Figure 2: preorder(node) visits node (appended to the log below),
      // then forks preorder(right), preorder(left); preorder(-1) ends.
      const int32_t node = a0v, n = (int32_t)(tp >> 8);
      act = ACT_FINISH;
      if (node < 0) break;
      if (node >= n) {
        sink = or_agent(errf, (int32_t)TF_ENCODING);
        break;
      }
      const TreeStatic *T = &C.ts[slot];
      nk = 2;
      x1 = ((const int32_t *)T->ptr1)[node];
      x2 = ((const int32_t *)T->ptr0)[node];
    } break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// One chunk of kChunk work items.
// ---------------------------------------------------------------------------
// A tree's finish check whose atomic is still in flight: the work-group that
// retires a tree's last items of the epoch runs its Phase 3 (tree_finish).
// The check is made in the next chunk, once its allocation atomic has
// returned, or after the last chunk, so the atomic's latency overlaps the
// next chunk.
struct PendingFinish {
  int slot = -1;
  uint32_t items = 0, range = 0, joins = 0;
  uint64_t prev = 0;
};

__device__ __forceinline__ void settle(const DevCtx &C, PendingFinish &f) {
  if (f.slot >= 0) {
    if ((uint32_t)f.prev + f.items == f.range) tree_finish(C, f.slot, (uint32_t)(f.prev >> 32) + f.joins);
    f.slot = -1;
  }
}

// ---------------------------------------------------------------------------
// Arc phase (batched forms): publication by the owner chunk, and tiles.
// ---------------------------------------------------------------------------

// Last index i in [0, kChunk) with pre[i] <= e (pre is non-decreasing, pre[0] = 0).
__device__ __forceinline__ int last_le(const int32_t *pre, int e) {
  int lo = 0, hi = kChunk;
  while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (pre[mid] <= e) lo = mid; else hi = mid; }
  return lo;
}

// Turns the claim queue (V.qn vertices with their segment and, for SSSP,
// the distance that forked them) into entries of the next epoch: offsets from
// the LDS segment counters, one device atomic per segment (seg_commit), then
// code, a0 and, for an SSSP entry, a1.  Every thread of the work-group calls
// it after a barrier that follows the last push; it empties the queue.
template <int WG, bool MULTI, bool SSSP, int NS>
__device__ void flush_claims(const DevCtx &C, Lds<WG, NS> &L, VisitLds &V, const PlainArgs &P) {
  const int tid = threadIdx.x;
  const int qn = V.qn;
  for (int q0 = 0; q0 < qn; q0 += WG) {
    const int q = q0 + tid;
    const int o = lds_reserve(L.seg_cnt, q < qn ? V.qs[q] : -1, q < qn ? 1 : 0);
    if (q < qn) V.qo[q] = (int16_t)o;
  }
  seg_commit<WG, MULTI>(C, L, P, false);
  for (int q = tid; q < qn; q += WG) {
    const int ss = V.qs[q];
    const int32_t vb = L.seg_base[ss];
    if (vb >= 0) {
      const int64_t c = ((int64_t)L.seg_tb[ss] << 6) + vb + V.qo[q];
      C.code[c] = (L.seg_cen[ss] + 1) * C.ntt + (int32_t)(L.seg_tp[ss] & 0xFF);
      C.a0[c] = V.qu[q];
      if (SSSP && V.qd[q] >= 0) C.a1[c] = V.qd[q];
    }
  }
  __syncthreads();
  if (tid == 0) V.qn = 0;
  __syncthreads();
}

// Publishes the chunk's VISIT arcs (V: lane-major degree prefix, first arcs,
// segments; tot arcs in all) as a job of tiles.  Returns the job number, or
// -1 when the epoch's job table is full (the chunk then expands locally).
// Plain stores: the arc phase reads them after a grid barrier or a kernel
// boundary.
template <int WG>
__device__ int publish_arcs(const DevCtx &C, Lds<WG> &L, VisitLds &V, int tot, int max_tiles) {
  SchedHdr *H = C.hdr;
  const int tid = threadIdx.x;
  const int tile = max(kArcTile, (tot + max_tiles - 1) / max_tiles);
  const int ntiles = (tot + tile - 1) / tile;
  const int nseg = L.nseg;
  if (tid == 0) {
    // a job, its tiles and its segment records; any table full: no job
    // (the counters keep growing, and a later claim sees they are full)
    int j = (int)add_agent(&H->arc_jobs, 1u);
    uint32_t tb = 0, sb = 0;
    if (j < kArcJobs) {
      tb = add_agent(&H->arc_tiles, (uint32_t)ntiles);
      sb = add_agent(&H->arc_segs, (uint32_t)nseg);
      // reserved tiles of a job that cannot be kept are marked empty (-2)
      if (tb + (uint32_t)ntiles > (uint32_t)kArcTilesAll || sb + (uint32_t)nseg > (uint32_t)kArcSegPool) j = -2;
    } else {
      j = -1;
    }
    L.flag = j;
    L.flag2 = (int)tb;
    L.jbase = sb;
  }
  __syncthreads();
  const int j = L.flag;
  const uint32_t tbase = (uint32_t)L.flag2;
  const uint32_t sbase = L.jbase;
  __syncthreads();
  if (j == -2) {
    for (int t = tid; t < ntiles; t += WG)
      if (tbase + (uint32_t)t < (uint32_t)kArcTilesAll) C.arc_tile[tbase + t] = make_int4(-1, 0, 0, 0);
  }
  if (j < 0) return -1;
  int32_t *it = C.arc_item + (size_t)j * kArcItemWords;
  for (int i = tid; i < kChunk; i += WG) {
    it[i] = V.pre[i];
    it[kChunk + i] = V.row[i];
    it[2 * kChunk + i] = V.seg[i];
    it[3 * kChunk + i] = V.dv[i];
  }
  int32_t *sg = C.arc_seg + sbase;
  for (int q = tid; q < nseg; q += WG) {
    sg[q] = L.seg_slot[q];
    sg[kArcSegPool + q] = L.seg_cen[q];
    sg[2 * kArcSegPool + q] = (int32_t)L.seg_tb[q];
    sg[3 * kArcSegPool + q] = (int32_t)L.seg_tp[q];
  }
  for (int t = tid; t < ntiles; t += WG)
    C.arc_tile[tbase + t] = make_int4(j, last_le(V.pre, t * tile), last_le(V.pre, min((t + 1) * tile, tot) - 1), 0);
  if (tid == 0) {
    ArcJob *J = &C.arc_job[j];
    J->tot = tot; J->tile = tile; J->ntiles = ntiles; J->nseg = nseg; J->tbase = tbase; J->sbase = sbase;
    st_agent(&J->done, 0u);
  }
  return j;
}

// Task-vector entries of the next chunk of a work-group's run, loaded while
// the current chunk is processed (only when the next chunk lies inside the
// current chunk's last tree, so its indices need no locate).
template <int IT>
struct Prefetch {
  uint32_t w0 = 0xFFFFFFFFu;   // first item of the prefetched chunk (none: ~0)
  int32_t code[IT], a0[IT], a1[IT], a2[IT], a3[IT];
};

template <int WG, uint32_t OPS, bool MULTI, typename VL, int NS, int IT>
__device__ void run_chunk(const DevCtx &C, Lds<WG, NS> &L, VL &V, uint32_t w0, uint32_t S, int32_t nL,
                          const PlainArgs &P, PendingFinish &pend, Prefetch<IT> &pf, uint32_t run_end,
                          bool follows = false, uint32_t wo = 0) {
  static_assert(IT == kChunk / WG, "items per lane");
  static_assert(MULTI ? NS == kChunk : NS >= 1, "a batched chunk can touch kChunk trees");
  // the previous chunk already loaded this chunk's entries (same tree, same
  // window); kernels with merge sort or BFS do not prefetch (their register
  // budget is spent on leaf sorts and arc expansion)
  constexpr bool kPrefetch = MULTI && (OPS & (OPS_MS | OPS_EXPAND)) == 0;
  const bool hit = kPrefetch && follows && pf.w0 == w0;
  const int tid = threadIdx.x;
  const int lane = lane_id();

  // ---- locate the chunk's trees ---------------------------------------------
  // A chunk touches the work-list entries kfirst .. kfirst + nseg - 1.  The
  // first chunk of a work-group's run finds kfirst by a 64-ary search; a
  // following chunk starts in the last entry of the previous one or in the
  // entry after it.  One round trip then brings the next 64 entries' ends
  // and tree data; a chunk that spans more than 64 trees loads the rest.
  if (hit) {
    // one segment that extends past this chunk: the window stays as it is
  } else if (MULTI && nL > 1) {
    if (follows) {
      if (tid == 0) {
        const int ps = L.nseg - 1;
        const int adv = (L.win[ps] <= w0) ? ps + 1 : ps;
        if (adv) L.off0 = L.win[adv - 1];
        L.kfirst += adv;
      }
    } else if (tid < 64) {
      // 64-ary search for the last entry whose offset is <= w0
      int lo = 0, hi = nL;
      while (hi - lo > 1) {
        const int step = (hi - lo + 63) >> 6;
        const int p = lo + tid * step;
        const bool ok = p < hi && C.wl_off[wo + p] <= w0;
        const int j = __popcll(ballot64(ok)) - 1;
        lo = lo + j * step;
        hi = min(lo + step, hi);
      }
      if (tid == 0) { L.kfirst = lo; L.off0 = C.wl_off[wo + lo]; }
    }
    __syncthreads();
    const int kf = L.kfirst;
    const uint32_t wl = min(w0 + (uint32_t)kChunk, S) - 1;   // the chunk's last item
    if (tid < 64) {
      const int e = kf + tid;
      const uint32_t end = (e + 1 <= nL) ? C.wl_off[wo + e + 1] : 0xFFFFFFFFu;
      if (e < nL) {
        L.seg_slot[tid] = C.wl_tree[wo + e];
        L.seg_cen[tid] = C.wl_cen[wo + e];
        L.seg_b[tid] = C.wl_b[wo + e];
        L.seg_tb[tid] = C.wl_tb[wo + e];
        L.seg_tp[tid] = C.wl_tp[wo + e];
      }
      L.win[tid] = end;
      const int ended = __popcll(ballot64(end <= wl));   // entries that end inside the chunk
      if (tid == 0) L.nseg = ended + 1;
    }
    __syncthreads();
    if (L.nseg > 64) {   // more than 64 trees in this chunk
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        const int t = k * WG + tid;
        const int e = kf + t;
        if (t < 64) continue;
        L.win[t] = (e + 1 <= nL) ? C.wl_off[wo + e + 1] : 0xFFFFFFFFu;
        if (e < nL) {
          L.seg_slot[t] = C.wl_tree[wo + e];
          L.seg_cen[t] = C.wl_cen[wo + e];
          L.seg_b[t] = C.wl_b[wo + e];
          L.seg_tb[t] = C.wl_tb[wo + e];
          L.seg_tp[t] = C.wl_tp[wo + e];
        }
      }
      __syncthreads();
      if (tid == 0) {
        int lo2 = 64, hi2 = kChunk;
        while (lo2 < hi2) { const int mid = (lo2 + hi2) >> 1; if (L.win[mid] <= wl) lo2 = mid + 1; else hi2 = mid; }
        L.nseg = lo2 + 1;
      }
    }
  } else if (tid == 0) {
    L.kfirst = 0; L.nseg = 1; L.off0 = 0; L.win[0] = S;
    if (MULTI) {
      if (!follows) {   // one tree in the work list: its data stays for the whole run
        L.seg_slot[0] = C.wl_tree[wo + 0]; L.seg_cen[0] = C.wl_cen[wo + 0]; L.seg_b[0] = C.wl_b[wo + 0];
        L.seg_tb[0] = C.wl_tb[wo + 0]; L.seg_tp[0] = C.wl_tp[wo + 0];
      }
    } else {
      L.seg_slot[0] = P.slot; L.seg_cen[0] = P.cen; L.seg_b[0] = P.b;
      L.seg_tb[0] = P.tb; L.seg_tp[0] = P.tp;
    }
  }
  __syncthreads();

  phase_mark(C, L, 0);
  // ---- fetch and decode (all loads of all items issued together) ----------
  const int32_t ntt = C.ntt;
  int seg[IT], slot[IT], op[IT];
  int32_t cen[IT];
  int64_t idx[IT];
  int64_t tb[IT];      // arena base of the item's tree
  uint32_t tp[IT];     // its first type id | parameter << 8
  int32_t code[IT], a0v[IT];
  // a1..a3: loaded with code and a0 when the item's program reads them
  // (the program is known from the tree before the entry's type is)
  constexpr bool kWide = (OPS & (OPS_NQ | OPS_MS | OPS_FFT)) != 0;
  int32_t a1v[IT], a2v[IT], a3v[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const uint32_t w = w0 + (uint32_t)(k * WG + tid);
    seg[k] = -1; slot[k] = 0; cen[k] = 0; idx[k] = 0; code[k] = 0; a0v[k] = 0; op[k] = OP_NONE;
    tb[k] = 0; tp[k] = 0;
    a1v[k] = a2v[k] = a3v[k] = 0;
    if (w < S) {
      int s = 0;
      if (MULTI && nL > 1) {   // segments past the item's offset in the chunk cannot hold it
        int lo2 = 0, hi2 = min(L.nseg - 1, (int)(w - w0));
        while (lo2 < hi2) { const int mid = (lo2 + hi2) >> 1; if (L.win[mid] <= w) lo2 = mid + 1; else hi2 = mid; }
        s = lo2;
      }
      seg[k] = s;
      slot[k] = L.seg_slot[s];
      cen[k] = L.seg_cen[s];
      tb[k] = (int64_t)L.seg_tb[s] << 6;
      tp[k] = L.seg_tp[s];
      idx[k] = tb[k] + L.seg_b[s] + (int64_t)(w - (s == 0 ? L.off0 : L.win[s - 1]));
      if (hit) {
        code[k] = pf.code[k]; a0v[k] = pf.a0[k];
        a1v[k] = pf.a1[k]; a2v[k] = pf.a2[k]; a3v[k] = pf.a3[k];
      } else {
        code[k] = C.code[idx[k]];
        a0v[k] = C.a0[idx[k]];
        if (kWide) {
          const int pop = L.op_tab[tp[k] & 0xFF];   // the program's first operation
          if (pop == OP_Q || pop == OP_MS || pop == OP_FFT) { a1v[k] = C.a1[idx[k]]; a2v[k] = C.a2[idx[k]]; }
          if (pop == OP_Q) a3v[k] = C.a3[idx[k]];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    if (code[k] != 0) {
      const int32_t gtype = code[k] - cen[k] * ntt;
      if (gtype >= 1 && gtype <= ntt) op[k] = L.op_tab[gtype];
      // an entry outside the epoch's encoding window, or of a type this
      // kernel was not built for, is an error of its tree
      if (op[k] == OP_NONE || (opbit(op[k]) & OPS) == 0) {
        op[k] = OP_NONE;
        const int32_t prev = or_agent(MULTI ? &C.hot[slot[k]].flags : &C.plain->flags[P.par],
                                      (int32_t)TF_ENCODING);
        if (prev < 0) L.sink = prev;
      }
    }
  }

  // ---- task bodies: decide children, join or emit ---------------------------
  int nk[IT], act[IT];
  int64_t val[IT];
  int32_t x0[IT], x1[IT], x2[IT], x3[IT];
  bool want_map[IT], leaf[IT], fleaf[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    int32_t *errf = MULTI ? &C.hot[slot[k]].flags : &C.plain->flags[P.par];
    task_body<OPS>(C, op[k], a0v[k], a1v[k], a2v[k], a3v[k], tb[k], tp[k], slot[k], errf, L.sink, nk[k], act[k],
                   val[k], x0[k], x1[k], x2[k], x3[k], want_map[k], leaf[k], fleaf[k]);
  }

  // ---- traversal visits (postorder's visit continuation, a preorder task
  // with a node): each appends its node to the tree's log, whose last word
  // (log[n]) counts the visits; one atomic per wavefront when its visiting
  // lanes share a tree
  if constexpr ((OPS & OPS_PO) != 0) {
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const bool vis = op[k] == OP_PVISIT || (op[k] == OP_PRE && nk[k] == 2);
      const uint64_t m = ballot64(vis);
      if (!m) continue;
      int32_t *log = vis ? (int32_t *)C.ts[slot[k]].ptr2 : nullptr;
      const int32_t n = (int32_t)(tp[k] >> 8);
      int32_t pos = 0;
      const int leader = __ffsll((unsigned long long)m) - 1;
      const int s0 = __shfl(seg[k], leader, 64);
      if (__all(!vis || seg[k] == s0)) {
        int32_t base = 0;
        if (lane == leader) base = atomicAdd(&log[n], __popcll(m));
        pos = __shfl(base, leader, 64) + mbcnt64(m);
      } else if (vis) {
        pos = atomicAdd(&log[n], 1);
      }
      if (vis && pos >= 0 && pos < n) log[pos] = a0v[k];   // (more visits than nodes: the input was no tree)
    }
  }

  // ---- FFT leaves (at most 64 points): each is transformed by a whole
  // wavefront, lane j holding point j; the lanes load their inputs in
  // bit-reversed order and run the radix-2 butterfly stages across lanes.
  // Leaves go G at a time, their gathers in flight together (G = 4 in the
  // kernel for FFT alone, 2 where other programs' registers are live too).
  if constexpr ((OPS & OPS_FFT) != 0) {
    constexpr int G = OPS == OPS_FFT ? 8 : 2;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      uint64_t lm = ballot64(fleaf[k]);
      while (lm) {
        // the next leaves' parameters, read from their lanes into scalar
        // registers (lg = -1: no such leaf)
        int32_t lo[G], ls[G], sl[G], lg[G];
        float2 v[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          lg[g] = -1; lo[g] = ls[g] = sl[g] = 0;
          v[g] = make_float2(0.f, 0.f);
          if (lm) {
            const int src = __ffsll((unsigned long long)lm) - 1;
            lm &= lm - 1;
            lo[g] = __builtin_amdgcn_readlane(a0v[k], src);
            const int32_t o = __builtin_amdgcn_readlane(a1v[k], src);
            ls[g] = __builtin_amdgcn_readlane(a2v[k], src);
            sl[g] = __builtin_amdgcn_readlane(slot[k], src);
            lg[g] = (int)((uint32_t)__builtin_amdgcn_readlane((int32_t)tp[k], src) >> 8) - ls[g];
            if (lane < (1 << lg[g])) {
              const int j = lg[g] > 0 ? (int)(__builtin_bitreverse32((uint32_t)lane) >> (32 - lg[g])) : 0;
              v[g] = ((const float2 *)C.ts[sl[g]].ptr0)[o + (j << ls[g])];
            }
          }
        }
        // stage by stage across the group, so that the leaves' cross-lane
        // exchanges overlap; a stage's twiddle is the same for every leaf
        int lgmax = lg[0];
#pragma unroll
        for (int g = 1; g < G; ++g) lgmax = max(lgmax, lg[g]);
        for (int st = 0; st < lgmax; ++st) {
          const int h = 1 << st;
          float sn, cs;
          sincospif((float)(lane & (h - 1)) / (float)h, &sn, &cs);   // w = exp(-i pi k / h)
          const bool hi = (lane & h) != 0;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            if (st >= lg[g]) continue;   // (uniform across the wavefront)
            const float pr = __shfl(v[g].x, lane ^ h, 64), pi = __shfl(v[g].y, lane ^ h, 64);
            if (hi) {          // b: the partner holds a; b' = a - w b
              const float tr = cs * v[g].x + sn * v[g].y, ti = cs * v[g].y - sn * v[g].x;
              v[g] = make_float2(pr - tr, pi - ti);
            } else {           // a: the partner holds b; a' = a + w b
              const float tr = cs * pr + sn * pi, ti = cs * pi - sn * pr;
              v[g] = make_float2(v[g].x + tr, v[g].y + ti);
            }
          }
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
          if (lg[g] >= 0 && lane < (1 << lg[g])) ((float2 *)C.ts[sl[g]].ptr1)[lo[g] + lane] = v[g];
      }
    }
  }

  // ---- merge-sort leaves: each wavefront sorts its lanes' runs, 8 at a time,
  // all 64 lanes on each run (the leaf body is "sort these <= 64 keys"; the
  // keys it leaves behind are those of an insertion sort)
  if (OPS & opbit(OP_MS)) {
    constexpr int B = 8;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      uint64_t lm = ballot64(leaf[k]);
      while (lm) {
        uint32_t v[B];
        int32_t lo[B], n[B];
        uint32_t *dst[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
          n[b] = 0; lo[b] = 0; dst[b] = nullptr; v[b] = 0xFFFFFFFFu;
          if (lm) {
            const int l = __ffsll((unsigned long long)lm) - 1;
            lm &= lm - 1;
            const int32_t d = __shfl(x2[k], l, 64);
            lo[b] = __shfl(x0[k], l, 64);
            n[b] = __shfl(x1[k], l, 64) - lo[b];
            const TreeStatic *T = &C.ts[__shfl(slot[k], l, 64)];
            const uint32_t *keys = (const uint32_t *)T->ptr0;
            dst[b] = (d & 1) ? (uint32_t *)T->ptr1 : (uint32_t *)T->ptr0;
            if (lane < n[b]) v[b] = keys[lo[b] + lane];
          }
        }
        wave_bitonic64<B>(v);
#pragma unroll
        for (int b = 0; b < B; ++b)
          if (lane < n[b]) dst[b][lo[b] + lane] = v[b];
      }
    }
  }

  // ---- map (Section 4.2): a MERGE continuation hands its merge to the
  // data-parallel map phase that runs before the next epoch.  One atomic per
  // work-group reserves job slots and output units together.
  if (OPS & opbit(OP_MERGE)) {
    int jl = 0;
    int64_t ul = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k)
      if (want_map[k]) { ++jl; ul += (int64_t)(x1[k] - x0[k]); }
    if (__syncthreads_or(jl > 0)) {
      int jtot;
      int jpre = wg_excl_scan<WG>(jl, L.scan_tmp, &jtot);
      int64_t utot;
      int64_t upre = wg_excl_scan64<WG>(ul, L.scan_tmp64, &utot);
      if (tid == 0) {
        uint64_t *ctr = MULTI ? &C.hdr->map_ctr : &C.plain->map[P.par];
        const uint64_t prev = add_agent(ctr, ((uint64_t)jtot << kMapShift) | (uint64_t)utot);
        L.jbase = (uint32_t)(prev >> kMapShift);
        L.ubase = prev & kMapUnitMask;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        if (!want_map[k]) continue;
        const uint32_t j = L.jbase + (uint32_t)jpre;
        const TreeStatic *T = &C.ts[slot[k]];
        if (j < (uint32_t)C.mj_cap) {
          C.mj_lo[j] = x0[k]; C.mj_hi[j] = x1[k];
          C.mj_src[j] = ((x2[k] + 1) & 1) ? (const uint32_t *)T->ptr1 : (const uint32_t *)T->ptr0;
          C.mj_dst[j] = (x2[k] & 1) ? (uint32_t *)T->ptr1 : (uint32_t *)T->ptr0;
          C.mj_off[j] = L.ubase + (uint64_t)upre;
        } else {   // job list full: this lane merges by itself
          ms_merge((uint32_t *)T->ptr0, (uint32_t *)T->ptr1, x0[k], x1[k], x2[k]);
        }
        ++jpre;
        upre += (int64_t)(x1[k] - x0[k]);
      }
    }
  }

  // ---- fork: co-operative slot allocation, structure-of-arrays writes ------
  __syncthreads();
  phase_mark(C, L, 1);
  int off[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    // joins (and, when tracing, valid tasks) per tree segment
    seg_add_pair(L.seg_jv, seg[k], act[k] == ACT_JOIN, op[k] != OP_NONE);
    off[k] = lds_reserve(L.seg_cnt, seg[k], nk[k]);
  }
  seg_commit<WG, MULTI>(C, L, P, true);
  phase_mark(C, L, 2);
  // The previous chunk's finish check: with prefetching, here, where nothing
  // issued later than its atomic is still in flight (a tree whose last items
  // that chunk retired has none in this chunk); otherwise at the bookkeeping.
  if (MULTI && kPrefetch) settle(C, pend);
  // Prefetch: when the next chunk of the run lies wholly inside this chunk's
  // only tree, issue its loads now (after the allocation atomic has returned,
  // before this chunk's stores): they complete during the stores, the
  // bookkeeping and the barrier.  (Vector memory operations complete in
  // order, so loads issued before this chunk's own waits would be waited
  // for there.)
  pf.w0 = 0xFFFFFFFFu;
  if (kPrefetch) {
    const uint32_t n0 = w0 + (uint32_t)kChunk;
    if (n0 < run_end && L.nseg == 1 && L.win[0] >= min(n0 + (uint32_t)kChunk, S)) {
      const int64_t base = ((int64_t)L.seg_tb[0] << 6) + L.seg_b[0] - (int64_t)L.off0;
      const int pop = kWide ? L.op_tab[L.seg_tp[0] & 0xFF] : OP_NONE;
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        const uint32_t w = n0 + (uint32_t)(k * WG + tid);
        pf.code[k] = 0; pf.a0[k] = 0; pf.a1[k] = 0; pf.a2[k] = 0; pf.a3[k] = 0;
        if (w < S) {
          const int64_t i = base + (int64_t)w;
          pf.code[k] = C.code[i];
          pf.a0[k] = C.a0[i];
          if (kWide) {
            if (pop == OP_Q || pop == OP_MS) { pf.a1[k] = C.a1[i]; pf.a2[k] = C.a2[i]; }
            if (pop == OP_Q) pf.a3[k] = C.a3[i];
          }
        }
      }
      pf.w0 = n0;
    }
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int32_t cb = child_base(L.seg_base, seg[k], nk[k], off[k]);
    if (nk[k] > 0 && cb >= 0) {
      const int64_t c = tb[k] + cb;
      const int32_t nxt = (cen[k] + 1) * ntt + (int32_t)(tp[k] & 0xFF);   // local type 1, next epoch
      if (op[k] == OP_FIB32 || op[k] == OP_FIB64) {
        C.code[c] = nxt; C.a0[c] = x0[k] - 1;
        C.code[c + 1] = nxt; C.a0[c + 1] = x0[k] - 2;
      } else if (op[k] == OP_Q) {
        const int32_t n = (int32_t)(tp[k] >> 8);
        const uint32_t full = (1u << n) - 1u;
        const uint32_t cols = (uint32_t)x1[k], ld = (uint32_t)x2[k], rd = (uint32_t)x3[k];
        uint32_t avail = ~(cols | ld | rd) & full;
        int64_t cc = c;
        while (avail) {
          const uint32_t bit = avail & (0u - avail);
          avail ^= bit;
          C.code[cc] = nxt;
          C.a0[cc] = x0[k] + 1;
          C.a1[cc] = (int32_t)(cols | bit);
          C.a2[cc] = (int32_t)(((ld | bit) << 1) & full);
          C.a3[cc] = (int32_t)((rd | bit) >> 1);
          ++cc;
        }
      } else if (op[k] == OP_MS) {
        const int32_t mid = x0[k] + (x1[k] - x0[k]) / 2;
        C.code[c] = nxt; C.a0[c] = x0[k]; C.a1[c] = mid; C.a2[c] = x2[k] + 1;
        C.code[c + 1] = nxt; C.a0[c + 1] = mid; C.a1[c + 1] = x1[k]; C.a2[c + 1] = x2[k] + 1;
      } else if (op[k] == OP_POST || op[k] == OP_PRE) {
        C.code[c] = nxt; C.a0[c] = x1[k];
        C.code[c + 1] = nxt; C.a0[c + 1] = x2[k];
      } else if (op[k] == OP_FFT) {
        // even-index half into [lo, lo + n/2), odd-index half after it
        const int32_t h = 1 << ((int)(tp[k] >> 8) - x2[k] - 1);
        C.code[c] = nxt; C.a0[c] = x0[k]; C.a1[c] = x1[k]; C.a2[c] = x2[k] + 1;
        C.code[c + 1] = nxt; C.a0[c + 1] = x0[k] + h; C.a1[c + 1] = x1[k] + (1 << x2[k]);
        C.a2[c + 1] = x2[k] + 1;
      }
    }
    // ---- join / emit: writes to the item's own entry ----------------------
    const int64_t i = idx[k];
    if (act[k] == ACT_EMIT) {
      C.r[i] = val[k];
      C.code[i] = 0;
    } else if (act[k] == ACT_FINISH) {
      C.code[i] = 0;
    } else if (act[k] == ACT_JOIN) {
      C.code[i] = cen[k] * ntt + (int32_t)(tp[k] & 0xFF) + 1;   // local type 2: SUM / QSUM / MERGE / visit
      if (op[k] != OP_MS && op[k] != OP_POST && op[k] != OP_FFT) {   // (their joins keep their own arguments)
        C.a0[i] = cb;
        if (op[k] == OP_Q) C.a1[i] = nk[k];
      }
    }
  }

  __syncthreads();
  phase_mark(C, L, 3);
  // ---- co-operative expansion: the arcs of BFS and SSSP visits, the
  // butterflies of FFT combines (units of work spread over the work-group's
  // lanes after a scan of the items' unit counts)
  int arc_job = -1;   // >= 0: this chunk's units (and its retirement) went to that job
  if constexpr ((OPS & OPS_EXPAND) != 0) {
    constexpr bool kSssp = (OPS & OPS_SSSP) != 0;
    constexpr bool kArcs = (OPS & OPS_GRAPH) != 0;
    constexpr bool kFft = (OPS & OPS_FFT) != 0;
    bool anyv = false, anyc = false;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      anyv |= (op[k] == OP_VISIT || op[k] == OP_SVISIT || op[k] == OP_COMB);
      anyc |= (op[k] == OP_COMB);
    }
    if (__syncthreads_or(anyv)) {
      // deg: units of the item; -1: an SSSP visit that waits (dvs then holds
      // the distance that forked it)
      int32_t deg[IT], row[IT], dvs[IT];
      bool anyw = false;
      int dsum = 0;
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        deg[k] = 0; row[k] = 0; dvs[k] = -1;
        if (op[k] == OP_VISIT || op[k] == OP_SVISIT) {
          int32_t off = 0;     // SSSP: the distance that forked the visit (its a1)
          bool waits = false;  // with a bucket width delta (> 0), a visit whose distance
                               // is at least (CEN + 1) * delta waits: it forks itself unchanged
          if (kSssp && op[k] == OP_SVISIT) {
            off = C.a1[idx[k]];
            const int32_t delta = (int32_t)(tp[k] >> 8);
            waits = delta > 0 && (int64_t)off >= (int64_t)(cen[k] + 1) * delta;
          }
          if (waits) {
            deg[k] = -1; dvs[k] = off; anyw = true;
          } else {
            const TreeStatic *ST = &C.ts[slot[k]];
            const int32_t *rp = (const int32_t *)ST->ptr0;
            row[k] = rp[a0v[k]];
            deg[k] = rp[a0v[k] + 1] - row[k];
            // SSSP: the vertex's distance as it stands now.  If a lower one
            // than the entry's has been set since, it forked another visit,
            // which relaxes the arcs instead (this one is stale)
            if (kSssp && op[k] == OP_SVISIT) {
              dvs[k] = ld_agent((const int32_t *)ST->ptr2 + a0v[k]);
              if (dvs[k] < off) deg[k] = 0;
            }
          }
        } else if (kFft && op[k] == OP_COMB) {
          // COMB(lo, ls): n/2 butterflies over outputs [lo, lo + n)
          row[k] = a0v[k];
          deg[k] = 1 << ((int)(tp[k] >> 8) - a2v[k] - 1);
          dvs[k] = -(a2v[k] + 2);
        }
        dsum += max(deg[k], 0);
      }
      int tot;
      int pre = wg_excl_scan<WG>(dsum, L.scan_tmp, &tot);
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        V.row[tid * IT + k] = row[k];
        V.pre[tid * IT + k] = pre;
        V.seg[tid * IT + k] = seg[k];
        if (kSssp || kFft) V.dv[tid * IT + k] = dvs[k];
        pre += max(deg[k], 0);
      }
      if (tid == 0) V.qn = 0;
      // many units: published as tiles for every work-group (batched forms;
      // butterflies, cheap and uniform, in smaller tiles than arcs)
      const bool bfly = kFft && __syncthreads_or(anyc);
      __syncthreads();
      // waiting visits: queued as their own copies for the next epoch (at
      // most kChunk, so the queue keeps room for one step's claims); the
      // expansion below flushes them with its first step
      bool waits = false;
      if constexpr (kSssp) {
        waits = __syncthreads_or(anyw);
        if (waits) {
#pragma unroll
          for (int k = 0; k < IT; ++k) {
            if (deg[k] >= 0) continue;
            const int q = atomicAdd(&V.qn, 1);
            V.qu[q] = a0v[k];
            V.qs[q] = (int16_t)seg[k];
            V.qd[q] = dvs[k];
          }
          __syncthreads();
        }
      }
      if constexpr (MULTI) {
        if (tot > kArcLocal) arc_job = publish_arcs<WG>(C, L, V, tot, bfly ? kBflyTilesMax : kArcTilesMax);
      }
      // One arc per lane per step.  A claimed vertex is queued in LDS; the
      // queue is turned into child entries in bulk (one device atomic per
      // tree per flush) when it is nearly full and at the end.
      constexpr int A = arcs_per_lane<WG>();
      static_assert(WG * A <= kClaimQ / 2, "claim queue too small for one step");
      int from = 0;   // arcs are visited in increasing order: item searches only move forward
      static_assert(kChunk <= kClaimQ - WG * A, "claim queue too small for a chunk's waits and a step");
      const int lim = arc_job >= 0 ? 0 : tot;   // units this work-group expands itself
      for (int e0 = 0; e0 < lim || (waits && e0 == 0); e0 += WG * A) {
        int32_t u[A], sseg[A];   // arc: head vertex; butterfly: k
        int32_t *dep[A];
        int32_t dv[A];   // arc: the head's depth or distance as probed; butterfly: log2 of n/2
        int32_t nd[A];   // SSSP arc: the distance it offers its head; BFS arc: -1
        float2 *fy[A];   // butterfly: the combine's first output
        float2 bu[A], bb[A];
        bool bf[A];
#pragma unroll
        for (int a = 0; a < A; ++a) {
          const int e = e0 + a * WG + tid;
          sseg[a] = -1;
          nd[a] = -1;
          bf[a] = false;
          if (e < lim) {
            int lo = from, hi = kChunk;   // last item with pre <= e
            while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (V.pre[mid] <= e) lo = mid; else hi = mid; }
            from = lo;
            sseg[a] = V.seg[lo];
            const TreeStatic *ST = &C.ts[L.seg_slot[sseg[a]]];
            if (kFft && V.dv[lo] <= -2) {
              bf[a] = true;
              fy[a] = (float2 *)ST->ptr1 + V.row[lo];
              u[a] = e - V.pre[lo];
              dv[a] = (int)(L.seg_tp[sseg[a]] >> 8) + V.dv[lo] + 1;   // log2 N - ls - 1
            } else if (kArcs) {
              const int32_t arc = V.row[lo] + (e - V.pre[lo]);
              u[a] = ((const int32_t *)ST->ptr1)[arc];
              dep[a] = (int32_t *)ST->ptr2;
              if (kSssp && V.dv[lo] >= 0) nd[a] = V.dv[lo] + ((const int32_t *)ST->ptr3)[arc];
            }
          }
        }
#pragma unroll
        for (int a = 0; a < A; ++a) {   // probes and butterfly inputs issued together
          if (kFft && bf[a]) { bu[a] = fy[a][u[a]]; bb[a] = fy[a][u[a] + (1 << dv[a])]; }
          else if (kArcs) dv[a] = sseg[a] >= 0 ? dep[a][u[a]] : 0;
        }
#pragma unroll
        for (int a = 0; a < A; ++a) {
          // butterfly k: y[k], y[k + n/2] = y[k] +- exp(-2 pi i k / n) y[k + n/2].
          // BFS arc: test, then claim an unreached vertex; SSSP arc: test, then
          // lower the head's distance; either way the winner forks a visit of it
          bool won = false;
          if (kFft && bf[a]) {
            float sn, cs;
            sincospif((float)u[a] / (float)(1 << dv[a]), &sn, &cs);
            const float tr = cs * bb[a].x + sn * bb[a].y, ti = cs * bb[a].y - sn * bb[a].x;
            fy[a][u[a]] = make_float2(bu[a].x + tr, bu[a].y + ti);
            fy[a][u[a] + (1 << dv[a])] = make_float2(bu[a].x - tr, bu[a].y - ti);
          } else if (kArcs && sseg[a] >= 0) {
            if (kSssp && nd[a] >= 0) won = nd[a] < dv[a] && atomicMin(&dep[a][u[a]], nd[a]) > nd[a];
            else won = dv[a] == -1 && atomicCAS(&dep[a][u[a]], -1, L.seg_cen[sseg[a]] + 1) == -1;
          }
          if (kArcs && won) {
            const int q = atomicAdd(&V.qn, 1);
            V.qu[q] = u[a];
            V.qs[q] = (int16_t)sseg[a];
            if (kSssp) V.qd[q] = nd[a];
          }
        }
        if constexpr (kArcs) {
          __syncthreads();
          if (V.qn > kClaimQ - WG * A || e0 + WG * A >= lim) flush_claims<WG, MULTI, kSssp>(C, L, V, P);
        }
      }
    }
  }

  // ---- per-tree bookkeeping: retired items ----------------------------------
  __syncthreads();
  phase_mark(C, L, 4);
  const int nseg = L.nseg;
  if (MULTI && !kPrefetch) settle(C, pend);
  for (int s = tid; s < nseg; s += WG) {
    const int32_t j = L.seg_jv[s] & 0xFFFF;
    const int32_t v = (int32_t)((uint32_t)L.seg_jv[s] >> 16);
    L.seg_jv[s] = 0;
    if (MULTI) {
      const int sl = L.seg_slot[s];
      const uint32_t beg = (s == 0) ? L.off0 : L.win[s - 1];
      const uint32_t end = L.win[s];
      const uint32_t lo = max(beg, w0), hi = min(min(end, w0 + (uint32_t)kChunk), S);
      const uint32_t items = hi - lo;
      if (arc_job >= 0) {   // retired by the arc job's last tile
        int32_t *sg = C.arc_seg + C.arc_job[arc_job].sbase;
        sg[4 * kArcSegPool + s] = (int32_t)items;
        sg[5 * kArcSegPool + s] = (int32_t)(end - beg);
        sg[6 * kArcSegPool + s] = j | (v << 16);
        continue;
      }
      // (the valid count shares the done counter's line: performed before it)
      if (v) L.sink = add_agent(&C.hot[sl].valid, v);
      const uint64_t add = ((uint64_t)(uint32_t)j << 32) | items;
      PendingFinish f;
      f.slot = sl; f.items = items; f.range = end - beg; f.joins = (uint32_t)j;
      f.prev = add_agent(&C.hot[sl].done, add);
      if (s + WG < nseg) settle(C, f);   // (only a thread's last segment waits)
      else pend = f;
    } else {
      if (v) add_agent(&C.plain->valid[P.par], v);
    }
  }
  __syncthreads();
  phase_mark(C, L, 5);
}

// ---------------------------------------------------------------------------
// Batched epochs, one chunk per wavefront (the programs without co-operative
// expansion: fib, N-queens, merge sort, the traversals).  A wavefront sweeps
// its own run of work items, 64 * IT at a time, with no work-group barrier:
// its fork allocation takes one device atomic per tree it touches (the
// paper's one atomic per wavefront, Section 5.2.3), and so does its
// retirement count.  The CU overlaps the round trips of many wavefronts
// instead of stalling a whole work-group on each.
// ---------------------------------------------------------------------------
constexpr int kWSeg = 64;   // work-list entries a wavefront caches at once

struct NoWaveLds {};

struct WaveLds {
  uint32_t end[kWSeg];   // wl_off[kfirst + 1 + e]: where cached entry e ends (~0 past the list)
  int32_t slot[kWSeg];   // tree slot of entry e
  int32_t cen[kWSeg];    // its epoch number
  int32_t b[kWSeg];      // arena-relative start of its range
  uint32_t tb[kWSeg];    // its arena base / 64
  uint32_t tp[kWSeg];    // first type id | parameter << 8
  int32_t cnt[kWSeg];    // children requested per entry in this step (LDS atomics)
  int32_t base[kWSeg];   // arena-relative first child per entry (-1: overflow)
  int32_t jv[kWSeg];     // joins | valid tasks << 16 per entry in the current step
  uint32_t ritems[kWSeg];  // items retired per entry, not yet counted in the tree
  uint32_t rjoins[kWSeg];  // joins of those items
  uint32_t rvalid[kWSeg];  // valid tasks among them
  uint32_t beg0;         // wl_off[kfirst]
  int32_t kfirst;        // first cached entry (-1: nothing cached)
  int32_t sink;
  int32_t pad;
};

// Orders this wavefront's LDS writes before its later LDS reads of other
// lanes' words (one wavefront: no work-group barrier is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Counts the items the wavefront retired in its cached entries into their
// trees (one atomic per tree: retired items | joins << 32); the count that
// completes a tree's range runs its Phase 3.  Called when the cache is
// replaced and when the wavefront's run ends.
__device__ void wave_retire(const DevCtx &C, WaveLds &W) {
  const int lane = lane_id();
  const uint32_t it = W.ritems[lane];
  NextRange n;
  const int sl = W.slot[lane];
  if (W.kfirst >= 0 && it > 0) {
    const uint32_t j = W.rjoins[lane];
    const int32_t v = (int32_t)W.rvalid[lane];
    const uint32_t beg = (lane == 0) ? W.beg0 : W.end[lane - 1];
    if (v) W.sink = add_agent(&C.hot[sl].valid, v);
    const uint64_t prev = add_agent(&C.hot[sl].done, ((uint64_t)j << 32) | it);
    if ((uint32_t)prev + it == W.end[lane] - beg) n = tree_phase3(C, sl, (uint32_t)(prev >> 32) + j);
  }
  // the trees this wavefront completed the epoch of: one append for all
  // their next ranges
  const uint64_t m = ballot64(n.len > 0);
  if (m) {
    const int incl = wave_incl_scan(n.len);
    const uint32_t tot = (uint32_t)__shfl(incl, 63, 64);   // (every lane takes part in the shuffle)
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint64_t prev = 0;
    if (lane == leader) prev = add_agent(&C.hdr->wl_next, ((uint64_t)__popcll(m) << kWlShift) | (uint64_t)tot);
    prev = __shfl(prev, leader, 64);
    if (n.len > 0)
      wl_put(C, n, sl, (int)(prev >> kWlShift) + mbcnt64(m), (uint32_t)(prev & kWlItemMask) + (uint32_t)(incl - n.len));
  }
  W.ritems[lane] = 0;
  W.rjoins[lane] = 0;
  W.rvalid[lane] = 0;
  W.jv[lane] = 0;
  wave_sync();
}

// Caches the 64 work-list entries from the one holding item w (a 64-ary
// search of the entries' start offsets, then one round trip for the rest).
// wo: the current work-list buffer's first entry.
__device__ void wave_locate(const DevCtx &C, WaveLds &W, uint32_t w, int32_t nL, uint32_t wo) {
  const int lane = lane_id();
  const uint32_t *off = C.wl_off + wo;
  int lo = 0, hi = nL;
  while (hi - lo > 64) {   // last entry whose start is <= w
    const int step = (hi - lo + 63) >> 6;
    const int p = lo + lane * step;
    const bool ok = p < hi && off[p] <= w;
    lo = lo + (__popcll(ballot64(ok)) - 1) * step;
    hi = min(lo + step, hi);
  }
  // at most 64 candidates left: their starts and the entries after them
  // come in one round trip
  int e = lo + lane;
  uint32_t beg = e < nL ? off[e] : 0xFFFFFFFFu;
  uint32_t end = (e + 1 <= nL) ? off[e + 1] : 0xFFFFFFFFu;
  int32_t sl = 0, ce = 0, bb = 0;
  uint32_t tb = 0, tp = 0;
  if (e < nL) {
    sl = C.wl_tree[wo + e]; ce = C.wl_cen[wo + e]; bb = C.wl_b[wo + e];
    tb = C.wl_tb[wo + e]; tp = C.wl_tp[wo + e];
  }
  const int sh = __popcll(ballot64(e < nL && beg <= w)) - 1;   // the entry holding w, from lo
  if (sh > 0) {
    // cache from that entry on; the slots past the entries loaded repeat
    // the last end, so no item maps to them (the next locate loads on)
    const uint32_t end_last = __shfl(end, 63, 64);
    const int src = min(lane + sh, 63);
    beg = __shfl(beg, src, 64); end = __shfl(end, src, 64);
    sl = __shfl(sl, src, 64); ce = __shfl(ce, src, 64); bb = __shfl(bb, src, 64);
    tb = __shfl(tb, src, 64); tp = __shfl(tp, src, 64);
    if (lane + sh > 63) end = end_last;
    lo += sh;
    e = lo + lane;
  }
  W.end[lane] = end;
  if (e < nL) {
    W.slot[lane] = sl;
    W.cen[lane] = ce;
    W.b[lane] = bb;
    W.tb[lane] = tb;
    W.tp[lane] = tp;
  }
  W.cnt[lane] = 0;
  W.jv[lane] = 0;
  W.ritems[lane] = 0;
  W.rjoins[lane] = 0;
  W.rvalid[lane] = 0;
  const uint32_t b0 = __shfl(beg, 0, 64);
  if (lane == 0) {
    W.kfirst = lo;
    W.beg0 = b0;
  }
  wave_sync();
}

// Cached entry holding item w (its end lies above w; w is inside the cache).
__device__ __forceinline__ int wave_seg(const WaveLds &W, uint32_t w) {
  int lo = 0, hi = kWSeg - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (W.end[mid] <= w) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Traversal visits, merge-sort leaves and map registrations of a step's
// items (the parts of a task's body that act co-operatively): visits append
// to the tree's log with one atomic per wavefront and tree; the wavefront
// sorts its leaves, 8 at a time; merge continuations reserve map job slots
// and output units with one atomic per wavefront (Section 4.2).
template <uint32_t OPS, int IT>
__device__ __forceinline__ void wave_cooperative(const DevCtx &C, const int *seg, const int *slot, const int *op,
                                                 const uint32_t *tp, const int32_t *a0v, const int *nk,
                                                 const bool *leaf, const bool *want_map, const int32_t *x0,
                                                 const int32_t *x1, const int32_t *x2) {
  const int lane = lane_id();
  if constexpr ((OPS & OPS_PO) != 0) {
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const bool vis = op[k] == OP_PVISIT || (op[k] == OP_PRE && nk[k] == 2);
      const uint64_t m = ballot64(vis);
      if (!m) continue;
      int32_t *log = vis ? (int32_t *)C.ts[slot[k]].ptr2 : nullptr;
      const int32_t n = (int32_t)(tp[k] >> 8);
      int32_t pos = 0;
      const int leader = __ffsll((unsigned long long)m) - 1;
      const int s0 = __shfl(seg[k], leader, 64);
      if (__all(!vis || seg[k] == s0)) {
        int32_t bs = 0;
        if (lane == leader) bs = atomicAdd(&log[n], __popcll(m));
        pos = __shfl(bs, leader, 64) + mbcnt64(m);
      } else if (vis) {
        pos = atomicAdd(&log[n], 1);
      }
      if (vis && pos >= 0 && pos < n) log[pos] = a0v[k];
    }
  }
  if constexpr ((OPS & opbit(OP_MS)) != 0) {
    constexpr int B = 8;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      uint64_t lm = ballot64(leaf[k]);
      while (lm) {
        uint32_t v[B];
        int32_t lo[B], n[B];
        uint32_t *dst[B];
#pragma unroll
        for (int bb = 0; bb < B; ++bb) {
          n[bb] = 0; lo[bb] = 0; dst[bb] = nullptr; v[bb] = 0xFFFFFFFFu;
          if (lm) {
            const int l = __ffsll((unsigned long long)lm) - 1;
            lm &= lm - 1;
            const int32_t d = __shfl(x2[k], l, 64);
            lo[bb] = __shfl(x0[k], l, 64);
            n[bb] = __shfl(x1[k], l, 64) - lo[bb];
            const TreeStatic *T = &C.ts[__shfl(slot[k], l, 64)];
            const uint32_t *keys = (const uint32_t *)T->ptr0;
            dst[bb] = (d & 1) ? (uint32_t *)T->ptr1 : (uint32_t *)T->ptr0;
            if (lane < n[bb]) v[bb] = keys[lo[bb] + lane];
          }
        }
        wave_bitonic64<B>(v);
#pragma unroll
        for (int bb = 0; bb < B; ++bb)
          if (lane < n[bb]) dst[bb][lo[bb] + lane] = v[bb];
      }
    }
  }
  if constexpr ((OPS & opbit(OP_MERGE)) != 0) {
    int jl = 0;
    int64_t ul = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k)
      if (want_map[k]) { ++jl; ul += (int64_t)(x1[k] - x0[k]); }
    if (__any(jl > 0)) {
      const int jinc = wave_incl_scan(jl);
      const int64_t uinc = wave_incl_scan64(ul);
      const int jtot = __shfl(jinc, 63, 64);
      const int64_t utot = __shfl(uinc, 63, 64);
      uint64_t prev = 0;
      if (lane == 0) prev = add_agent(&C.hdr->map_ctr, ((uint64_t)jtot << kMapShift) | (uint64_t)utot);
      prev = __shfl(prev, 0, 64);
      uint32_t j = (uint32_t)(prev >> kMapShift) + (uint32_t)(jinc - jl);
      uint64_t u = (prev & kMapUnitMask) + (uint64_t)(uinc - ul);
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        if (!want_map[k]) continue;
        const TreeStatic *T = &C.ts[slot[k]];
        if (j < (uint32_t)C.mj_cap) {
          C.mj_lo[j] = x0[k]; C.mj_hi[j] = x1[k];
          C.mj_src[j] = ((x2[k] + 1) & 1) ? (const uint32_t *)T->ptr1 : (const uint32_t *)T->ptr0;
          C.mj_dst[j] = (x2[k] & 1) ? (uint32_t *)T->ptr1 : (uint32_t *)T->ptr0;
          C.mj_off[j] = u;
        } else {   // job list full: this lane merges by itself
          ms_merge((uint32_t *)T->ptr0, (uint32_t *)T->ptr1, x0[k], x1[k], x2[k]);
        }
        ++j;
        u += (uint64_t)(x1[k] - x0[k]);
      }
    }
  }
}

// A forking task's children, from c (arena-relative, through the tree's
// arena pointers), and its own entry e: join (the continuation at the same
// epoch) or emit / finish.
template <int K>
__device__ __forceinline__ void write_task(int32_t *code, int32_t *a0, int32_t *a1, int32_t *a2, int32_t *a3, int64_t *r,
                                           int op, int act, int nk, int32_t cb, int32_t e, int32_t nxt, int32_t own,
                                           uint32_t tp, int64_t val, int32_t x0, int32_t x1, int32_t x2, int32_t x3,
                                           bool kids = true) {
  if (kids && nk > 0 && cb >= 0) {
    const int32_t c = cb;
    if (op == OP_FIB32 || op == OP_FIB64) {
      code[c] = nxt; a0[c] = x0 - 1;
      code[c + 1] = nxt; a0[c + 1] = x0 - 2;
    } else if (op == OP_Q) {
      const int32_t n = (int32_t)(tp >> 8);
      const uint32_t full = (1u << n) - 1u;
      const uint32_t cols = (uint32_t)x1, ld = (uint32_t)x2, rd = (uint32_t)x3;
      uint32_t avail = ~(cols | ld | rd) & full;
      int32_t cc = c;
      while (avail) {
        const uint32_t bit = avail & (0u - avail);
        avail ^= bit;
        code[cc] = nxt;
        a0[cc] = x0 + 1;
        a1[cc] = (int32_t)(cols | bit);
        a2[cc] = (int32_t)(((ld | bit) << 1) & full);
        a3[cc] = (int32_t)((rd | bit) >> 1);
        ++cc;
      }
    } else if (op == OP_MS) {
      const int32_t mid = x0 + (x1 - x0) / 2;
      code[c] = nxt; a0[c] = x0; a1[c] = mid; a2[c] = x2 + 1;
      code[c + 1] = nxt; a0[c + 1] = mid; a1[c + 1] = x1; a2[c + 1] = x2 + 1;
    } else if (op == OP_POST || op == OP_PRE) {
      code[c] = nxt; a0[c] = x1;
      code[c + 1] = nxt; a0[c + 1] = x2;
    }
  }
  if (act == ACT_EMIT) {
    r[e] = val;
    code[e] = 0;
  } else if (act == ACT_FINISH) {
    code[e] = 0;
  } else if (act == ACT_JOIN) {
    code[e] = own;   // local type 2: SUM / QSUM / MERGE / visit, same epoch
    if (op != OP_MS && op != OP_POST) {   // (their joins keep their own arguments)
      a0[e] = cb;
      if (op == OP_Q) a1[e] = nk;
    }
  }
}

// The N-queens children of a single-tree step, written with consecutive
// lanes on consecutive entries: the step's children fill one block from
// base (slot k's children from kb[k], lane by lane, each lane's nk[k] of
// them from off[k]); each output position finds its parent lane by a
// binary search over the lanes' running totals and takes the parent's
// board from it, and the child's column is the parent's r-th free one
// (r: the position's rank among the parent's children), as the lane-serial
// writer takes them in increasing order.
template <int IT>
__device__ __forceinline__ void write_q_children(int32_t *code, int32_t *a0, int32_t *a1, int32_t *a2, int32_t *a3,
                                                 int32_t base, const int *off, const int *nk, const int *kb,
                                                 const int32_t *x0, const int32_t *x1, const int32_t *x2,
                                                 const int32_t *x3, int32_t nxt, uint32_t tp) {
  const int lane = lane_id();
  const int32_t n = (int32_t)(tp >> 8);
  const uint32_t full = (1u << n) - 1u;
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int incl = off[k] + nk[k];   // the end of this lane's children
    for (int p0 = kb[k]; p0 < kb[k + 1]; p0 += 64) {
      const int p = p0 + lane;
      // the first lane whose children end after p (every lane searches, so
      // that every lane's register is there to be read)
      int lo = 0, hi = 63;
#pragma unroll
      for (int st = 0; st < 6; ++st) {
        const int mid = (lo + hi) >> 1;
        if (__shfl(incl, mid, 64) > p) hi = mid; else lo = mid + 1;
      }
      const int l = min(lo, 63);
      const int r = p - __shfl(off[k], l, 64);
      const int32_t row = __shfl(x0[k], l, 64);
      const uint32_t cols = (uint32_t)__shfl(x1[k], l, 64);
      const uint32_t ld = (uint32_t)__shfl(x2[k], l, 64), rd = (uint32_t)__shfl(x3[k], l, 64);
      if (p < kb[k + 1]) {
        uint32_t avail = ~(cols | ld | rd) & full;
        for (int i = 0; i < r; ++i) avail &= avail - 1u;
        const uint32_t bit = avail & (0u - avail);
        const int32_t c = base + p;
        code[c] = nxt;
        a0[c] = row + 1;
        a1[c] = (int32_t)(cols | bit);
        a2[c] = (int32_t)(((ld | bit) << 1) & full);
        a3[c] = (int32_t)((rd | bit) >> 1);
      }
    }
  }
}

// One step of a wavefront whose items [wa, wb) all belong to the tree of
// cached entry s: the tree's values are uniform (scalar registers), entries
// are addressed by 32-bit offsets from the tree's arena, and the wavefront
// takes one allocation atomic for all its children.
template <uint32_t OPS, int IT>
__device__ void wave_step_tree(const DevCtx &C, WaveLds &W, const uint8_t *op_tab, int s, uint32_t wa, uint32_t wb) {
  const int lane = lane_id();
  const int slot = __builtin_amdgcn_readfirstlane(W.slot[s]);
  const int32_t cen = __builtin_amdgcn_readfirstlane(W.cen[s]);
  const uint32_t tp = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)W.tp[s]);
  const uint32_t beg = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(s == 0 ? W.beg0 : W.end[s - 1]));
  const int32_t b = __builtin_amdgcn_readfirstlane(W.b[s]);
  const int64_t ab = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)W.tb[s]) << 6;
  int32_t *code = C.code + ab, *pa0 = C.a0 + ab, *pa1 = C.a1 + ab, *pa2 = C.a2 + ab, *pa3 = C.a3 + ab;
  int64_t *pr = C.r + ab;
  const int32_t ntt = C.ntt;
  const int t1 = (int)(tp & 0xFF);                 // the program's first type id
  const int32_t lo_code = cen * ntt;               // this epoch's codes: lo_code + type
  const int op1 = op_tab[t1], op2 = op_tab[min(t1 + 1, kMaxTypes)];
  const int pop = op1;                             // the program, by its first operation
  constexpr bool kWide = (OPS & (OPS_NQ | OPS_MS)) != 0;
  int32_t *errf = &C.hot[slot].flags;

  int32_t e[IT], a0v[IT], a1v[IT], a2v[IT], a3v[IT];
  int op[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const uint32_t w = wa + (uint32_t)(k * 64 + lane);
    e[k] = b + (int32_t)(w - beg);
    op[k] = OP_NONE;
    a0v[k] = a1v[k] = a2v[k] = a3v[k] = 0;
    int32_t cd = 0;
    if (w < wb) {
      cd = code[e[k]];
      a0v[k] = pa0[e[k]];
      if (kWide) {
        if (pop == OP_Q || pop == OP_MS) { a1v[k] = pa1[e[k]]; a2v[k] = pa2[e[k]]; }
        if (pop == OP_Q) a3v[k] = pa3[e[k]];
      }
    }
    if (cd != 0) {
      const int32_t gt = cd - lo_code;
      op[k] = gt == t1 ? op1 : (gt == t1 + 1 ? op2 : OP_NONE);
      if (op[k] == OP_NONE || (opbit(op[k]) & OPS) == 0) {   // outside the epoch's window
        op[k] = OP_NONE;
        W.sink = or_agent(errf, (int32_t)TF_ENCODING);
      }
    }
  }
  int nk[IT], act[IT];
  int64_t val[IT];
  int32_t x0[IT], x1[IT], x2[IT], x3[IT];
  bool want_map[IT], leaf[IT], fleaf[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k)
    task_body<OPS>(C, op[k], a0v[k], a1v[k], a2v[k], a3v[k], ab, tp, slot, errf, W.sink, nk[k], act[k], val[k],
                   x0[k], x1[k], x2[k], x3[k], want_map[k], leaf[k], fleaf[k]);
  if constexpr ((OPS & (OPS_PO | OPS_MS)) != 0) {
    int seg[IT], sl[IT];
    uint32_t tpk[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) { seg[k] = s; sl[k] = slot; tpk[k] = tp; }
    wave_cooperative<OPS, IT>(C, seg, sl, op, tpk, a0v, nk, leaf, want_map, x0, x1, x2);
  }
  // fork: the wavefront's children in one block of the tree's arena
  int off[IT], kb[IT + 1];
  int run = 0, joins = 0, valid = 0;
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    int tot;
    kb[k] = run;
    off[k] = run + wave_prefix_small<4>(nk[k], &tot);
    run += tot;
    joins += __popcll(ballot64(act[k] == ACT_JOIN));
    valid += __popcll(ballot64(op[k] != OP_NONE));
  }
  int32_t base = 0;
  if (run > 0) {
    if (lane == 0) {
      base = add_agent(&C.hot[slot].nfc, (int32_t)run);
      if (base < 0 || (int64_t)base + run > (int64_t)C.ts[slot].cap) {
        W.sink = or_agent(errf, (int32_t)TF_OVERFLOW);
        base = -1;
      }
    }
    base = __builtin_amdgcn_readfirstlane(base);
  }
  kb[IT] = run;
  const int32_t nxt = (cen + 1) * ntt + t1;   // local type 1, next epoch
  const int32_t own = lo_code + t1 + 1;       // local type 2, this epoch
  // N-queens children go out coalesced; the others' with their own entries
  const bool qkids = (OPS & opbit(OP_Q)) != 0 && pop == OP_Q;
  if constexpr ((OPS & opbit(OP_Q)) != 0) {
    if (qkids && base >= 0 && run > 0)
      write_q_children<IT>(code, pa0, pa1, pa2, pa3, base, off, nk, kb, x0, x1, x2, x3, nxt, tp);
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int32_t cb = nk[k] == 0 ? 0 : (base < 0 ? -1 : base + off[k]);
    write_task<0>(code, pa0, pa1, pa2, pa3, pr, op[k], act[k], nk[k], cb, e[k], nxt, own, tp, val[k], x0[k], x1[k],
                  x2[k], x3[k], !qkids);
  }
  // retirement: counted into the tree when the run moves on
  if (lane == 0) {
    W.ritems[s] += wb - wa;
    W.rjoins[s] += (uint32_t)joins;
    W.rvalid[s] += (uint32_t)valid;
  }
}

// Items [wa, w1) of the current epoch's work list, by one wavefront: steps of
// 64 * ITF items inside one tree take the scalar path above; steps that span
// trees (64 * IT items) locate each item's tree in the cached entries and
// take one allocation atomic per tree.  Retirements are counted once per
// tree when the run leaves the cached entries or ends.
template <uint32_t OPS, int IT, int ITF>
__device__ void run_wave(const DevCtx &C, WaveLds &W, const uint8_t *op_tab, uint32_t wa, uint32_t w1, int32_t nL,
                         uint32_t wo) {
  const int lane = lane_id();
  const int32_t ntt = C.ntt;
  constexpr bool kWide = (OPS & (OPS_NQ | OPS_MS)) != 0;
  while (wa < w1) {
    // ---- the cached entries must hold item wa ------------------------------
    if (!(W.kfirst >= 0 && W.beg0 <= wa && wa < W.end[kWSeg - 1])) {
      wave_retire(C, W);
      wave_locate(C, W, wa, nL, wo);
    }
    const uint32_t beg0 = W.beg0;
    const uint32_t end63 = W.end[kWSeg - 1];
    {
      const uint32_t wf = min(min(w1, wa + (uint32_t)(64 * ITF)), end63);
      const int s0 = wave_seg(W, wa);
      if (W.end[s0] >= wf) {   // one tree
        wave_step_tree<OPS, ITF>(C, W, op_tab, s0, wa, wf);
        wa = wf;
        continue;
      }
    }
    const uint32_t wb = min(min(w1, wa + (uint32_t)(64 * IT)), end63);   // this step's items
    const int s_lo = wave_seg(W, wa), s_hi = wave_seg(W, wb - 1);

    // ---- fetch and decode ------------------------------------------------------
    int seg[IT], slot[IT], op[IT];
    int32_t cen[IT];
    int64_t idx[IT], tb[IT];
    uint32_t tp[IT];
    int32_t code[IT], a0v[IT], a1v[IT], a2v[IT], a3v[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t w = wa + (uint32_t)(k * 64 + lane);
      seg[k] = -1; slot[k] = 0; cen[k] = 0; idx[k] = 0; tb[k] = 0; tp[k] = 0; op[k] = OP_NONE;
      code[k] = 0; a0v[k] = a1v[k] = a2v[k] = a3v[k] = 0;
      if (w < wb) {
        const int sg = wave_seg(W, w);
        seg[k] = sg;
        slot[k] = W.slot[sg];
        cen[k] = W.cen[sg];
        tb[k] = (int64_t)W.tb[sg] << 6;
        tp[k] = W.tp[sg];
        idx[k] = tb[k] + W.b[sg] + (int64_t)(w - (sg == 0 ? beg0 : W.end[sg - 1]));
        code[k] = C.code[idx[k]];
        a0v[k] = C.a0[idx[k]];
        if (kWide) {
          const int pop = op_tab[tp[k] & 0xFF];   // the program's first operation
          if (pop == OP_Q || pop == OP_MS) { a1v[k] = C.a1[idx[k]]; a2v[k] = C.a2[idx[k]]; }
          if (pop == OP_Q) a3v[k] = C.a3[idx[k]];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      if (code[k] != 0) {
        const int32_t gtype = code[k] - cen[k] * ntt;
        if (gtype >= 1 && gtype <= ntt) op[k] = op_tab[gtype];
        if (op[k] == OP_NONE || (opbit(op[k]) & OPS) == 0) {   // outside the epoch's window
          op[k] = OP_NONE;
          W.sink = or_agent(&C.hot[slot[k]].flags, (int32_t)TF_ENCODING);
        }
      }
    }

    // ---- task bodies -------------------------------------------------------------
    int nk[IT], act[IT];
    int64_t val[IT];
    int32_t x0[IT], x1[IT], x2[IT], x3[IT];
    bool want_map[IT], leaf[IT], fleaf[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k)
      task_body<OPS>(C, op[k], a0v[k], a1v[k], a2v[k], a3v[k], tb[k], tp[k], slot[k], &C.hot[slot[k]].flags,
                     W.sink, nk[k], act[k], val[k], x0[k], x1[k], x2[k], x3[k], want_map[k], leaf[k], fleaf[k]);
    wave_cooperative<OPS, IT>(C, seg, slot, op, tp, a0v, nk, leaf, want_map, x0, x1, x2);

    // ---- fork: one device atomic per tree of this step -------------------------
    int off[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      seg_add_pair(W.jv, seg[k], act[k] == ACT_JOIN, op[k] != OP_NONE);
      off[k] = lds_reserve(W.cnt, seg[k], nk[k]);
    }
    wave_sync();
    {
      const int es = s_lo + lane;
      if (es <= s_hi) {
        const int c = W.cnt[es];
        int bse = 0;
        if (c > 0) {
          W.cnt[es] = 0;
          const int sl = W.slot[es];
          bse = add_agent(&C.hot[sl].nfc, (int32_t)c);
          if (bse < 0 || (int64_t)bse + c > (int64_t)C.ts[sl].cap) {
            W.sink = or_agent(&C.hot[sl].flags, (int32_t)TF_OVERFLOW);
            bse = -1;
          }
        }
        W.base[es] = bse;
        // the step's items, counted into the tree when the run moves on
        const uint32_t bg = (es == 0) ? beg0 : W.end[es - 1];
        W.ritems[es] += min(W.end[es], wb) - max(bg, wa);
        const int32_t jv = W.jv[es];
        W.jv[es] = 0;
        W.rjoins[es] += (uint32_t)(jv & 0xFFFF);
        W.rvalid[es] += (uint32_t)jv >> 16;
      }
    }
    wave_sync();

    // ---- children and own entries -----------------------------------------------
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      if (seg[k] < 0) continue;
      const int32_t cb = child_base(W.base, seg[k], nk[k], off[k]);
      const int64_t ab = tb[k];
      write_task<0>(C.code + ab, C.a0 + ab, C.a1 + ab, C.a2 + ab, C.a3 + ab, C.r + ab, op[k], act[k], nk[k], cb,
                    (int32_t)(idx[k] - ab), (cen[k] + 1) * ntt + (int32_t)(tp[k] & 0xFF),
                    cen[k] * ntt + (int32_t)(tp[k] & 0xFF) + 1, tp[k], val[k], x0[k], x1[k], x2[k], x3[k]);
    }
    wa = wb;
  }
  wave_retire(C, W);   // the run's retirements
}

// ---------------------------------------------------------------------------
// Admission of a tree on the device: its descriptor, state and counters, and
// its root in entry 0 of its arena, to run in epoch 0 (Section 5.2.1).
// ---------------------------------------------------------------------------
__device__ void admit_one(const DevCtx &C, const Admit &a) {
  const int s = a.slot;
  ((TreeStatic *)C.ts)[s] = a.ts;
  TreeState T = {};
  T.cen = 0; T.b = 0; T.e = 1; T.old = 1; T.sp = 0; T.status = TS_LIVE; T.err = 0;
  T.epochs = 0; T.tasks = 0; T.launched = 0; T.result = 0; T.done_gepoch = -1;
  T.start_gepoch = -1; T.peak = 1; T.ntrace = 0;
  C.st[s] = T;
  TreeHot Hh = {};
  Hh.nfc = 1;
  C.hot[s] = Hh;
  C.t_len[s] = 1; C.t_cen[s] = 0; C.t_b[s] = 0;
  const int64_t r0 = a.ts.base;
  C.code[r0] = a.root_code;
  C.a0[r0] = a.a0; C.a1[r0] = a.a1; C.a2[r0] = a.a2; C.a3[r0] = a.a3;
  C.r[r0] = 0;
}

// Whether a program's per-vertex or log buffer is initialised before its
// first epoch (BFS depth, SSSP distance, a traversal's visit counter).
__device__ __forceinline__ bool needs_init(int kind) {
  return kind == TREES_PROG_BFS_CSR || kind == TREES_PROG_SSSP_CSR || kind == TREES_PROG_POSTORDER ||
         kind == TREES_PROG_PREORDER;
}

// Asynchronous run: adopt the trees published in the admission ring since the
// last look.  Each becomes a work-list entry of one item (its root, epoch 0)
// appended after the `*ctot` entries already built (whose items end at
// `*itot`); the ones whose buffers need initialising are listed for the init
// phase that precedes the next epoch's chunks.  Every thread of the scanning
// work-group calls it.
template <int WG, int NS>
__device__ void adopt(const DevCtx &C, Lds<WG, NS> &L, uint32_t wo, int *ctot, uint32_t *itot, int64_t g) {
  SchedHdr *H = C.hdr;
  const int tid = threadIdx.x;
  if (tid == 0) {
    const uint32_t tail = __hip_atomic_load(&C.ring->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
    L.sflag = (int)(tail - H->adm_head);
    L.scnt = H->initN;
  }
  __syncthreads();
  const int k0 = *ctot;
  const int nn = min(L.sflag, C.tmax - k0);   // (never clamped: a record needs a free slot)
  const uint32_t head = H->adm_head;
  __syncthreads();
  if (nn <= 0) return;
  for (int j = tid; j < nn; j += WG) {
    // the record, read word by word from host memory (no struct temporary:
    // this code is inlined into the epoch kernel and must stay lean)
    const Admit *a = &C.ring_adm[(head + (uint32_t)j) % (uint32_t)C.tmax];
    const int s = a->slot;
    const int64_t base = a->ts.base;
    const uint32_t tp = a->ts.tp;
    const int32_t kind = a->ts.kind;
    {
      const uint32_t *src = (const uint32_t *)&a->ts;
      uint32_t *dts = (uint32_t *)&C.ts[s];
      for (int w = 0; w < (int)(sizeof(TreeStatic) / 4); ++w) dts[w] = src[w];
    }
    TreeState *T = &C.st[s];
    T->cen = 0; T->b = 0; T->e = 1; T->old = 1; T->sp = 0; T->status = TS_LIVE; T->err = 0;
    T->epochs = 0; T->tasks = 0; T->launched = 0; T->result = 0; T->done_gepoch = -1;
    T->start_gepoch = g; T->peak = 1; T->ntrace = 0;
    TreeHot *Hh = &C.hot[s];
    Hh->nfc = 1; Hh->flags = 0; Hh->done = 0; Hh->valid = 0;
    C.t_len[s] = 1; C.t_cen[s] = 0; C.t_b[s] = 0;
    C.code[base] = a->root_code;
    C.a0[base] = a->a0; C.a1[base] = a->a1; C.a2[base] = a->a2; C.a3[base] = a->a3;
    C.r[base] = 0;
    const uint32_t k = wo + (uint32_t)(k0 + j);
    C.wl_tree[k] = s;
    C.wl_off[k] = *itot + (uint32_t)j;
    C.wl_b[k] = 0;
    C.wl_tb[k] = (uint32_t)(base >> 6);
    C.wl_tp[k] = tp;
    C.wl_cen[k] = 0;
    if (needs_init(kind)) C.init_slot[atomicAdd(&L.scnt, 1)] = s;
  }
  __syncthreads();
  if (tid == 0) {
    H->adm_head = head + (uint32_t)nn;
    H->initN = L.scnt;
    __hip_atomic_store(&C.ring->head, head + (uint32_t)nn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  __syncthreads();
  *ctot = k0 + nn;
  *itot += (uint32_t)nn;
}

// Asynchronous run: make the completion records written so far visible to
// the host (after the records themselves, and after any merge of the epoch
// the trees finished in).
__device__ __forceinline__ void publish_completions(const DevCtx &C) {
  SchedHdr *H = C.hdr;
  if (H->ctail_pub != H->ctail) {
    H->ctail_pub = H->ctail;
    __hip_atomic_store(&C.ring->ctail, H->ctail, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// The init phase of an asynchronous run: every work-group sweeps the buffers
// of the trees adopted by the last scan (grid-stride), before their roots run.
__device__ void run_inits(const DevCtx &C, int n) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int j = 0; j < n; ++j) {
    const TreeStatic &T = C.ts[C.init_slot[j]];
    int32_t *p = (int32_t *)T.ptr2;
    int64_t cnt = T.p0, src = T.p1;
    int32_t fill = -1;   // BFS depth
    if (T.kind == TREES_PROG_SSSP_CSR) fill = INT32_MAX;
    if (T.kind == TREES_PROG_POSTORDER || T.kind == TREES_PROG_PREORDER) { p += T.p0; cnt = 1; src = -1; fill = 0; }
    for (int64_t x = gid; x < cnt; x += step) p[x] = (x == src) ? 0 : fill;
  }
}

// ---------------------------------------------------------------------------
// End of an epoch (one work-group): the results of trees that finished, the
// totals of the next work list (appended during the epoch by the trees'
// Phase 3; at the start of a run, an exclusive scan of every slot's range
// length builds it here), adoption of submitted trees in an asynchronous
// run, and the header of the next epoch.
// ---------------------------------------------------------------------------
template <int WG, int NS>
__device__ void schedule_scan(const DevCtx &C, Lds<WG, NS> &L, bool after_epoch) {
  SchedHdr *H = C.hdr;
  const int tid = threadIdx.x;
  // an epoch that had no work list (an asynchronous run waiting for
  // submissions) is not counted
  const bool real = after_epoch && H->L > 0;
  if (after_epoch) {   // trees finished this epoch: result and end epoch
    const int nd = H->done_count;
    const int64_t ge = H->gepoch;
    const uint32_t ct = H->ctail;
    constexpr int RD = WG >= 1024 ? 1 : 1024 / WG;
    for (int j0 = 0; j0 < nd; j0 += WG * RD) {
      int slot[RD], err[RD];
      int64_t base[RD], res[RD];
#pragma unroll
      for (int r = 0; r < RD; ++r) {
        const int j = j0 + r * WG + tid;
        slot[r] = j < nd ? C.done_list[j] : -1;
      }
#pragma unroll
      for (int r = 0; r < RD; ++r) {
        err[r] = 1; base[r] = 0;
        if (slot[r] >= 0) { err[r] = C.st[slot[r]].err; base[r] = C.ts[slot[r]].base; }
      }
#pragma unroll
      for (int r = 0; r < RD; ++r) res[r] = (slot[r] >= 0 && err[r] == 0) ? C.r[base[r]] : 0;
#pragma unroll
      for (int r = 0; r < RD; ++r) {
        if (slot[r] < 0) continue;
        TreeState *T = &C.st[slot[r]];
        if (err[r] == 0) T->result = res[r];
        T->done_gepoch = ge;
      }
    }
    if (C.async_mode) {   // a completion record per finished tree, for the host
      __syncthreads();      // (the results above, written by other threads)
      for (int j = tid; j < nd; j += WG) {
        const int sl = C.done_list[j];
        const TreeState *T = &C.st[sl];
        Completion *q = &C.ring_done[(ct + (uint32_t)j) % (uint32_t)C.tmax];
        // (the state's fields, then the record's, one word at a time: the
        // record lives in host memory)
        const int32_t err = T->err;
        __hip_atomic_store(&q->slot, sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&q->err, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&q->epochs, T->epochs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&q->peak, T->peak, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&q->tasks, T->tasks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&q->launched, T->launched, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&q->result, err == 0 ? T->result : (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&q->start_gepoch, T->start_gepoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&q->done_gepoch, ge, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    if (C.async_mode && nd > 0) {   // the records are written; published below
      wait_vmem();
      __syncthreads();
      if (tid == 0) H->ctail = ct + (uint32_t)nd;
    }
  }
  // The next work list.  After an epoch it is complete already: each tree's
  // Phase 3 appended its next range to the other buffer, so only the totals
  // are read.  At the start of a run it is built here from every slot's
  // range: rounds of WG x R slots, every load of a round issued before any
  // of its values is used, then one work-group scan places the round.
  const int nb = after_epoch ? (H->wsel ^ 1) : 0;
  const uint32_t wo = (uint32_t)nb * (uint32_t)(C.tmax + 1);
  const int64_t g = H->gepoch + (real ? 1 : 0);
  int ctot = 0;
  uint32_t itot = 0;
  if (after_epoch) {
    const uint64_t pk = ld_agent(&H->wl_next);
    ctot = (int)(pk >> kWlShift);
    itot = (uint32_t)(pk & kWlItemMask);
  } else {
    const int n = H->tslots;
    constexpr int R = WG >= 1024 ? 1 : 1024 / WG;
    for (int base = 0; base < n; base += WG * R) {
      int slot[R], len[R], b[R], cen[R];
      int64_t tbase[R], sg[R];
      uint32_t tp[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int t = base + r * WG + tid;
        slot[r] = t < n ? t : -1;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        len[r] = 0; b[r] = 0; cen[r] = 0; tbase[r] = 0; tp[r] = 0; sg[r] = 0;
        if (slot[r] >= 0) {
          const int s = slot[r];
          len[r] = C.t_len[s]; b[r] = C.t_b[s]; cen[r] = C.t_cen[s];
          tbase[r] = C.ts[s].base; tp[r] = C.ts[s].tp; sg[r] = C.st[s].start_gepoch;
        }
      }
      int cnt = 0, items = 0;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (len[r] > 0) { ++cnt; items += len[r]; }
      int rc, ri;
      int k = ctot + wg_excl_scan<WG>(cnt, L.scan_tmp, &rc);
      uint32_t off = itot + (uint32_t)wg_excl_scan<WG>(items, L.scan_tmp, &ri);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (len[r] <= 0) continue;
        const int s = slot[r];
        C.wl_tree[wo + k] = s;
        C.wl_off[wo + k] = off;
        C.wl_b[wo + k] = b[r];
        C.wl_tb[wo + k] = (uint32_t)(tbase[r] >> 6);
        C.wl_tp[wo + k] = tp[r];
        C.wl_cen[wo + k] = cen[r];
        if (sg[r] < 0) C.st[s].start_gepoch = g;
        ++k;
        off += (uint32_t)len[r];
      }
      ctot += rc;
      itot += (uint32_t)ri;
    }
  }
  // Asynchronous run.  The work list now holds only live trees, so the slots
  // of the trees that finished this epoch may be handed back: their
  // completions are published now, or, if the epoch registered merges, after
  // the map phase that completes them.  Then the trees submitted since the
  // last look are adopted, after the live ones (a slot the host has reused
  // already is no longer among them).
  const bool asy = C.async_mode != 0 && after_epoch;
  if (asy) {
    const bool merges = (ld_agent(&H->map_ctr) >> kMapShift) != 0;
    __syncthreads();
    if (tid == 0) {
      H->initN = 0;   // (the last scan's list was swept before this epoch)
      if (!merges) publish_completions(C);
    }
    __syncthreads();
    for (;;) {
      adopt<WG, NS>(C, L, wo, &ctot, &itot, g);
      if (ctot > 0 || merges) break;
      // Nothing live: wait for a submission, the close request or an abort,
      // for at most one slice; then run an empty epoch (every work-group
      // returns to the barrier, whose waits stay short).
      if (tid == 0) {
        const int64_t t0 = realtime();
        int more = 0;
        while (true) {
          if ((int)(__hip_atomic_load(&C.ring->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) - H->adm_head) > 0) {
            more = 1;
            break;
          }
          if (__hip_atomic_load(&C.ring->close, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
          if (C.abort_flag && *C.abort_flag) break;
          if (realtime() - t0 > C.slice_ticks) break;
          __builtin_amdgcn_s_sleep(8);
        }
        L.sflag = more;
      }
      __syncthreads();
      if (!L.sflag) break;
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (after_epoch) {   // the map jobs of this epoch run before the next one
      const uint64_t mc = ld_agent(&H->map_ctr);
      H->mapJ = (uint32_t)(mc >> kMapShift);
      st_agent(&H->map_ctr, (uint64_t)0);
    }
    if (!asy) H->initN = 0;
    st_agent(&H->chunk_ctr, 0u);   // every work-group has stopped claiming this epoch's chunks
    st_agent(&H->arc_jobs, 0u);    // and has left this epoch's arc phase
    st_agent(&H->arc_tiles, 0u);
    st_agent(&H->arc_segs, 0u);
    st_agent(&H->arc_next, 0u);
    H->arc_phase = 0;
    H->wsel = nb;
    st_agent(&H->wl_next, (uint64_t)0);   // the following epoch appends to the other buffer
    C.wl_off[wo + ctot] = (uint32_t)itot;
    H->S = (uint32_t)itot;
    H->L = ctot;
    H->live = ctot;
    H->done_count = 0;
    if (real) {
      if (H->run_epochs < kEpochStamps) H->stamp[H->run_epochs] = realtime();
      H->gepoch += 1;
      H->run_epochs += 1;
    }
    int stop = 0;
    if (ctot == 0) {
      stop = 1;
      if (C.async_mode) {   // an asynchronous run drains only once the host closes it
        const int64_t now = realtime();
        if (H->idle_t0 == 0) H->idle_t0 = now;
        const bool closed = __hip_atomic_load(&C.ring->close, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
        stop = closed ? 1 : (now - H->idle_t0 > C.idle_ticks ? 5 : 0);
        // a submission published before the close request is adopted first
        // (the host writes the tail before close, so it is visible here)
        if ((int)(__hip_atomic_load(&C.ring->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) - H->adm_head) > 0)
          stop = 0;
      }
    } else {
      H->idle_t0 = 0;
      if (H->max_epochs >= 0 && H->run_epochs >= H->max_epochs) stop = 2;
    }
    if (C.abort_flag && *C.abort_flag) stop = 3;
    if (H->stop_reason == 4) stop = 4;   // a barrier timed out: stay stopped
    H->stop = stop;
    if (stop) H->stop_reason = stop;
  }
  __syncthreads();
}

// The work-list scan out of line, reading the context from its copy in
// device memory: the epoch kernels' register budget (two work-groups per CU)
// is then set by their chunk code alone, not by the scan's.
template <int WG, int NS>
__device__ __noinline__ void schedule_scan_ext(const DevCtx *C, Lds<WG, NS> *L, int after_epoch) {
  schedule_scan<WG, NS>(*C, *L, after_epoch != 0);
}

template <int WG, int NS>
__device__ __forceinline__ void lds_init(const DevCtx &C, Lds<WG, NS> &L) {
  for (int t = threadIdx.x; t < NS; t += WG) { L.seg_cnt[t] = 0; L.seg_jv[t] = 0; }
  if (threadIdx.x <= kMaxTypes) L.op_tab[threadIdx.x] = C.op_of_type[threadIdx.x];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Plain form: one launch per epoch of one tree; grid covers the range.
// Publishes a plain epoch's counters to the host: the totals go to the
// host-mapped mirror, `seq` after the rest has landed, for the host to poll
// instead of synchronising the stream.  Run by one thread of the epoch's last
// work-group to finish.
__device__ void publish(const DevCtx &C, int32_t par, uint32_t seq) {
  PlainMirror *M = C.mirror;
  __hip_atomic_store(&M->fj, ld_agent(&C.plain->fj[par]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&M->map, ld_agent(&C.plain->map[par]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&M->valid, ld_agent(&C.plain->valid[par]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&M->flags, ld_agent(&C.plain->flags[par]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  wait_vmem();
  __hip_atomic_store(&M->seq, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int WG, uint32_t OPS>
__global__ __launch_bounds__(WG) void k_plain(DevCtx C, PlainArgs P) {
  using VL = typename std::conditional<(OPS & OPS_EXPAND) != 0, VisitLds, NoVisitLds>::type;
  __shared__ Lds<WG, 1> L;   // one tree: one segment
  __shared__ VL V;
  lds_init<WG>(C, L);
  if (C.debug) {
    if (threadIdx.x < 8) L.prof[threadIdx.x] = 0;
    if (threadIdx.x == 0) L.tprof = realtime();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int q = P.par ^ 1;   // the next epoch's counters
    C.plain->fj[q] = 0; C.plain->valid[q] = 0; C.plain->flags[q] = 0;
    C.plain->map[q] = 0;
  }
  const uint32_t S = (uint32_t)(P.e - P.b);
  PendingFinish none;
  Prefetch<kChunk / WG> nopf;
  run_chunk<WG, OPS, false>(C, L, V, blockIdx.x * kChunk, S, 1, P, none, nopf, 0u);
  phase_mark(C, L, 6);
  if (C.debug && threadIdx.x == 0)
    for (int ph = 0; ph < 8; ++ph) add_agent(&C.hdr->phase[ph], (uint64_t)L.prof[ph]);
  // The work-group that finishes last publishes the counters.  Every counter
  // moves only by device-scope atomics, and each work-group's have been
  // performed before it takes a ticket, so the last ticket sees every
  // work-group's counts (no cache writeback needed): the atomics whose result
  // a thread uses are waited for before the barrier; the one that returns
  // nothing (the valid count) is waited for here.
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = add_agent(&C.plain->ticket, 1u);
    if (t + 1 == P.nwg) {
      st_agent(&C.plain->ticket, 0u);   // for the next epoch's launch
      publish(C, P.par, P.seq);
    }
  }
}

// The arc phase: every work-group claims tiles of the epoch's expansion
// jobs.  A tile expands units [t * tile, (t + 1) * tile) of its job with the
// same steps as a chunk's own expansion (arcs: probe, then a BFS claim by CAS
// or an SSSP relaxation by atomic min, LDS queue, child entries in bulk; FFT
// butterflies: load, combine, store); the work-group that expands a job's
// last tile retires the owner chunk's items, running Phase 3 of a tree whose
// last items they were.
template <int WG, uint32_t OPS>
__device__ void arc_phase(const DevCtx &C, Lds<WG> &L, VisitLds &V) {
  constexpr bool kSssp = (OPS & OPS_SSSP) != 0;
  constexpr bool kArcs = (OPS & OPS_GRAPH) != 0;
  constexpr bool kFft = (OPS & OPS_FFT) != 0;
  SchedHdr *H = C.hdr;
  const int tid = threadIdx.x;
  const PlainArgs P{};
  const uint32_t T = min(ld_agent(&H->arc_tiles), (uint32_t)kArcTilesAll);
  constexpr int A = arcs_per_lane<WG>();
      static_assert(WG * A <= kClaimQ / 2, "claim queue too small for one step");
  while (true) {
    if (tid == 0) L.flag = (int)add_agent(&H->arc_next, 1u);
    __syncthreads();
    const uint32_t t = (uint32_t)L.flag;
    __syncthreads();
    if (t >= T) break;
    const int4 td = C.arc_tile[t];
    const int j = td.x;
    if (j < 0) continue;   // a reservation whose job was not kept
    const ArcJob *J = &C.arc_job[j];
    const int tot = J->tot, tile = J->tile, ntiles = J->ntiles, nseg = J->nseg;
    const int lt = (int)(t - J->tbase);
    const int ilo = td.y, ihi = td.z;
    const int32_t *it = C.arc_item + (size_t)j * kArcItemWords;
    for (int i = ilo + tid; i <= ihi; i += WG) {
      V.pre[i] = it[i];
      V.row[i] = it[kChunk + i];
      V.seg[i] = it[2 * kChunk + i];
      if (kSssp || kFft) V.dv[i] = it[3 * kChunk + i];
    }
    const int32_t *sg = C.arc_seg + J->sbase;
    for (int q = tid; q < nseg; q += WG) {
      L.seg_slot[q] = sg[q];
      L.seg_cen[q] = sg[kArcSegPool + q];
      L.seg_tb[q] = (uint32_t)sg[2 * kArcSegPool + q];
      L.seg_tp[q] = (uint32_t)sg[3 * kArcSegPool + q];
      L.seg_cnt[q] = 0;
    }
    if (tid == 0) { L.nseg = nseg; V.qn = 0; }
    __syncthreads();
    const int e_lo = lt * tile, e_hi = min(e_lo + tile, tot);
    int from = ilo;   // arcs in increasing order: item searches only move forward
    for (int e0 = e_lo; e0 < e_hi; e0 += WG * A) {
      int32_t u[A], sseg[A];
      int32_t *dep[A];
      int32_t dv[A];
      int32_t nd[A];   // SSSP arc: the distance it offers its head; BFS arc: -1
      float2 *fy[A];
      float2 bu[A], bb[A];
      bool bf[A];
#pragma unroll
      for (int a = 0; a < A; ++a) {
        const int e = e0 + a * WG + tid;
        sseg[a] = -1;
        nd[a] = -1;
        bf[a] = false;
        if (e < e_hi) {
          int lo = from, hi = ihi + 1;   // last item with pre <= e
          while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (V.pre[mid] <= e) lo = mid; else hi = mid; }
          from = lo;
          sseg[a] = V.seg[lo];
          const TreeStatic *ST = &C.ts[L.seg_slot[sseg[a]]];
          if (kFft && V.dv[lo] <= -2) {
            bf[a] = true;
            fy[a] = (float2 *)ST->ptr1 + V.row[lo];
            u[a] = e - V.pre[lo];
            dv[a] = (int)(L.seg_tp[sseg[a]] >> 8) + V.dv[lo] + 1;   // log2 N - ls - 1
          } else if (kArcs) {
            const int32_t arc = V.row[lo] + (e - V.pre[lo]);
            u[a] = ((const int32_t *)ST->ptr1)[arc];
            dep[a] = (int32_t *)ST->ptr2;
            if (kSssp && V.dv[lo] >= 0) nd[a] = V.dv[lo] + ((const int32_t *)ST->ptr3)[arc];
          }
        }
      }
#pragma unroll
      for (int a = 0; a < A; ++a) {   // probes and butterfly inputs issued together
        if (kFft && bf[a]) { bu[a] = fy[a][u[a]]; bb[a] = fy[a][u[a] + (1 << dv[a])]; }
        else if (kArcs) dv[a] = sseg[a] >= 0 ? dep[a][u[a]] : 0;
      }
#pragma unroll
      for (int a = 0; a < A; ++a) {
        bool won = false;
        if (kFft && bf[a]) {
          float sn, cs;
          sincospif((float)u[a] / (float)(1 << dv[a]), &sn, &cs);
          const float tr = cs * bb[a].x + sn * bb[a].y, ti = cs * bb[a].y - sn * bb[a].x;
          fy[a][u[a]] = make_float2(bu[a].x + tr, bu[a].y + ti);
          fy[a][u[a] + (1 << dv[a])] = make_float2(bu[a].x - tr, bu[a].y - ti);
        } else if (kArcs && sseg[a] >= 0) {
          if (kSssp && nd[a] >= 0) won = nd[a] < dv[a] && atomicMin(&dep[a][u[a]], nd[a]) > nd[a];
          else won = dv[a] == -1 && atomicCAS(&dep[a][u[a]], -1, L.seg_cen[sseg[a]] + 1) == -1;
        }
        if (kArcs && won) {
          const int q = atomicAdd(&V.qn, 1);
          V.qu[q] = u[a];
          V.qs[q] = (int16_t)sseg[a];
          if (kSssp) V.qd[q] = nd[a];
        }
      }
      if constexpr (kArcs) {
        __syncthreads();
        if (V.qn > kClaimQ - WG * A || e0 + WG * A >= e_hi) flush_claims<WG, true, kSssp>(C, L, V, P);
      }
    }
    // the tile's forks are performed before the tile counts as done
    wait_vmem();
    __syncthreads();
    if (tid == 0) L.flag = (add_agent(&((ArcJob *)J)->done, 1u) + 1u == (uint32_t)ntiles) ? 1 : 0;
    __syncthreads();
    if (L.flag) {   // the job's last tile: retire the owner chunk's items
      for (int q = tid; q < nseg; q += WG) {
        const int sl = L.seg_slot[q];
        const uint32_t items = (uint32_t)sg[4 * kArcSegPool + q];
        const uint32_t range = (uint32_t)sg[5 * kArcSegPool + q];
        const int32_t jv = sg[6 * kArcSegPool + q];
        const uint32_t joins = (uint32_t)(jv & 0xFFFF);
        const int32_t v = (int32_t)((uint32_t)jv >> 16);
        if (v) L.sink = add_agent(&C.hot[sl].valid, v);
        const uint64_t prev = add_agent(&C.hot[sl].done, ((uint64_t)joins << 32) | items);
        if ((uint32_t)prev + items == range) tree_finish(C, sl, (uint32_t)(prev >> 32) + joins);
      }
    }
    __syncthreads();
  }
}

// Grid barrier between epochs (Tenet 1: one arrival per work-group).  Every
// wavefront waits until its task-vector and state stores have reached the
// XCD's L2; then one thread writes the L2 back (a release) and arrives.  The
// last arriver optionally runs the work-list scan and opens the barrier.
// Leaving, one thread invalidates the CU's and XCD's caches (an acquire).
// wait = false (graph form): the others return at once, the kernel
// boundary is their barrier.  Returns 0 if this work-group gave up waiting
// after the spin limit, 2 if it is the last arriver and keeps the barrier
// closed to run the next epoch alone (SOLO: the largest such epoch, 0:
// never), 1 otherwise.
// Whether the next epoch (its work list just built) can run in this
// work-group alone: at most `kMax` items, and nothing in it that needs the
// grid (merges of the map phase, buffers of adopted trees to initialise).
// Thread 0 decides; the answer is in L.flag2.
template <uint32_t kMax, int WG, int NS>
__device__ __forceinline__ void solo_decide(const DevCtx &C, Lds<WG, NS> &L) {
  if (threadIdx.x == 0) {
    const SchedHdr *H = C.hdr;
    const uint32_t S = H->S, nL = (uint32_t)H->L, stop = (uint32_t)ld_agent(&H->stop), mapJ = H->mapJ,
                   initN = (uint32_t)H->initN, wsel = (uint32_t)H->wsel;
    L.hdr[0] = S; L.hdr[1] = nL; L.hdr[2] = stop; L.hdr[3] = mapJ; L.hdr[4] = initN; L.hdr[5] = wsel;
    L.flag2 = (kMax > 0 && stop == 0 && mapJ == 0 && initN == 0 && S > 0 && S <= kMax) ? 1 : 0;
  }
  __syncthreads();
}

// The release that opens the barrier (its arrival counter cleared first).
template <int WG, int NS>
__device__ __forceinline__ void barrier_release(const DevCtx &C, Lds<WG, NS> &L) {
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) {
    st_agent(&C.hdr->arrive, 0u);
    fence_release();
    __hip_atomic_store(&C.hdr->gen, L.gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int WG, int NS, uint32_t SOLO = 0>
__device__ int grid_barrier(const DevCtx &C, Lds<WG, NS> &L, bool with_scan, bool wait) {
  SchedHdr *H = C.hdr;
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) {
    // two-level arrival: work-groups arrive at their group's counter (group
    // = blockIdx % 8, one group per XCD under round-robin dispatch); the last
    // of each group arrives at the top counter
    const uint32_t g = ld_agent(&H->gen);
    fence_release();
    const uint32_t G = gridDim.x;
    const uint32_t ng = G < 8 ? G : 8;
    const uint32_t grp = blockIdx.x & 7;
    const uint32_t gsize = (G - grp + 7) / 8;
    int last = 0;
    const uint32_t a = add_agent(&H->grp[grp].n, 1u);
    if (a == gsize - 1) {
      st_agent(&H->grp[grp].n, 0u);
      const uint32_t b = add_agent(&H->arrive, 1u);
      last = (b == ng - 1);
    }
    L.flag = last;
    L.gen = g;
  }
  __syncthreads();
  if (L.flag) {
    if (threadIdx.x == 0) fence_acquire();
    __syncthreads();
    if (with_scan) {
      // an epoch that published arc jobs has its arc phase first; the
      // barrier that ends the arc phase builds the next work list
      if (threadIdx.x == 0) L.flag2 = (ld_agent(&H->arc_tiles) > 0u && H->arc_phase == 0) ? 1 : 0;
      __syncthreads();
      if (L.flag2) {
        if (threadIdx.x == 0) H->arc_phase = 1;
      } else {
        schedule_scan_ext<WG, NS>(C.self, &L, 1);
        if constexpr (SOLO > 0) {
          // a narrow next epoch: this work-group runs it alone and keeps the
          // barrier closed meanwhile (k_epochs)
          solo_decide<SOLO>(C, L);
          if (L.flag2) return 2;
        }
      }
    }
    barrier_release<WG, NS>(C, L);
  } else if (wait) {
    if (threadIdx.x == 0) {
      const int64_t t0 = realtime();
      int timed_out = 0;
      while (ld_agent(&H->gen) == L.gen) {
        __builtin_amdgcn_s_sleep(2);
        if (realtime() - t0 > C.timeout_ticks) { timed_out = 1; break; }
      }
      L.tflag = timed_out;
      if (timed_out) {   // give up: every other work-group stops at its next boundary
        st_agent(&H->stop_reason, 4);
        st_agent(&H->stop, 1);
      }
    }
    __syncthreads();
    if (L.tflag) return 0;
  }
  if (threadIdx.x == 0) fence_acquire();
  __syncthreads();
  return 1;
}

// Batched form.  persistent != 0: a co-resident grid loops over epochs with
// device grid barriers; an epoch that registered map jobs is followed by the
// map phase and one more barrier.  persistent == 0: one epoch per launch (a
// chain of such launches, each followed by a map launch, is captured in a
// graph); the last work-group to finish builds the next work list and the
// kernel boundary is the barrier.
struct NoMapLds {};

// The map merge of the persistent kernel, kept out of line (its registers
// then do not add to the epoch code's, and the kernel stays small enough for
// the compiler to inline the chunk); the arguments are plain pointers so that
// the call needs no copy of the kernel arguments in private memory.
template <int WG>
__device__ __noinline__ void map_merge_call(const uint32_t *part_job, const int64_t *part_ia, const uint64_t *mj_off,
                                            const int32_t *mj_lo, const int32_t *mj_hi,
                                            const uint32_t *const *mj_src, uint32_t *const *mj_dst,
                                            MapLds<kMapTile> &M, uint32_t J, uint64_t U) {
  const MapView v{part_job, part_ia, mj_off, mj_lo, mj_hi, mj_src, mj_dst};
  map_merge<WG, kMapTile, false>(v, M, J, U);   // (the lean form: fewer registers)
}

template <int WG, uint32_t OPS>
__global__ __launch_bounds__(WG) void k_epochs(DevCtx C, int32_t persistent) {
  constexpr bool kMap = (OPS & opbit(OP_MERGE)) != 0;
  // programs without the co-operative expansion or merge sort can sweep one
  // chunk per wavefront (chosen per epoch, see below); the others sweep one
  // chunk per work-group (their leaf sorts and merges want the registers)
  constexpr bool kWave = (OPS & (OPS_EXPAND | OPS_MS)) == 0;
  // (256-lane work-groups sweep by wavefronts only: their work-group sweep
  // holds four items per lane and would spill)
  constexpr bool kGroupSweep = !kWave || WG >= 512;
  constexpr int NSL = kGroupSweep ? kChunk : 1;   // segments the work-group's LDS caches
  using MapL = typename std::conditional<kMap, MapLds<kMapTile>, NoMapLds>::type;
  using VL = typename std::conditional<(OPS & OPS_EXPAND) != 0, VisitLds, NoVisitLds>::type;
  using WLT = typename std::conditional<kWave, WaveLds, NoWaveLds>::type;
  __shared__ Lds<WG, NSL> L;
  __shared__ MapL M;
  __shared__ VL V;
  __shared__ WLT WLs[kWave ? WG / 64 : 1];
  __shared__ uint32_t s_hdr[8];
  // Narrow epochs run in one work-group: the last arriver at an epoch's
  // barrier that finds the next epoch small (at most kSolo items; for a
  // wavefront sweep one step of 256 items a wavefront) and free of merges,
  // buffer initialisation and arc expansion runs it alone while the rest of
  // the grid waits at the barrier (persistent) or has ended (graph), then the
  // next one, and opens the barrier when an epoch needs the grid again.  Such
  // an epoch costs one work-group's round trips instead of a grid barrier's.
  constexpr uint32_t kSolo = (OPS & OPS_EXPAND) != 0 ? 0u
                             : (OPS & OPS_MS) != 0 ? 2u * (uint32_t)kChunk : (uint32_t)WG * 4u;
  bool solo = false;   // (uniform in the work-group)
  lds_init(C, L);
  if (threadIdx.x == 0) L.tflag = 0;
  if (threadIdx.x < 8) L.prof[threadIdx.x] = 0;
  if (threadIdx.x == 0) L.tprof = realtime();
  SchedHdr *H = C.hdr;
  const PlainArgs P{};
  while (true) {
    if (threadIdx.x == 0) {
      if (solo) {   // (the header this work-group's last scan wrote)
        s_hdr[0] = L.hdr[0]; s_hdr[1] = L.hdr[1]; s_hdr[2] = L.hdr[2]; s_hdr[3] = L.hdr[3];
        s_hdr[5] = L.hdr[4]; s_hdr[6] = L.hdr[5];
      } else {
        s_hdr[0] = H->S; s_hdr[1] = (uint32_t)H->L; s_hdr[2] = (uint32_t)H->stop; s_hdr[3] = H->mapJ;
        s_hdr[5] = (uint32_t)H->initN;
        s_hdr[6] = (uint32_t)H->wsel;
      }
    }
    __syncthreads();
    const uint32_t S = s_hdr[0];
    const int32_t nL = (int32_t)s_hdr[1];
    const uint32_t wo = s_hdr[6] * (uint32_t)(C.tmax + 1);   // the current work-list buffer
    const bool stop = s_hdr[2] != 0;
    const uint32_t mapJ = persistent ? s_hdr[3] : 0u;
    // trees adopted by an asynchronous run's last scan: their buffers are
    // initialised by every work-group before their roots run (also when the
    // run stops here: they stay live for the next run)
    const int32_t initN = persistent ? (int32_t)s_hdr[5] : 0;
    if (initN > 0) run_inits(C, initN);
    if constexpr (kMap) {
      if (mapJ) {   // merges registered by the previous epoch: partition, barrier, merge
        uint32_t J;
        uint64_t U;
        map_extent<kMapTile>(C, mapJ, &J, &U);
        map_partition<kMapTile>(C, J, U, (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6),
                      (int64_t)gridDim.x * (WG / 64));
        if (!grid_barrier<WG, NSL>(C, L, false, true)) break;
        map_merge_call<WG>(C.part_job, C.part_ia, C.mj_off, C.mj_lo, C.mj_hi, C.mj_src, C.mj_dst, M, J, U);
      }
    }
    if (stop) break;
    if ((mapJ || initN > 0) && !grid_barrier<WG, NSL>(C, L, false, true)) break;
    // asynchronous run: trees that finished in the epoch whose merges just
    // ran are complete now
    if (C.async_mode && mapJ && blockIdx.x == 0 && threadIdx.x == 0) publish_completions(C);
    // Chunks go to work-groups in runs of consecutive chunks; within a run
    // each chunk continues where the previous one ended.  Kernels with BFS
    // (whose chunks differ in cost by orders of magnitude) claim runs from a
    // shared counter, guided: a run is about a quarter of an even share, so
    // a work-group that drew expensive chunks takes fewer.  The others take
    // one even share each.
    // The wavefront sweep takes one allocation and one retirement atomic per
    // wavefront and tree; when many wavefronts share a tree, those atomics
    // on the tree's counters serialize, and the work-group sweep (one per
    // 1024 items) is faster.  So: wavefronts while the wavefronts that get
    // work number at most four per live tree, work-groups otherwise.
    // (a wavefront's share: an even split of the items, at least 64)
    // (a work-group that runs the epoch alone is the only part)
    const uint32_t nparts = solo ? 1u : gridDim.x, part = solo ? 0u : blockIdx.x;
    const uint32_t nw = nparts * (WG / 64);
    const uint32_t share = max(64u, (S + nw - 1) / nw);
    bool wave_sweep = false;
    if constexpr (kWave) wave_sweep = !kGroupSweep || (S + share - 1) / share <= 4u * (uint32_t)nL;
    if (wave_sweep) {
      if constexpr (kWave) {
        // consecutive wavefronts take consecutive shares
        const uint32_t wid = part * (WG / 64) + (threadIdx.x >> 6);
        WaveLds &W = WLs[threadIdx.x >> 6];
        if (lane_id() == 0) W.kfirst = -1;   // (a new work list every epoch)
        wave_sync();
        const uint64_t w0 = (uint64_t)wid * share, w1 = w0 + share < S ? w0 + share : S;
        if (w0 < S) run_wave<OPS, 2, 4>(C, W, L.op_tab, (uint32_t)w0, (uint32_t)w1, nL, wo);
      }
    } else if constexpr (kGroupSweep) {
      const uint32_t nchunks = (S + kChunk - 1) / kChunk;
      constexpr bool kGuided = (OPS & OPS_EXPAND) != 0;
      const uint32_t run = kGuided ? max(1u, nchunks / (4u * gridDim.x)) : (nchunks + nparts - 1) / nparts;
      PendingFinish pend;
      Prefetch<kChunk / WG> pf;
      for (uint32_t turn = 0;; ++turn) {
        uint32_t c0;
        if (kGuided) {
          if (threadIdx.x == 0) s_hdr[4] = add_agent(&H->chunk_ctr, run);
          __syncthreads();
          c0 = s_hdr[4];
          __syncthreads();
        } else {
          c0 = turn == 0 ? part * run : nchunks;
        }
        if (c0 >= nchunks) break;
        const uint32_t c1 = min(c0 + run, nchunks);
        pf.w0 = 0xFFFFFFFFu;
        for (uint32_t c = c0; c < c1; ++c)
          run_chunk<WG, OPS, true>(C, L, V, c * kChunk, S, nL, P, pend, pf, c1 * kChunk, c != c0, wo);
      }
      settle(C, pend);
    }
    phase_mark(C, L, 6);
    bool ok = true;
    if (solo) {
      // this work-group ran the epoch alone: the next work list, then the
      // next epoch alone too, or the barrier opened for the grid
      wait_vmem();
      __syncthreads();
      schedule_scan_ext<WG, NSL>(C.self, &L, 1);
      solo_decide<kSolo>(C, L);
      solo = L.flag2 != 0;
      if (!solo) barrier_release<WG, NSL>(C, L);
    } else {
      const int r = grid_barrier<WG, NSL, kSolo>(C, L, true, persistent != 0);
      ok = r != 0;
      solo = r == 2;
    }
    if constexpr ((OPS & OPS_EXPAND) != 0) {
      if (persistent && ok) {
        if (threadIdx.x == 0) s_hdr[4] = (uint32_t)H->arc_phase;
        __syncthreads();
        const bool arcs = s_hdr[4] != 0;
        __syncthreads();
        if (arcs) {
          arc_phase<WG, OPS>(C, L, V);
          ok = grid_barrier<WG, kChunk>(C, L, true, true);
        }
      }
    }
    phase_mark(C, L, 7);
    if (!ok || (!persistent && !solo)) break;
  }
  if (C.debug && threadIdx.x == 0)
    for (int ph = 0; ph < 8; ++ph) add_agent(&H->phase[ph], (uint64_t)L.prof[ph]);
}

// The arc phase of a captured chain: launched after each epoch launch of a
// kernel with BFS, SSSP or FFT; returns at once unless the epoch published arc jobs.  The
// last work-group to finish builds the next work list (the epoch launch left
// it for this launch).
template <int WG, uint32_t OPS>
__global__ __launch_bounds__(WG) void k_arcs(DevCtx C) {
  __shared__ Lds<WG> L;
  __shared__ VisitLds V;
  __shared__ int32_t s_phase;
  SchedHdr *H = C.hdr;
  if (threadIdx.x == 0) s_phase = H->arc_phase;
  __syncthreads();
  if (!s_phase) return;
  lds_init<WG>(C, L);
  arc_phase<WG, OPS>(C, L, V);
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) {
    fence_release();
    L.flag = (add_agent(&H->arc_arrive, 1u) == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (L.flag) {
    if (threadIdx.x == 0) { fence_acquire(); st_agent(&H->arc_arrive, 0u); }
    __syncthreads();
    schedule_scan_ext<WG, kChunk>(C.self, &L, 1);
  }
}

// Builds the first work list of a run from the trees' current ranges.
template <int WG>
__global__ __launch_bounds__(WG) void k_scan(DevCtx C) {
  __shared__ Lds<WG> L;
  if (threadIdx.x < 8) C.hdr->grp[threadIdx.x].n = 0;
  if (threadIdx.x == 0) { C.hdr->arrive = 0; C.hdr->done_count = 0; C.hdr->stop_reason = 0; C.hdr->stamp0 = realtime(); }
  __syncthreads();
  schedule_scan<WG, kChunk>(C, L, false);
}

// Admission: make staged trees live (root in entry 0 of the arena, epoch 0).
__global__ void k_admit(DevCtx C, const Admit *adm, int32_t n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  admit_one(C, adm[j]);
}

// A graph program's per-vertex array before its first epoch: 0 at the
// source, `fill` elsewhere (BFS depth: -1; SSSP distance: the largest int32).
__global__ void k_depth_init(int32_t *depth, int32_t V, int32_t src, int32_t fill) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x)
    depth[v] = (v == src) ? 0 : fill;
}

// Release a slot: no range, status free.
__global__ void k_release(DevCtx C, int32_t slot) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    C.t_len[slot] = 0;
    C.st[slot].status = TS_FREE;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
#define TREES_FOR_OPS(M, WG)      \
  M(WG, OPS_FIB)                  \
  M(WG, OPS_NQ)                   \
  M(WG, OPS_FIB | OPS_NQ)         \
  M(WG, OPS_MS)                   \
  M(WG, OPS_FIB | OPS_MS)         \
  M(WG, OPS_GRAPH)                \
  M(WG, OPS_FFT)                  \
  M(WG, OPS_PO)                   \
  M(WG, OPS_ALL)

static uint32_t pick_ops(uint32_t need) {
  const uint32_t sets[] = {OPS_FIB, OPS_NQ, OPS_FIB | OPS_NQ, OPS_MS, OPS_FIB | OPS_MS, OPS_GRAPH, OPS_FFT, OPS_PO,
                          OPS_ALL};
  for (uint32_t s : sets)
    if ((need & ~s) == 0) return s;
  return OPS_ALL;
}

template <int WG>
static const void *plain_fn(uint32_t ops) {
#define M(W, O) if (ops == (O)) return (const void *)&k_plain<W, O>;
  TREES_FOR_OPS(M, WG)
#undef M
  return nullptr;
}
template <int WG>
static const void *epochs_fn(uint32_t ops) {
#define M(W, O) if (ops == (O)) return (const void *)&k_epochs<W, O>;
  TREES_FOR_OPS(M, WG)
#undef M
  return nullptr;
}

const void *kernel_plain(int wg, uint32_t need) {
  const uint32_t ops = pick_ops(need);
  switch (wg) {
    case 256: return plain_fn<256>(ops);
    case 512: return plain_fn<512>(ops);
    case 1024: return plain_fn<1024>(ops);
    default: return nullptr;
  }
}
const void *kernel_epochs(int wg, uint32_t need) {
  const uint32_t ops = pick_ops(need);
  switch (wg) {
    case 256: return epochs_fn<256>(ops);
    case 512: return epochs_fn<512>(ops);
    case 1024: return epochs_fn<1024>(ops);
    default: return nullptr;
  }
}

// One plain epoch and the publication of its counters.  ev0 / ev1 (may be
// null): HIP events that take the epoch kernel's start and end.
hipError_t launch_plain(const DevCtx &C, const PlainArgs &P, int wg, uint32_t need, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1) {
  const void *fn = kernel_plain(wg, need);
  if (!fn) return hipErrorInvalidValue;
  const uint32_t S = (uint32_t)(P.e - P.b);
  if (S == 0) return hipErrorInvalidValue;
  dim3 grid((S + kChunk - 1) / kChunk), block(wg);
  DevCtx c = C;
  PlainArgs p = P;
  p.nwg = grid.x;
  void *args[] = {&c, &p};
  return hipExtLaunchKernel(fn, grid, block, args, 0, s, ev0, ev1, 0);
}

hipError_t launch_epochs(const DevCtx &C, int wg, uint32_t need, int grid, int persistent, hipStream_t s) {
  const void *fn = kernel_epochs(wg, need);
  if (!fn) return hipErrorInvalidValue;
  DevCtx c = C;
  int32_t p = persistent;
  void *args[] = {&c, &p};
  if (persistent) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(wg), args, 0, s);
  return hipLaunchKernel(fn, dim3(grid), dim3(wg), args, 0, s);
}

// End of a captured chain of epochs: the header's first 64 bytes to the
// host-mapped mirror, then the chain's number, written after the rest has
// landed (one wavefront).
// M: device address of the host-mapped mirror.
__global__ __launch_bounds__(64) void k_publish_hdr(SchedHdr *H, HdrMirror *M) {
  const int lane = threadIdx.x;
  const uint32_t seq = ld_agent(&H->pub_seq) + 1u;
  if (lane < 16)
    __hip_atomic_store(&M->hdr[lane], ld_agent(&((const int32_t *)H)[lane]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  wait_vmem();
  if (lane == 0) {
    st_agent(&H->pub_seq, seq);
    __hip_atomic_store(&M->seq, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

hipError_t launch_publish_hdr(SchedHdr *hdr, HdrMirror *mirror_dev, hipStream_t s) {
  void *args[] = {&hdr, &mirror_dev};
  return hipLaunchKernel((const void *)&k_publish_hdr, dim3(1), dim3(64), args, 0, s);
}

hipError_t launch_arcs(const DevCtx &C, int wg, uint32_t need, int grid, hipStream_t s) {
  const void *fn = nullptr;
  switch (wg) {
    case 256: fn = (const void *)&k_arcs<256, OPS_EXPAND>; break;
    case 512: fn = (const void *)&k_arcs<512, OPS_EXPAND>; break;
    case 1024: fn = (const void *)&k_arcs<1024, OPS_EXPAND>; break;
    default: return hipErrorInvalidValue;
  }
  (void)need;
  DevCtx c = C;
  void *args[] = {&c};
  return hipLaunchKernel(fn, dim3(grid), dim3(wg), args, 0, s);
}

// Co-resident work-groups per CU of a batched epoch kernel: the runtime's
// occupancy figure, bounded by the kernel's own resource use (VGPRs in
// granules of 8 out of 512 per SIMD lane, at most 8 waves per SIMD; static
// LDS out of the CU's; SGPRs counted at a conservative 128 of the SIMD's
// 800, so that a kernel limited by SGPRs is never over-subscribed).  *scratch
// receives the kernel's private bytes per lane: a persistent grid of a
// kernel that uses scratch is sized more cautiously by the caller.
int coresident_blocks_per_cu(int wg, uint32_t need, int *scratch, int *own) {
  const void *fn = kernel_epochs(wg, need);
  if (!fn) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, wg, 0) != hipSuccess) return 0;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, fn) != hipSuccess) return 0;
  int dev = 0, lds_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
    return 0;
  const int waves = (wg + 63) / 64;
  const int per_simd = (waves + 3) / 4;                 // a work-group's waves spread over the 4 SIMDs
  const int vg = ((fa.numRegs > 0 ? fa.numRegs : 1) + 7) / 8 * 8;
  const int w_v = std::min(8, 512 / vg);
  const int w_s = 800 / 128;
  const int by_regs = std::min(w_v, w_s) / per_simd;
  const int lds = (int)((fa.sharedSizeBytes + 511) / 512 * 512);
  const int by_lds = lds > 0 ? lds_cu / lds : 1 << 20;
  const int by_waves = 32 / waves;
  const int mine = std::min(by_regs, std::min(by_lds, by_waves));
  if (scratch) *scratch = (int)fa.localSizeBytes;
  if (own) *own = mine;
  return std::min(nb, mine);
}

hipError_t launch_scan(const DevCtx &C, hipStream_t s) {
  DevCtx c = C;
  void *args[] = {&c};
  return hipLaunchKernel((const void *)&k_scan<256>, dim3(1), dim3(256), args, 0, s);
}

hipError_t launch_admit(const DevCtx &C, const void *adm, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  DevCtx c = C;
  const Admit *a = (const Admit *)adm;
  int32_t nn = n;
  void *args[] = {&c, &a, &nn};
  return hipLaunchKernel((const void *)&k_admit, dim3((n + 255) / 256), dim3(256), args, 0, s);
}

hipError_t launch_depth_init(int32_t *depth, int32_t V, int32_t src, int32_t fill, hipStream_t s) {
  int32_t v = V, sc = src, f = fill;
  void *args[] = {&depth, &v, &sc, &f};
  int blocks = (int)((V + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  return hipLaunchKernel((const void *)&k_depth_init, dim3(blocks), dim3(256), args, 0, s);
}

hipError_t launch_release(const DevCtx &C, int slot, hipStream_t s) {
  DevCtx c = C;
  int32_t sl = slot;
  void *args[] = {&c, &sl};
  return hipLaunchKernel((const void *)&k_release, dim3(1), dim3(64), args, 0, s);
}

size_t admit_record_size() { return sizeof(Admit); }

}  // namespace trees
