// libtrees host side: contexts, program registration, admission of task
// trees into task-vector arenas, and the three epoch schedulers.
#include "trees.h"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "trees_dev.h"

namespace trees {
hipError_t launch_plain(const DevCtx &C, const PlainArgs &P, int wg, uint32_t need, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_epochs(const DevCtx &C, int wg, uint32_t need, int grid, int persistent, hipStream_t s);
hipError_t launch_map(const DevCtx &C, int wg, uint32_t jobs, int from_hdr, int grid_part, int grid_merge,
                      hipStream_t s, const hipEvent_t *ev);
hipError_t launch_arcs(const DevCtx &C, int wg, uint32_t need, int grid, hipStream_t s);
hipError_t launch_publish_hdr(SchedHdr *hdr, HdrMirror *mirror_dev, hipStream_t s);
int coresident_blocks_per_cu(int wg, uint32_t need, int *scratch, int *own);
hipError_t launch_scan(const DevCtx &C, hipStream_t s);
hipError_t launch_admit(const DevCtx &C, const void *adm, int n, hipStream_t s);
hipError_t launch_depth_init(int32_t *depth, int32_t V, int32_t src, int32_t fill, hipStream_t s);
const void *kernel_epochs(int wg, uint32_t need);
hipError_t launch_wl(const WlArgs &a, int wg, bool sssp, hipStream_t s);
hipError_t launch_wl_init(int32_t *val, int32_t *stamp, int32_t V, int32_t src, int32_t fill, int32_t *in,
                          void *ctl, hipStream_t s);
hipError_t wl_scratch_setup(int device);
void *wl_scratch_ptr(int device);
}  // namespace trees

using namespace trees;

namespace {

constexpr int kBytesPerEntry = 28;   // code + a0..a3 (int32) + r (int64)
constexpr int kMapJobs = 1 << 20;    // map jobs per epoch; merges beyond it run serially
constexpr uint64_t kMapTileUnits = kMapLaunchTile;
constexpr int kPartCap = 1 << 20;    // tile boundaries: 2^32 merged keys per epoch
// Map grids of a captured chain, per CU (the job count is not known when the
// chain is captured; both passes loop over their work, and a pass with no
// jobs returns at once).
constexpr int kGraphPartPerCU = 2;
constexpr int kGraphMergePerCU = 4;

std::string g_create_error;

struct Prog {
  int kind = 0;
  int tbase = 0;
  int ntypes = 0;
  uint32_t ops = 0;
};

enum HostStatus { H_FREE = 0, H_STAGED = 1, H_LIVE = 2, H_DONE = 3 };

struct HostTree {
  int hstatus = H_FREE;
  uint32_t gen = 1;
  int prog = 0;
  int kind = 0;
  int64_t base = 0, cap = 0;
  uint64_t order = 0;              // submission order
  uint32_t tp = 0;                 // first type id | nqueens n << 8 (as the kernels cache it)
  TreeState st{};                  // mirror of the device state
};

uint32_t ops_of_kind(int kind) {
  switch (kind) {
    case TREES_PROG_FIB_I32: return opbit(OP_FIB32) | opbit(OP_SUM32);
    case TREES_PROG_FIB_I64: return opbit(OP_FIB64) | opbit(OP_SUM64);
    case TREES_PROG_MSORT_U32: return OPS_MS;
    case TREES_PROG_NQUEENS: return OPS_NQ;
    case TREES_PROG_BFS_CSR: return OPS_BFS;
    case TREES_PROG_POSTORDER: return OPS_PO;
    case TREES_PROG_PREORDER: return OPS_PO;
    case TREES_PROG_FFT: return OPS_FFT;
    case TREES_PROG_SSSP_CSR: return OPS_SSSP;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Exact task-vector bounds (admission sizes).  The task vector only shrinks
// when a join range is popped (nextFreeCore returns to the value saved with
// the range), so a tree's high-water mark is reached when its deepest level
// has been forked: every task of the forking type is then allocated.
// ---------------------------------------------------------------------------
int64_t fib_bound(int64_t n) {
  if (n < 2) return 1;
  int64_t a = 0, b = 1;   // F(n+1)
  for (int64_t k = 0; k < n + 1; ++k) { int64_t t = a + b; a = b; b = t; }
  return 2 * a - 1;       // nodes of the naive call tree
}

int64_t nq_nodes_rec(int n, int row, uint32_t cols, uint32_t ld, uint32_t rd) {
  if (row == n) return 1;
  const uint32_t full = (1u << n) - 1u;
  uint32_t avail = ~(cols | ld | rd) & full;
  int64_t s = 1;
  while (avail) {
    uint32_t bit = avail & (0u - avail);
    avail ^= bit;
    s += nq_nodes_rec(n, row + 1, cols | bit, ((ld | bit) << 1) & full, (rd | bit) >> 1);
  }
  return s;
}
int64_t nq_bound(int n) {
  static std::mutex mu;
  static int64_t memo[16] = {0};
  std::lock_guard<std::mutex> g(mu);
  if (!memo[n]) memo[n] = nq_nodes_rec(n, 0, 0, 0, 0);
  return memo[n];
}

int64_t ms_bound(int64_t n) {
  // MS tasks of the split tree: 1 + bound(floor(n/2)) + bound(ceil(n/2))
  static std::mutex mu;
  static std::map<int64_t, int64_t> memo;
  if (n <= kLeaf) return 1;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = memo.find(n);
    if (it != memo.end()) return it->second;
  }
  int64_t v = 1 + ms_bound(n / 2) + ms_bound(n - n / 2);
  std::lock_guard<std::mutex> g(mu);
  memo[n] = v;
  return v;
}

trees_status tv_bound(int kind, const int64_t *args, int nargs, int64_t *out, std::string *err) {
  auto bad = [&](const char *m) { if (err) *err = m; return (trees_status)TREES_E_INVALID; };
  switch (kind) {
    case TREES_PROG_FIB_I32:
    case TREES_PROG_FIB_I64:
      if (nargs < 1 || args[0] < 0 || args[0] > 43) return bad("fib: need 0 <= n <= 43");
      *out = fib_bound(args[0]);
      return TREES_OK;
    case TREES_PROG_NQUEENS:
      if (nargs < 1 || args[0] < 1 || args[0] > 14) return bad("nqueens: need 1 <= n <= 14");
      *out = nq_bound((int)args[0]);
      return TREES_OK;
    case TREES_PROG_MSORT_U32:
      if (nargs < 1 || args[0] < 0 || args[0] >= (1ll << 31)) return bad("msort: need 0 <= N < 2^31");
      *out = ms_bound(args[0]);
      return TREES_OK;
    case TREES_PROG_BFS_CSR:
      if (nargs < 2 || args[0] < 1 || args[0] >= (1ll << 31) || args[1] < 0 || args[1] >= args[0])
        return bad("bfs: need V >= 1 and 0 <= source < V");
      *out = args[0];
      return TREES_OK;
    case TREES_PROG_SSSP_CSR:
      // a vertex is visited once per improvement of its distance, so the
      // task count depends on the schedule: the arena holds max_entries
      // (default 8 V) and a run that needs more fails with OVERFLOW
      if (nargs < 2 || args[0] < 1 || args[0] >= (1ll << 31) || args[1] < 0 || args[1] >= args[0])
        return bad("sssp: need V >= 1 and 0 <= source < V");
      if (nargs >= 3 && (args[2] < 0 || args[2] >= (1ll << 31)))
        return bad("sssp: need 0 <= max_entries < 2^31 (0: the default)");
      if (nargs >= 4 && (args[3] < 0 || args[3] >= (1ll << 24))) return bad("sssp: need 0 <= delta < 2^24");
      *out = (nargs >= 3 && args[2] > 0) ? args[2] : std::min<int64_t>(8 * args[0], (1ll << 31) - 1);
      return TREES_OK;
    case TREES_PROG_FFT: {
      // the binary tree of FFT tasks down to 64-point leaves: its nodes
      // (a combine reuses its own entry)
      if (nargs < 1 || args[0] < 0 || args[0] > kFftMaxLog)
        return bad("fft: need 0 <= log2 N <= 20");
      const int64_t leaves = args[0] > kFftLeafLog ? (1ll << (args[0] - kFftLeafLog)) : 1;
      *out = 2 * leaves - 1;
      return TREES_OK;
    }
    case TREES_PROG_POSTORDER:
    case TREES_PROG_PREORDER:
      // every traversal task (the root and two per node, null children
      // included) holds one entry; a postorder join reuses its own
      if (nargs < 2 || args[0] < 1 || args[0] >= (1ll << 24) || args[1] < -1 || args[1] >= args[0])
        return bad("traversal: need 1 <= n < 2^24 and -1 <= root < n");
      *out = 2 * args[0] + 1;
      return TREES_OK;
  }
  return bad("unknown program kind");
}

}  // namespace

struct trees_ctx {
  trees_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char *arena = nullptr;
  bool own_arena = false;
  int64_t nent = 0;
  void *ctl = nullptr;             // control block (descriptors, stacks, work list, header)
  DevCtx dc{};
  std::vector<Prog> progs;
  int ntt = 0;
  bool frozen = false;
  int tmax = 4096;
  std::vector<HostTree> trees;
  int tslots = 0;
  int ntrees = 0;
  uint64_t order = 0;
  std::map<int64_t, int64_t> freel;   // arena free list: start -> length
  int64_t free_ent = 0;
  std::vector<Admit> staged;
  struct DepthInit { int32_t *depth; int32_t V, src, fill; };
  std::vector<DepthInit> depth_inits;
  Admit *adm_host = nullptr;       // pinned staging
  Admit *adm_dev = nullptr;
  PlainMirror *mirror = nullptr;   // host-mapped, written after each plain epoch
  HdrMirror *hmirror = nullptr;    // host-mapped, written after each captured chain
  HdrMirror *hmirror_dev = nullptr;
  uint32_t hseq = 0;               // captured chains launched (HdrMirror::seq of the last)
  uint32_t plain_seq = 0;
  DevCtx *self_dev = nullptr;      // device copies of dc (out-of-line device code reads them)
  DevCtx *self_host = nullptr;     // pinned staging for them
  WlMirror *wl_mirror = nullptr;   // host-mapped, written after each worklist iteration
  WlMirror *wl_mirror_dev = nullptr;
  uint32_t wl_seq = 0;
  SchedHdr *hdr_host = nullptr;
  TreeState *st_host = nullptr;
  int32_t *abort_flag = nullptr;
  int64_t *r_host = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int gkey_wg = 0, gkey_grid = 0, gkey_chunk = 0;
  uint32_t gkey_ops = 0;
  int sched = TREES_SCHED_PERSISTENT;
  int wg = 256, bpc = 0, chunk = 8;
  std::string devname;              // hipDeviceProp_t::name (the tuned file's device key)
  bool tuned_done = false;          // AUTO: the tuned file has been consulted
  bool tuned_ok = false;            // ... and held a shape for this device and workload class
  trees_shape tuned{};
  int ncu = 0;
  int last_grid = 0, last_api_bpc = 0, last_wg = 0, last_scratch = 0;
  bool profile = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // plain-scheduler launch timing: event pairs resolved after the tree's
  // last epoch, so timing adds no synchronisation per epoch
  std::vector<hipEvent_t> evpool;
  std::vector<std::pair<int, size_t>> evpend;   // (ktime slot, first event of the pair)
  trees_ktime ktime[11] = {};  // 1..5 plain epochs per kind, 0 batched, 6/7 map passes, 8/9/10 plain traversal/sssp/fft
  uint32_t prof_mask = 0x7FFu;  // which of the slots above are timed
  double clock_hz = 1e8;
  double timeout_s = 60.0;   // host and device waits give up after this long
  bool running = false;
  // asynchronous runs (TREES_RUN_ASYNC)
  bool async_on = false;           // an asynchronous run is in flight
  AsyncRing *ring = nullptr;       // host-mapped: ring header
  Admit *ring_adm = nullptr;       // host-mapped: admission records [tmax]
  Completion *ring_done = nullptr; // host-mapped: completion records [tmax]
  uint32_t ring_tail = 0;          // admission records published in this run
  uint32_t chead = 0;              // completion records consumed in this run
  uint64_t async_tasks = 0;        // tasks of the trees finished in this run
  std::chrono::steady_clock::time_point async_t0;
  std::deque<uint64_t> finished;   // finished trees not yet reported by trees_poll
  std::string err;
  std::mutex mu;
};

namespace {

trees_status fail(trees_ctx *c, trees_status st, const std::string &m) {
  if (c) c->err = m; else g_create_error = m;
  return st;
}

#define HIPCHK(ctx, call)                                                             \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, TREES_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TRY(call)                         \
  do {                                    \
    const trees_status s_ = (call);       \
    if (s_ != TREES_OK) return s_;        \
  } while (0)

// Arenas start on 64-entry boundaries (work lists keep base / 64 in 32 bits).
int64_t arena_alloc(trees_ctx *c, int64_t n) {
  n = (n + 63) & ~(int64_t)63;
  for (auto it = c->freel.begin(); it != c->freel.end(); ++it) {
    if (it->second >= n) {
      int64_t s = it->first, len = it->second;
      c->freel.erase(it);
      if (len > n) c->freel[s + n] = len - n;
      c->free_ent -= n;
      return s;
    }
  }
  return -1;
}

void arena_free(trees_ctx *c, int64_t s, int64_t n) {
  n = (n + 63) & ~(int64_t)63;
  if (n <= 0) return;
  c->free_ent += n;
  auto it = c->freel.emplace(s, n).first;
  auto nx = std::next(it);
  if (nx != c->freel.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    c->freel.erase(nx);
  }
  if (it != c->freel.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      c->freel.erase(it);
    }
  }
}

uint32_t ops_needed(trees_ctx *c) {
  uint32_t o = 0;
  for (auto &p : c->progs) o |= p.ops;
  return o;
}

uint64_t tree_id(const trees_ctx *c, int slot) { return ((uint64_t)c->trees[slot].gen << 32) | (uint32_t)slot; }

// Stage a submission for the next trees_run, with the initialisation of the
// program's per-vertex or log buffer that precedes the tree's first epoch.
void stage(trees_ctx *c, const Admit &a) {
  c->staged.push_back(a);
  const TreeStatic &ts = a.ts;
  switch (ts.kind) {
    case TREES_PROG_BFS_CSR: c->depth_inits.push_back({(int32_t *)ts.ptr2, ts.p0, ts.p1, -1}); break;
    case TREES_PROG_SSSP_CSR: c->depth_inits.push_back({(int32_t *)ts.ptr2, ts.p0, ts.p1, INT32_MAX}); break;
    // a traversal's visit counter (log[n]) starts at zero: cleared inside
    // trees_run, on the context's stream, after the caller's own work on it
    case TREES_PROG_POSTORDER:
    case TREES_PROG_PREORDER: c->depth_inits.push_back({(int32_t *)ts.ptr2 + ts.p0, 1, -1, 0}); break;
  }
}

// Mark a tree finished (its state mirror filled) and queue it for trees_poll.
void mark_done(trees_ctx *c, int slot) {
  c->trees[slot].hstatus = H_DONE;
  c->finished.push_back(tree_id(c, slot));
  if (c->finished.size() > 2 * (size_t)c->tmax) {   // a caller that never polls: drop released ids
    std::deque<uint64_t> keep;
    for (uint64_t id : c->finished) {
      const int s = (int)(uint32_t)id;
      const HostTree &t = c->trees[s];
      if (t.hstatus == H_DONE && t.gen == (uint32_t)(id >> 32)) keep.push_back(id);
    }
    c->finished.swap(keep);
  }
}

// Consume the completion records an asynchronous run has published.
void drain_completions(trees_ctx *c) {
  const uint32_t ct = __atomic_load_n(&c->ring->ctail, __ATOMIC_ACQUIRE);
  while (c->chead != ct) {
    const Completion q = c->ring_done[c->chead % (uint32_t)c->tmax];
    ++c->chead;
    if (q.slot < 0 || q.slot >= c->tmax) continue;
    HostTree &t = c->trees[q.slot];
    if (t.hstatus != H_LIVE) continue;
    t.st.status = TS_DONE;
    t.st.err = q.err;
    t.st.epochs = q.epochs;
    t.st.peak = q.peak;
    t.st.tasks = q.tasks;
    t.st.launched = q.launched;
    t.st.result = q.result;
    t.st.start_gepoch = q.start_gepoch;
    t.st.done_gepoch = q.done_gepoch;
    if (q.err == 0) c->async_tasks += (uint64_t)q.tasks;
    mark_done(c, q.slot);
  }
}

trees_status flush_admissions(trees_ctx *c) {
  const int n = (int)c->staged.size();
  if (n) {
    memcpy(c->adm_host, c->staged.data(), sizeof(Admit) * n);
    HIPCHK(c, hipMemcpyAsync(c->adm_dev, c->adm_host, sizeof(Admit) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_admit(c->dc, c->adm_dev, n, c->stream));
    for (auto &a : c->staged) {
      HostTree &t = c->trees[a.slot];
      t.hstatus = H_LIVE;
      memset(&t.st, 0, sizeof(t.st));
      t.st.e = 1; t.st.old = 1; t.st.status = TS_LIVE; t.st.tasks = 0; t.st.peak = 1;
      t.st.done_gepoch = -1; t.st.start_gepoch = -1;
    }
    c->staged.clear();
  }
  for (auto &d : c->depth_inits) HIPCHK(c, launch_depth_init(d.depth, d.V, d.src, d.fill, c->stream));
  c->depth_inits.clear();
  // the admission staging buffer is reused: wait for the copy
  if (n) HIPCHK(c, hipStreamSynchronize(c->stream));
  return TREES_OK;
}

// Read the device state of every slot back into the host mirrors.
trees_status sync_states(trees_ctx *c) {
  if (c->tslots == 0) return TREES_OK;
  HIPCHK(c, hipMemcpyAsync(c->st_host, c->dc.st, sizeof(TreeState) * c->tslots, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int s = 0; s < c->tslots; ++s) {
    HostTree &t = c->trees[s];
    if (t.hstatus != H_LIVE) continue;
    t.st = c->st_host[s];
    if (t.st.status == TS_DONE) {
      mark_done(c, s);
      if (t.st.err == 0) c->async_tasks += (uint64_t)t.st.tasks;   // (counted only for asynchronous runs)
    }
  }
  return TREES_OK;
}

// Whether launches of ktime slot `slot` are timed.
bool timed(const trees_ctx *c, int slot) { return c->profile && ((c->prof_mask >> slot) & 1u); }

// Two timing events for a launch whose duration accumulates in ktime[slot].
trees_status take_events(trees_ctx *c, int slot, hipEvent_t *e0, hipEvent_t *e1) {
  const size_t i = c->evpend.size() * 2;
  while (c->evpool.size() < i + 2) {
    hipEvent_t e = nullptr;
    HIPCHK(c, hipEventCreate(&e));
    c->evpool.push_back(e);
  }
  c->evpend.emplace_back(slot, i);
  *e0 = c->evpool[i];
  *e1 = c->evpool[i + 1];
  return TREES_OK;
}

// After the stream has drained: add up the pending launch durations.
trees_status resolve_events(trees_ctx *c) {
  for (const auto &p : c->evpend) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->evpool[p.second], c->evpool[p.second + 1]));
    c->ktime[p.first].ms += ms;
    c->ktime[p.first].launches += 1;
  }
  c->evpend.clear();
  return TREES_OK;
}

// Wait until the plain epoch launch `seq` has published its counters in the
// mirror.  Polls host memory; checks the stream for errors now and then.
trees_status wait_seq(trees_ctx *c, const uint32_t *seqp, uint32_t seq) {
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 1;; ++spin) {
    if (__atomic_load_n(seqp, __ATOMIC_ACQUIRE) == seq) return TREES_OK;
    if ((spin & 1023) == 0) {
      const hipError_t q = hipStreamQuery(c->stream);
      if (q == hipSuccess) {
        if (__atomic_load_n(seqp, __ATOMIC_ACQUIRE) == seq) return TREES_OK;
        return fail(c, TREES_E_DEVICE, "epoch launch ended without publishing its counters");
      }
      if (q != hipErrorNotReady) return fail(c, TREES_E_DEVICE, std::string("epoch launch: ") + hipGetErrorString(q));
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el > c->timeout_s) return fail(c, TREES_E_DEVICE, "epoch launch did not finish within the time limit");
    }
    __builtin_ia32_pause();
  }
}
trees_status wait_mirror(trees_ctx *c, uint32_t seq) { return wait_seq(c, &c->mirror->seq, seq); }

// ---------------------------------------------------------------------------
// PLAIN: the paper's host-driven loop, one tree at a time.
// ---------------------------------------------------------------------------
trees_status run_plain_tree(trees_ctx *c, int slot, int64_t *budget, uint64_t *gepochs, bool trace) {
  HostTree &t = c->trees[slot];
  TreeState st{};
  HIPCHK(c, hipMemcpyAsync(c->st_host, c->dc.st + slot, sizeof(TreeState), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  st = c->st_host[0];
  std::vector<int4> stk(st.sp);
  if (st.sp)
    HIPCHK(c, hipMemcpy(stk.data(), c->dc.stack + (size_t)slot * kStackMax, sizeof(int4) * st.sp,
                        hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemsetAsync(c->dc.plain, 0, sizeof(PlainCounters), c->stream));
  // this run's trace records, appended to the tree's device trace at the end
  // (a tree may run some epochs batched and others plain)
  std::vector<TraceRec> recs;
  const uint32_t need = c->progs[t.prog].ops;
  int par = 0;
  int err = 0;
  bool done = false;
  while (true) {
    if (*budget == 0 || *(volatile int32_t *)c->abort_flag) break;
    // Phase 1 happened when the range was popped; launch Phase 2.
    PlainArgs P{slot, st.cen, st.b, st.e, st.old, par, 0, (uint32_t)(t.base >> 6), t.tp, 0u /* nwg: the launcher's */};
    if (st.start_gepoch < 0) st.start_gepoch = (int64_t)*gepochs;
    P.seq = ++c->plain_seq ? c->plain_seq : ++c->plain_seq;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    // (6 and 7 are the map passes)
    const int kslot = (t.kind == TREES_PROG_POSTORDER || t.kind == TREES_PROG_PREORDER) ? 8
                      : t.kind == TREES_PROG_SSSP_CSR ? 9 : t.kind == TREES_PROG_FFT ? 10 : t.kind;
    if (timed(c, kslot)) TRY(take_events(c, kslot, &e0, &e1));
    HIPCHK(c, launch_plain(c->dc, P, c->wg, need, c->stream, e0, e1));
    TRY(wait_mirror(c, P.seq));
    const PlainMirror mir = *c->mirror;
    const int32_t forks = (int32_t)(uint32_t)mir.fj;
    const int32_t joins = (int32_t)(mir.fj >> 32);
    const int32_t valid = mir.valid;
    const int32_t flags = mir.flags;
    const uint64_t mc = mir.map;
    const int32_t nfc = st.old + forks;
    if (mc >> kMapShift) {
      // map phase: the merges registered by this epoch, before the next one
      const uint64_t units = mc & kMapUnitMask;
      const uint64_t tiles = (units + kMapTileUnits - 1) / kMapTileUnits;
      const uint64_t cap = (uint64_t)c->ncu * 16;
      const int gm = (int)std::max<uint64_t>(1, std::min<uint64_t>(tiles, (uint64_t)c->ncu * kMapBlocksPerCU));
      int gp = (int)std::max<uint64_t>(1, std::min<uint64_t>((tiles + 1 + kMapWG / 64 - 1) / (kMapWG / 64), cap));
      gp = (gp + 7) & ~7;   // a multiple of the XCD count (the partition pass maps blocks to XCDs)
      hipEvent_t ev[4] = {};
      if (timed(c, 6)) TRY(take_events(c, 6, &ev[0], &ev[1]));
      if (timed(c, 7)) TRY(take_events(c, 7, &ev[2], &ev[3]));
      HIPCHK(c, launch_map(c->dc, kMapWG, (uint32_t)(mc >> kMapShift), 0, gp, gm, c->stream,
                           ev));
    }
    if (trace && st.ntrace + (int)recs.size() < kTraceMax)
      recs.push_back(TraceRec{st.epochs, st.cen, st.b, st.e, st.e - st.b, valid, forks, joins, nfc});
    st.epochs += 1;
    st.launched += st.e - st.b;
    st.tasks += valid;   // tasks executed in this epoch
    if (nfc > st.peak) st.peak = nfc;
    ++*gepochs;
    if (*budget > 0) --*budget;
    par ^= 1;
    if (flags & TF_OVERFLOW) { err = TREES_E_OVERFLOW; done = true; break; }
    if (flags & TF_ENCODING) { err = TREES_E_ENCODING; done = true; break; }
    // Phase 3 (Section 5.2.4): push the join range, then the forked range.
    int4 top;
    bool have = false;
    if (joins) {
      if ((int)stk.size() >= kStackMax) { err = TREES_E_STACK; done = true; break; }
      stk.push_back(make_int4(st.cen, st.b, st.e, nfc));
    }
    if (forks) { top = make_int4(st.cen + 1, st.old, nfc, nfc); have = true; }
    else if (!stk.empty()) { top = stk.back(); stk.pop_back(); have = true; }
    if (!have) { done = true; break; }
    st.cen = top.x; st.b = top.y; st.e = top.z; st.old = top.w;
  }
  st.sp = (int)stk.size();
  if (done) {
    st.status = TS_DONE;
    st.err = err;
    st.done_gepoch = (int64_t)*gepochs - 1;
    if (!err) {
      HIPCHK(c, hipMemcpy(c->r_host, c->dc.r + t.base, sizeof(int64_t), hipMemcpyDeviceToHost));
      st.result = c->r_host[0];
    }
  }
  if (!recs.empty()) {
    HIPCHK(c, hipMemcpyAsync(c->dc.trace + (size_t)slot * kTraceMax + st.ntrace, recs.data(),
                             sizeof(TraceRec) * recs.size(), hipMemcpyHostToDevice, c->stream));
    st.ntrace += (int32_t)recs.size();
  }
  // Write the state back so any scheduler can continue a paused tree.
  c->st_host[0] = st;
  HIPCHK(c, hipMemcpyAsync(c->dc.st + slot, c->st_host, sizeof(TreeState), hipMemcpyHostToDevice, c->stream));
  if (st.sp)
    HIPCHK(c, hipMemcpyAsync(c->dc.stack + (size_t)slot * kStackMax, stk.data(), sizeof(int4) * st.sp,
                             hipMemcpyHostToDevice, c->stream));
  TreeHot hot{};
  hot.nfc = st.old;
  HIPCHK(c, hipMemcpyAsync(c->dc.hot + slot, &hot, sizeof(TreeHot), hipMemcpyHostToDevice, c->stream));
  int32_t lcb[3] = {done ? 0 : st.e - st.b, st.cen, st.b};
  HIPCHK(c, hipMemcpyAsync(c->dc.t_len + slot, &lcb[0], 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->dc.t_cen + slot, &lcb[1], 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->dc.t_b + slot, &lcb[2], 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  TRY(resolve_events(c));
  t.st = st;
  if (done) mark_done(c, slot);
  return TREES_OK;
}

// ---------------------------------------------------------------------------
// GRAPH / PERSISTENT: device Phases 1 and 3.
// ---------------------------------------------------------------------------
trees_status hdr_begin(trees_ctx *c, int64_t max_epochs, bool async = false) {
  // read-modify-write of the header's scalar part
  HIPCHK(c, hipMemcpyAsync(c->hdr_host, c->dc.hdr, sizeof(SchedHdr), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->hdr_host->stop = 0;
  c->hdr_host->stop_reason = 0;
  c->hdr_host->run_epochs = 0;
  c->hdr_host->max_epochs = max_epochs;
  c->hdr_host->tslots = c->tslots;
  c->hdr_host->arrive = 0;
  for (int g = 0; g < 8; ++g) c->hdr_host->grp[g].n = 0;
  c->hdr_host->wsel = 0;
  c->hdr_host->wl_next = 0;
  c->hdr_host->mapJ = 0;
  c->hdr_host->map_ctr = 0;
  c->hdr_host->map_arrive = 0;
  c->hdr_host->chunk_ctr = 0;
  c->hdr_host->arc_jobs = 0;
  c->hdr_host->arc_tiles = 0;
  c->hdr_host->arc_segs = 0;
  c->hdr_host->arc_next = 0;
  c->hdr_host->arc_arrive = 0;
  c->hdr_host->arc_phase = 0;
  c->hdr_host->initN = 0;
  c->hdr_host->adm_head = 0;
  c->hdr_host->ctail = 0;
  c->hdr_host->ctail_pub = 0;
  c->hdr_host->idle_t0 = 0;
  c->hdr_host->pub_seq = c->hseq;   // the next chain publishes hseq + 1
  HIPCHK(c, hipMemcpyAsync(c->dc.hdr, c->hdr_host, sizeof(SchedHdr), hipMemcpyHostToDevice, c->stream));
  // the context's device copies (out-of-line device code reads them): as it
  // stands now (programs registered since the last run included), and its
  // asynchronous-run form
  c->self_host[0] = c->dc;
  c->self_host[0].self = c->self_dev;
  c->self_host[1] = c->dc;
  c->self_host[1].async_mode = 1;
  c->self_host[1].self = c->self_dev + 1;
  HIPCHK(c, hipMemcpyAsync(c->self_dev, c->self_host, 2 * sizeof(DevCtx), hipMemcpyHostToDevice, c->stream));
  // (the first scan of an asynchronous run does not stop on an empty work
  // list: the run waits for submissions)
  DevCtx d = c->dc;
  d.async_mode = async ? 1 : 0;
  d.self = c->self_dev + (async ? 1 : 0);
  HIPCHK(c, launch_scan(d, c->stream));
  return TREES_OK;
}

trees_status read_hdr(trees_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->hdr_host, c->dc.hdr, 64, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TREES_OK;
}

// Work-groups per CU for the batched grids.  The persistent form needs every
// work-group resident at once: its grid is the co-resident count (the
// runtime's occupancy figure, bounded by the kernel's own VGPR, SGPR and LDS
// use).  A kernel that uses scratch (private memory) is held to 3/4 of it:
// scratch space is handed out per wave by the runtime and may admit fewer
// waves than the registers and LDS would.  The graph form has no residency
// requirement.
int blocks_per_cu(trees_ctx *c, uint32_t need, bool persistent) {
  int scratch = 0, own = 0;
  int api = coresident_blocks_per_cu(c->wg, need, &scratch, &own);
  if (api <= 0) api = 1;
  c->last_api_bpc = api;
  c->last_scratch = scratch;
  const int cap = (persistent && scratch > 0) ? std::max(1, (api * 3) / 4) : api;
  return (c->bpc > 0) ? std::min(c->bpc, cap) : cap;
}

int grid_size(trees_ctx *c, uint32_t need, bool persistent) {
  return blocks_per_cu(c, need, persistent) * c->ncu;
}

trees_status run_graph(trees_ctx *c, int64_t max_epochs) {
  trees_status s = hdr_begin(c, max_epochs);
  if (s) return s;
  const uint32_t need = ops_needed(c);
  const int grid = grid_size(c, need, false);
  c->last_grid = grid;
  if (!c->gexec || c->gkey_wg != c->wg || c->gkey_grid != grid || c->gkey_chunk != c->chunk ||
      c->gkey_ops != need) {
    if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < c->chunk; ++k) {
      hipError_t e = launch_epochs(c->dc, c->wg, need, grid, 0, c->stream);
      if (e == hipSuccess && (need & OPS_EXPAND)) e = launch_arcs(c->dc, c->wg, need, grid, c->stream);
      if (e == hipSuccess && c->dc.mj_cap > 0 && (need & OPS_MS))
        e = launch_map(c->dc, kMapWG, 0, 1, c->ncu * kGraphPartPerCU, c->ncu * kGraphMergePerCU, c->stream,
                       nullptr);
      if (e != hipSuccess) {
        hipGraph_t g;
        (void)hipStreamEndCapture(c->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        return fail(c, TREES_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
      }
    }
    {
      const hipError_t e = launch_publish_hdr(c->dc.hdr, c->hmirror_dev, c->stream);
      if (e != hipSuccess) {
        hipGraph_t g;
        (void)hipStreamEndCapture(c->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        return fail(c, TREES_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
      }
    }
    HIPCHK(c, hipStreamEndCapture(c->stream, &c->graph));
    HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    c->gkey_wg = c->wg; c->gkey_grid = grid; c->gkey_chunk = c->chunk; c->gkey_ops = need;
  }
  s = read_hdr(c);
  if (s) return s;
  while (!c->hdr_host->stop) {
    if (timed(c, 0)) HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    if (timed(c, 0)) HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    // the chain's last node publishes the header; poll for it
    s = wait_seq(c, &c->hmirror->seq, ++c->hseq);
    if (s) return s;
    for (int k = 0; k < 16; ++k)
      ((int32_t *)c->hdr_host)[k] = __atomic_load_n(&c->hmirror->hdr[k], __ATOMIC_RELAXED);
    if (timed(c, 0)) {
      float ms = 0;
      HIPCHK(c, hipEventSynchronize(c->ev1));
      HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
      c->ktime[0].ms += ms;
      c->ktime[0].launches += 1;
    }
  }
  return TREES_OK;
}

// Starts an asynchronous persistent run and returns while it runs: trees
// submitted meanwhile go through the admission ring, finished ones come back
// through the completion ring (Section 5.2.1's root placement happens on the
// device, at the epoch boundary after the submission).
trees_status start_async(trees_ctx *c, int64_t max_epochs) {
  c->ring->tail = 0;
  c->ring->head = 0;
  c->ring->ctail = 0;
  c->ring->close = 0;
  trees_status s = hdr_begin(c, max_epochs, true);
  if (s) return s;
  c->ring_tail = 0;
  c->chead = 0;
  c->async_tasks = 0;
  // every program's kernel code, since any may be submitted during the run
  uint32_t need = 0;
  for (auto &p : c->progs) need |= p.ops;
  if (!need) return fail(c, TREES_E_STATE, "asynchronous run: no program registered");
  const int grid = grid_size(c, need, true);
  c->last_grid = grid;
  DevCtx d = c->dc;
  d.async_mode = 1;
  d.self = c->self_dev + 1;
  HIPCHK(c, launch_epochs(d, c->wg, need, grid, 1, c->stream));
  c->async_on = true;
  c->async_t0 = std::chrono::steady_clock::now();
  return TREES_OK;
}

// After an asynchronous run's kernel has returned (or to make it return:
// close = it drains first): collect its completions and the state of the
// trees it left live; submissions it never adopted are staged for the next
// run.
trees_status finish_async(trees_ctx *c, bool close) {
  if (close) __atomic_store_n(&c->ring->close, 1, __ATOMIC_RELEASE);
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    const hipError_t q = hipStreamQuery(c->stream);
    if (q == hipSuccess) break;
    if (q != hipErrorNotReady) {
      c->async_on = false;
      return fail(c, TREES_E_DEVICE, std::string("asynchronous run: ") + hipGetErrorString(q));
    }
    drain_completions(c);
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (el > 2 * c->timeout_s + 10) {
      c->async_on = false;
      return fail(c, TREES_E_DEVICE, "asynchronous run did not end within the time limit");
    }
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  c->async_on = false;
  drain_completions(c);
  HIPCHK(c, hipMemcpyAsync(c->hdr_host, c->dc.hdr, sizeof(SchedHdr), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // records published after the kernel's last look at the ring
  for (uint32_t k = c->hdr_host->adm_head; k != c->ring_tail; ++k) stage(c, c->ring_adm[k % (uint32_t)c->tmax]);
  for (const Admit &a : c->staged) c->trees[a.slot].hstatus = H_STAGED;
  return sync_states(c);
}

trees_status run_persistent(trees_ctx *c, int64_t max_epochs) {
  trees_status s = hdr_begin(c, max_epochs);
  if (s) return s;
  const uint32_t need = ops_needed(c);
  const int grid = grid_size(c, need, true);
  c->last_grid = grid;
  if (timed(c, 0)) HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  HIPCHK(c, launch_epochs(c->dc, c->wg, need, grid, 1, c->stream));
  if (timed(c, 0)) HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  s = read_hdr(c);
  if (s) return s;
  if (timed(c, 0)) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->ktime[0].ms += ms;
    c->ktime[0].launches += 1;
  }
  return TREES_OK;
}

// The workload class of a context: its registered program kinds, ascending,
// joined by '+' (the key of a tuned shape beside the device name).
std::string workload_class(const trees_ctx *c) {
  std::vector<int> k;
  for (const auto &p : c->progs) k.push_back(p.kind);
  std::sort(k.begin(), k.end());
  std::string out;
  for (size_t i = 0; i < k.size(); ++i) out += (i ? "+" : "") + std::to_string(k[i]);
  return out;
}

std::string tuned_path(const char *path) {
  if (path && *path) return path;
  const char *e = getenv("TREES_TUNE_FILE");
  if (e && *e) return e;
  const char *h = getenv("HOME");
  return std::string(h && *h ? h : ".") + "/.cache/trees/tuned.txt";
}

// Reads the tuned file: one shape per line, "device<TAB>class<TAB>sched wg bpc
// chunk"; the last line for (device, class) wins.  Lines that do not parse
// are skipped.
bool read_tuned(const std::string &path, const std::string &dev, const std::string &wclass, trees_shape *out) {
  FILE *f = fopen(path.c_str(), "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char *t1 = strchr(line, '\t');
    if (!t1) continue;
    char *t2 = strchr(t1 + 1, '\t');
    if (!t2) continue;
    *t1 = 0; *t2 = 0;
    if (dev != line || wclass != (t1 + 1)) continue;
    trees_shape sh{};
    if (sscanf(t2 + 1, "%d %d %d %d", &sh.sched, &sh.wg_size, &sh.blocks_per_cu, &sh.graph_chunk) != 4) continue;
    if (sh.sched < TREES_SCHED_PLAIN || sh.sched > TREES_SCHED_PERSISTENT) continue;
    if (sh.wg_size != 256 && sh.wg_size != 512 && sh.wg_size != 1024) continue;
    if (sh.blocks_per_cu < 0 || sh.graph_chunk < 0) continue;
    *out = sh;
    found = true;
  }
  fclose(f);
  return found;
}

trees_status run_sched(trees_ctx *c, int sched, int64_t max_epochs, const std::vector<int> &before,
                       uint64_t *gepochs_out, int32_t *stop_out) {
  trees_status s = TREES_OK;
  uint64_t gepochs = 0;
  int32_t stop_reason = 1;
  c->last_wg = c->wg;
  if (sched == TREES_SCHED_PLAIN) {
    std::vector<int> order = before;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return c->trees[a].order < c->trees[b].order; });
    int64_t budget = max_epochs;
    const bool trace = c->dc.trace_on != 0;
    for (int slot : order) {
      s = run_plain_tree(c, slot, &budget, &gepochs, trace);
      if (s) return s;
      if (budget == 0) { stop_reason = 2; break; }
      if (*(volatile int32_t *)c->abort_flag) { stop_reason = 3; break; }
    }
  } else {
    s = (sched == TREES_SCHED_GRAPH) ? run_graph(c, max_epochs) : run_persistent(c, max_epochs);
    if (s) return s;
    gepochs = (uint64_t)c->hdr_host->run_epochs;
    stop_reason = c->hdr_host->stop_reason;
    s = sync_states(c);
    if (s) return s;
  }
  *gepochs_out = gepochs;
  *stop_out = stop_reason;
  return TREES_OK;
}

// ---------------------------------------------------------------------------
// Native worklist BFS / SSSP (Section 6.3's hand-managed comparison)
// ---------------------------------------------------------------------------
struct WlLayout {
  size_t ctl, in0, in1, stamp, total;
};
WlLayout wl_layout(int64_t V, bool sssp) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  WlLayout L{};
  L.ctl = 0;
  L.in0 = up(sizeof(WlCtl));
  L.in1 = L.in0 + up((size_t)V * 4);
  L.stamp = L.in1 + up((size_t)V * 4);
  L.total = L.stamp + (sssp ? up((size_t)V * 4) : 0);
  return L;
}

trees_status wl_run(trees_ctx *c, bool sssp, int32_t V, int32_t source, const int32_t *row_ptr,
                    const int32_t *col_idx, const int32_t *weights, int32_t *val, void *ws, uint64_t ws_bytes,
                    trees_wl_stats *out) {
  if (!c) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  const char *what = sssp ? "wl_sssp" : "wl_bfs";
  if (V < 1 || source < 0 || source >= V) return fail(c, TREES_E_INVALID, std::string(what) + ": need V >= 1 and 0 <= source < V");
  if (!row_ptr || !col_idx || !val || !ws || (sssp && !weights))
    return fail(c, TREES_E_INVALID, std::string(what) + ": null pointer");
  const WlLayout L = wl_layout(V, sssp);
  if (ws_bytes < L.total) return fail(c, TREES_E_INVALID, std::string(what) + ": workspace too small");
  const uintptr_t a = (uintptr_t)ws, b = (uintptr_t)val;
  if (a < b + (uint64_t)V * 4 && b < a + L.total)
    return fail(c, TREES_E_INVALID, std::string(what) + ": the output overlaps the workspace");
  if ((a & 255) != 0) return fail(c, TREES_E_INVALID, std::string(what) + ": workspace not 256-byte aligned");
  if (c->async_on) return fail(c, TREES_E_STATE, std::string(what) + ": an asynchronous run is active");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, TREES_E_DEVICE, "hipSetDevice failed");
  const auto t0 = std::chrono::steady_clock::now();
  char *w = (char *)ws;
  int32_t *lists[2] = {(int32_t *)(w + L.in0), (int32_t *)(w + L.in1)};
  int32_t *stamp = sssp ? (int32_t *)(w + L.stamp) : nullptr;
  HIPCHK(c, launch_wl_init(val, stamp, V, source, sssp ? INT32_MAX : -1, lists[0], w + L.ctl, c->stream));
  uint32_t n = 1;
  int32_t it = 0;
  uint64_t pushed = 0;
  while (n > 0) {
    WlArgs A{};
    A.row = row_ptr; A.col = col_idx; A.w = weights; A.val = val;
    A.in = lists[it & 1]; A.out = lists[(it & 1) ^ 1]; A.stamp = stamp;
    A.ctl = (WlCtl *)(w + L.ctl); A.mir = c->wl_mirror_dev;
    A.n_in = n; A.level = it; A.par = it & 1;
    A.seq = ++c->wl_seq ? c->wl_seq : ++c->wl_seq;
    HIPCHK(c, launch_wl(A, c->wg, sssp, c->stream));
    TRY(wait_seq(c, &c->wl_mirror->seq, A.seq));
    n = __atomic_load_n(&c->wl_mirror->count, __ATOMIC_ACQUIRE);
    if (n > (uint32_t)V) return fail(c, TREES_E_DEVICE, std::string(what) + ": output worklist beyond V entries");
    pushed += n;
    ++it;
  }
  if (out) {
    out->iterations = it;
    out->pad = 0;
    out->pushed = pushed;
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return TREES_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

trees_status trees_create(const trees_config *cfg, trees_ctx **out) {
  if (!cfg || !out || cfg->struct_size != sizeof(trees_config))
    return fail(nullptr, TREES_E_INVALID, "trees_create: bad config (struct_size mismatch?)");
  *out = nullptr;
  trees_ctx *c = new (std::nothrow) trees_ctx();
  if (!c) return fail(nullptr, TREES_E_NOMEM, "out of host memory");
  c->cfg = *cfg;
  c->device = cfg->device;
  c->tmax = cfg->max_trees > 0 ? cfg->max_trees : 4096;
  c->sched = cfg->sched;
  c->wg = cfg->wg_size ? cfg->wg_size : 256;
  c->bpc = cfg->blocks_per_cu;
  c->chunk = cfg->graph_chunk > 0 ? cfg->graph_chunk : 8;
  if (c->wg != 256 && c->wg != 512 && c->wg != 1024) {
    delete c;
    return fail(nullptr, TREES_E_INVALID, "wg_size must be 256, 512 or 1024");
  }
  auto bail = [&](trees_status st, const std::string &m) {
    g_create_error = m;
    trees_destroy(c);
    return st;
  };
  if (hipSetDevice(c->device) != hipSuccess) return bail(TREES_E_DEVICE, "hipSetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return bail(TREES_E_DEVICE, "no device properties");
  c->ncu = prop.multiProcessorCount;
  c->devname = prop.name;
  // the allocation-free worklist BFS's fixed workspace on this device
  if (wl_scratch_setup(c->device) != hipSuccess) return bail(TREES_E_DEVICE, "hipGetSymbolAddress of the worklist scratch failed");
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && khz > 0)
    c->clock_hz = khz * 1000.0;
  if (cfg->stream) {
    c->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(TREES_E_DEVICE, "hipStreamCreate failed");
    c->own_stream = true;
  }
  // task vector
  uint64_t bytes = cfg->arena_bytes;
  c->nent = (int64_t)(bytes / kBytesPerEntry) & ~(int64_t)63;
  if (c->nent <= 0) return bail(TREES_E_INVALID, "arena_bytes too small");
  if (cfg->arena_base) {
    c->arena = (char *)cfg->arena_base;
  } else {
    if (hipMalloc((void **)&c->arena, (size_t)c->nent * kBytesPerEntry + 256) != hipSuccess)
      return bail(TREES_E_NOMEM, "hipMalloc of the task vector failed");
    c->own_arena = true;
  }
  {
    char *p = c->arena;
    const size_t n = (size_t)c->nent;
    c->dc.r = (int64_t *)p; p += n * 8;     // 8-byte aligned first
    c->dc.code = (int32_t *)p; p += n * 4;
    c->dc.a0 = (int32_t *)p; p += n * 4;
    c->dc.a1 = (int32_t *)p; p += n * 4;
    c->dc.a2 = (int32_t *)p; p += n * 4;
    c->dc.a3 = (int32_t *)p; p += n * 4;
  }
  c->freel[0] = c->nent;
  c->free_ent = c->nent;
  // control block
  const size_t T = (size_t)c->tmax;
  const bool trace = (cfg->flags & TREES_F_TRACE) != 0;
  size_t off = 0;
  auto take = [&](size_t sz) { size_t o = off; off = (off + sz + 255) & ~(size_t)255; return o; };
  const size_t o_ts = take(T * sizeof(TreeStatic)), o_st = take(T * sizeof(TreeState)),
               o_hot = take(T * sizeof(TreeHot)), o_len = take(T * 4), o_cen = take(T * 4),
               o_b = take(T * 4), o_stk = take(T * kStackMax * sizeof(int4)),
               o_tr = trace ? take(T * kTraceMax * sizeof(TraceRec)) : 0, o_wt = take(2 * (T + 1) * 4),
               o_wo = take(2 * (T + 1) * 4), o_ws = take(2 * (T + 1) * 4), o_wc = take(2 * (T + 1) * 4),
               o_wtb = take(2 * (T + 1) * 4), o_wtp = take(2 * (T + 1) * 4),
               o_dl = take(T * 4), o_hdr = take(sizeof(SchedHdr)),
               o_pl = take(sizeof(PlainCounters)),
               o_adm = take(T * sizeof(Admit)), o_init = take(T * 4), o_self = take(2 * sizeof(DevCtx));
  const bool nomap = (cfg->flags & TREES_F_NOMAP) != 0;
  const size_t MJ = nomap ? 0 : (size_t)kMapJobs;
  const size_t PC = nomap ? 0 : (size_t)kPartCap;
  const size_t o_mjl = take(MJ * 4), o_mjh = take(MJ * 4), o_mjs = take(MJ * 8), o_mjd = take(MJ * 8),
               o_mjo = take(MJ * 8), o_pj = take(PC * 4), o_pi = take(PC * 8);
  const size_t o_aj = take((size_t)kArcJobs * sizeof(ArcJob)),
               o_ai = take((size_t)kArcJobs * kArcItemWords * 4),
               o_as = take((size_t)7 * kArcSegPool * 4),
               o_at = take((size_t)kArcTilesAll * sizeof(int4));
  if (hipMalloc(&c->ctl, off) != hipSuccess) return bail(TREES_E_NOMEM, "hipMalloc of control state failed");
  if (hipMemset(c->ctl, 0, off) != hipSuccess) return bail(TREES_E_DEVICE, "hipMemset failed");
  char *b = (char *)c->ctl;
  c->dc.ts = (const TreeStatic *)(b + o_ts);
  c->dc.st = (TreeState *)(b + o_st);
  c->dc.hot = (TreeHot *)(b + o_hot);
  c->dc.t_len = (int32_t *)(b + o_len);
  c->dc.t_cen = (int32_t *)(b + o_cen);
  c->dc.t_b = (int32_t *)(b + o_b);
  c->dc.stack = (int4 *)(b + o_stk);
  c->dc.trace = trace ? (TraceRec *)(b + o_tr) : nullptr;
  c->dc.wl_tree = (int32_t *)(b + o_wt);
  c->dc.wl_off = (uint32_t *)(b + o_wo);
  c->dc.wl_b = (int32_t *)(b + o_ws);
  c->dc.wl_tb = (uint32_t *)(b + o_wtb);
  c->dc.wl_tp = (uint32_t *)(b + o_wtp);
  c->dc.wl_cen = (int32_t *)(b + o_wc);
  c->dc.done_list = (int32_t *)(b + o_dl);
  c->dc.tmax = (int32_t)T;
  c->dc.hdr = (SchedHdr *)(b + o_hdr);
  c->dc.plain = (PlainCounters *)(b + o_pl);
  c->adm_dev = (Admit *)(b + o_adm);
  c->dc.init_slot = (int32_t *)(b + o_init);
  c->self_dev = (DevCtx *)(b + o_self);   // [0]: the context, [1]: its asynchronous-run form
  c->dc.self = c->self_dev;
  c->dc.mj_lo = (int32_t *)(b + o_mjl);
  c->dc.mj_hi = (int32_t *)(b + o_mjh);
  c->dc.mj_src = (const uint32_t **)(b + o_mjs);
  c->dc.mj_dst = (uint32_t **)(b + o_mjd);
  c->dc.mj_off = (uint64_t *)(b + o_mjo);
  c->dc.arc_job = (ArcJob *)(b + o_aj);
  c->dc.arc_item = (int32_t *)(b + o_ai);
  c->dc.arc_seg = (int32_t *)(b + o_as);
  c->dc.arc_tile = (int4 *)(b + o_at);
  c->dc.part_job = (uint32_t *)(b + o_pj);
  c->dc.part_ia = (int64_t *)(b + o_pi);
  c->dc.mj_cap = (int32_t)MJ;
  c->dc.part_cap = (int32_t)PC;
  c->dc.trace_on = trace ? 1 : 0;
  c->dc.debug = (cfg->flags & TREES_F_DEBUG) ? 1 : 0;
  const double to = cfg->timeout_s > 0 ? cfg->timeout_s : 60.0;
  c->dc.timeout_ticks = (int64_t)(to * c->clock_hz);
  c->dc.idle_ticks = (int64_t)(to * c->clock_hz);   // an idle asynchronous run ends by itself after this
  c->timeout_s = to;
  // pinned host memory
  if (hipHostMalloc((void **)&c->adm_host, T * sizeof(Admit), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->mirror, sizeof(PlainMirror), hipHostMallocCoherent | hipHostMallocMapped) !=
          hipSuccess ||
      hipHostMalloc((void **)&c->hdr_host, sizeof(SchedHdr), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->st_host, T * sizeof(TreeState), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->r_host, 64, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->abort_flag, 64, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
      hipHostMalloc((void **)&c->wl_mirror, sizeof(WlMirror), hipHostMallocCoherent | hipHostMallocMapped) !=
          hipSuccess ||
      hipHostMalloc((void **)&c->hmirror, sizeof(HdrMirror), hipHostMallocCoherent | hipHostMallocMapped) !=
          hipSuccess ||
      hipHostMalloc((void **)&c->self_host, 2 * sizeof(DevCtx), hipHostMallocDefault) != hipSuccess)
    return bail(TREES_E_NOMEM, "hipHostMalloc failed");
  memset(c->wl_mirror, 0, sizeof(WlMirror));
  {   // asynchronous runs: ring header, admission and completion records
    const size_t rb = sizeof(AsyncRing) + T * sizeof(Admit) + T * sizeof(Completion);
    char *rp = nullptr;
    if (hipHostMalloc((void **)&rp, rb, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
      return bail(TREES_E_NOMEM, "hipHostMalloc of the asynchronous rings failed");
    memset(rp, 0, rb);
    c->ring = (AsyncRing *)rp;
    c->ring_adm = (Admit *)(rp + sizeof(AsyncRing));
    c->ring_done = (Completion *)(rp + sizeof(AsyncRing) + T * sizeof(Admit));
    char *rd = nullptr;
    if (hipHostGetDevicePointer((void **)&rd, rp, 0) != hipSuccess)
      return bail(TREES_E_DEVICE, "hipHostGetDevicePointer failed");
    c->dc.ring = (AsyncRing *)rd;
    c->dc.ring_adm = (const Admit *)(rd + sizeof(AsyncRing));
    c->dc.ring_done = (Completion *)(rd + sizeof(AsyncRing) + T * sizeof(Admit));
    c->dc.async_mode = 0;
    c->dc.slice_ticks = (int64_t)(2e-3 * c->clock_hz);   // 2 ms of idle waiting per empty epoch
  }
  if (hipHostGetDevicePointer((void **)&c->wl_mirror_dev, c->wl_mirror, 0) != hipSuccess)
    return bail(TREES_E_DEVICE, "hipHostGetDevicePointer failed");
  *c->abort_flag = 0;
  int32_t *dev_abort = nullptr;
  if (hipHostGetDevicePointer((void **)&dev_abort, c->abort_flag, 0) != hipSuccess)
    return bail(TREES_E_DEVICE, "hipHostGetDevicePointer failed");
  c->dc.abort_flag = dev_abort;
  memset(c->mirror, 0, sizeof(PlainMirror));
  if (hipHostGetDevicePointer((void **)&c->dc.mirror, c->mirror, 0) != hipSuccess)
    return bail(TREES_E_DEVICE, "hipHostGetDevicePointer failed");
  memset(c->hmirror, 0, sizeof(HdrMirror));
  if (hipHostGetDevicePointer((void **)&c->hmirror_dev, c->hmirror, 0) != hipSuccess)
    return bail(TREES_E_DEVICE, "hipHostGetDevicePointer failed");
  c->profile = (cfg->flags & TREES_F_PROFILE) != 0;
  if (c->profile && (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess))
    return bail(TREES_E_DEVICE, "hipEventCreate failed");
  c->trees.resize(c->tmax);
  *out = c;
  return TREES_OK;
}

void trees_destroy(trees_ctx *c) {
  if (!c) return;
  if (c->async_on) {   // end the asynchronous run at its next epoch boundary
    __atomic_store_n(&c->ring->close, 1, __ATOMIC_RELEASE);
    __atomic_store_n(c->abort_flag, 1, __ATOMIC_SEQ_CST);
  }
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->own_arena && c->arena) (void)hipFree(c->arena);
  if (c->ctl) (void)hipFree(c->ctl);
  if (c->adm_host) (void)hipHostFree(c->adm_host);
  if (c->mirror) (void)hipHostFree(c->mirror);
  if (c->hmirror) (void)hipHostFree(c->hmirror);
  for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
  if (c->hdr_host) (void)hipHostFree(c->hdr_host);
  if (c->st_host) (void)hipHostFree(c->st_host);
  if (c->r_host) (void)hipHostFree(c->r_host);
  if (c->abort_flag) (void)hipHostFree(c->abort_flag);
  if (c->wl_mirror) (void)hipHostFree(c->wl_mirror);
  if (c->ring) (void)hipHostFree(c->ring);
  if (c->self_host) (void)hipHostFree(c->self_host);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char *trees_last_error(const trees_ctx *c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

trees_status trees_register_program(trees_ctx *c, int32_t kind, int32_t *out_prog) {
  if (!c || !out_prog) return fail(c, TREES_E_INVALID, "null argument");
  std::lock_guard<std::mutex> g(c->mu);
  const uint32_t ops = ops_of_kind(kind);
  if (!ops) return fail(c, TREES_E_INVALID, "unknown program kind");
  for (size_t p = 0; p < c->progs.size(); ++p)
    if (c->progs[p].kind == kind) { *out_prog = (int32_t)p; return TREES_OK; }
  if (c->frozen) return fail(c, TREES_E_STATE, "programs must be registered before the first submit");
  Prog p;
  p.kind = kind;
  p.ntypes = (kind == TREES_PROG_BFS_CSR || kind == TREES_PROG_SSSP_CSR || kind == TREES_PROG_PREORDER) ? 1 : 2;
  p.tbase = c->ntt + 1;
  p.ops = ops;
  if (c->ntt + p.ntypes > kMaxTypes) return fail(c, TREES_E_INVALID, "too many task types");
  c->ntt += p.ntypes;
  // type ids of the program: tbase = body type, tbase + 1 = its join continuation
  switch (kind) {
    case TREES_PROG_FIB_I32: c->dc.op_of_type[p.tbase] = OP_FIB32; c->dc.op_of_type[p.tbase + 1] = OP_SUM32; break;
    case TREES_PROG_FIB_I64: c->dc.op_of_type[p.tbase] = OP_FIB64; c->dc.op_of_type[p.tbase + 1] = OP_SUM64; break;
    case TREES_PROG_MSORT_U32: c->dc.op_of_type[p.tbase] = OP_MS; c->dc.op_of_type[p.tbase + 1] = OP_MERGE; break;
    case TREES_PROG_NQUEENS: c->dc.op_of_type[p.tbase] = OP_Q; c->dc.op_of_type[p.tbase + 1] = OP_QSUM; break;
    case TREES_PROG_BFS_CSR: c->dc.op_of_type[p.tbase] = OP_VISIT; break;
    case TREES_PROG_POSTORDER: c->dc.op_of_type[p.tbase] = OP_POST; c->dc.op_of_type[p.tbase + 1] = OP_PVISIT; break;
    case TREES_PROG_PREORDER: c->dc.op_of_type[p.tbase] = OP_PRE; break;
    case TREES_PROG_FFT: c->dc.op_of_type[p.tbase] = OP_FFT; c->dc.op_of_type[p.tbase + 1] = OP_COMB; break;
    case TREES_PROG_SSSP_CSR: c->dc.op_of_type[p.tbase] = OP_SVISIT; break;
  }
  c->dc.ntt = c->ntt;
  c->progs.push_back(p);
  *out_prog = (int32_t)(c->progs.size() - 1);
  return TREES_OK;
}

// Whether the first n bytes of buffers a and b share memory (a tree writes
// its output buffers while it reads its inputs).
bool overlap(const trees_buf &a, const trees_buf &b, uint64_t na, uint64_t nb) {
  const uintptr_t x = (uintptr_t)a.ptr, y = (uintptr_t)b.ptr;
  return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

trees_status trees_submit(trees_ctx *c, int32_t prog, const int64_t *args, int32_t nargs,
                          const trees_buf *bufs, int32_t nbufs, uint64_t *out_tree) {
  if (!c || !out_tree) return fail(c, TREES_E_INVALID, "null argument");
  std::lock_guard<std::mutex> g(c->mu);
  // an asynchronous run that has ended by itself (idle limit, budget, abort)
  // no longer adopts submissions: collect it, and stage this tree instead
  if (c->async_on && hipStreamQuery(c->stream) != hipErrorNotReady) TRY(finish_async(c, false));
  if (prog < 0 || prog >= (int)c->progs.size()) return fail(c, TREES_E_INVALID, "unknown program id");
  const Prog &P = c->progs[prog];
  int64_t bound = 0;
  std::string e;
  trees_status st = tv_bound(P.kind, args, nargs, &bound, &e);
  if (st) return fail(c, st, e);
  if (bound >= (1ll << 31)) return fail(c, TREES_E_INVALID, "tree too large for one arena");
  Admit a{};
  a.ts.kind = P.kind;
  a.ts.tbase = P.tbase;
  a.root_code = 0 * c->ntt + P.tbase;   // epoch 0, the program's first type
  switch (P.kind) {
    case TREES_PROG_FIB_I32:
    case TREES_PROG_FIB_I64:
      a.a0 = (int32_t)args[0];
      a.ts.p0 = (int32_t)args[0];
      break;
    case TREES_PROG_NQUEENS:
      a.ts.p0 = (int32_t)args[0];
      break;
    case TREES_PROG_MSORT_U32: {
      const int64_t N = args[0];
      if (nbufs < 2 || !bufs || (N > 0 && (!bufs[0].ptr || !bufs[1].ptr)) ||
          bufs[0].bytes < (uint64_t)N * 4 || bufs[1].bytes < (uint64_t)N * 4)
        return fail(c, TREES_E_INVALID, "msort: need bufs {keys[N], tmp[N]} of uint32");
      if (overlap(bufs[0], bufs[1], (uint64_t)N * 4, (uint64_t)N * 4))
        return fail(c, TREES_E_INVALID, "msort: keys and tmp must not overlap");
      a.a0 = 0; a.a1 = (int32_t)N; a.a2 = 0;
      a.ts.p0 = (int32_t)N;
      a.ts.ptr0 = (uint64_t)bufs[0].ptr;
      a.ts.ptr1 = (uint64_t)bufs[1].ptr;
    } break;
    case TREES_PROG_BFS_CSR: {
      const int64_t V = args[0], src = args[1];
      if (nbufs < 3 || !bufs || !bufs[0].ptr || !bufs[1].ptr || !bufs[2].ptr ||
          bufs[0].bytes < (uint64_t)(V + 1) * 4 || bufs[2].bytes < (uint64_t)V * 4)
        return fail(c, TREES_E_INVALID, "bfs: need bufs {row_ptr[V+1], col_idx[E], depth[V]} of int32");
      if (overlap(bufs[2], bufs[0], (uint64_t)V * 4, (uint64_t)(V + 1) * 4) ||
          overlap(bufs[2], bufs[1], (uint64_t)V * 4, bufs[1].bytes))
        return fail(c, TREES_E_INVALID, "bfs: depth must not overlap the graph");
      a.a0 = (int32_t)src;
      a.ts.p0 = (int32_t)V;
      a.ts.p1 = (int32_t)src;
      a.ts.ptr0 = (uint64_t)bufs[0].ptr;
      a.ts.ptr1 = (uint64_t)bufs[1].ptr;
      a.ts.ptr2 = (uint64_t)bufs[2].ptr;
    } break;
    case TREES_PROG_SSSP_CSR: {
      const int64_t V = args[0], src = args[1];
      if (nbufs < 4 || !bufs || !bufs[0].ptr || !bufs[1].ptr || !bufs[2].ptr || !bufs[3].ptr ||
          bufs[0].bytes < (uint64_t)(V + 1) * 4 || bufs[2].bytes < bufs[1].bytes ||
          bufs[3].bytes < (uint64_t)V * 4)
        return fail(c, TREES_E_INVALID,
                    "sssp: need bufs {row_ptr[V+1], col_idx[E], weights[E], dist[V]} of int32");
      if (overlap(bufs[3], bufs[0], (uint64_t)V * 4, (uint64_t)(V + 1) * 4) ||
          overlap(bufs[3], bufs[1], (uint64_t)V * 4, bufs[1].bytes) ||
          overlap(bufs[3], bufs[2], (uint64_t)V * 4, bufs[2].bytes))
        return fail(c, TREES_E_INVALID, "sssp: dist must not overlap the graph or the weights");
      a.a0 = (int32_t)src;
      a.ts.p0 = (int32_t)V;
      a.ts.p1 = (int32_t)src;
      a.ts.ptr0 = (uint64_t)bufs[0].ptr;
      a.ts.ptr1 = (uint64_t)bufs[1].ptr;
      a.ts.ptr2 = (uint64_t)bufs[3].ptr;   // the per-vertex array (as BFS depth)
      a.ts.ptr3 = (uint64_t)bufs[2].ptr;   // arc weights
    } break;
    case TREES_PROG_FFT: {
      const uint64_t bytes = (uint64_t)8 << args[0];
      if (nbufs < 2 || !bufs || !bufs[0].ptr || !bufs[1].ptr || bufs[0].bytes < bytes || bufs[1].bytes < bytes)
        return fail(c, TREES_E_INVALID, "fft: need bufs {x[N], y[N]} of complex fp32");
      const uintptr_t x0 = (uintptr_t)bufs[0].ptr, y0 = (uintptr_t)bufs[1].ptr;
      if (x0 < y0 + bytes && y0 < x0 + bytes)   // the leaves read x while combines write y
        return fail(c, TREES_E_INVALID, "fft: x and y must not overlap");
      a.a0 = 0; a.a1 = 0; a.a2 = 0;   // FFT(lo = 0, o = 0, ls = 0): the whole input
      a.ts.p0 = (int32_t)args[0];
      a.ts.ptr0 = (uint64_t)bufs[0].ptr;
      a.ts.ptr1 = (uint64_t)bufs[1].ptr;
    } break;
    case TREES_PROG_POSTORDER:
    case TREES_PROG_PREORDER: {
      const int64_t n = args[0];
      if (nbufs < 3 || !bufs || !bufs[0].ptr || !bufs[1].ptr || !bufs[2].ptr ||
          bufs[0].bytes < (uint64_t)n * 4 || bufs[1].bytes < (uint64_t)n * 4 ||
          bufs[2].bytes < (uint64_t)(n + 1) * 4)
        return fail(c, TREES_E_INVALID, "postorder: need bufs {left[n], right[n], log[n+1]} of int32");
      if (overlap(bufs[2], bufs[0], (uint64_t)(n + 1) * 4, (uint64_t)n * 4) ||
          overlap(bufs[2], bufs[1], (uint64_t)(n + 1) * 4, (uint64_t)n * 4))
        return fail(c, TREES_E_INVALID, "traversal: log must not overlap the tree");
      a.a0 = (int32_t)args[1];
      a.ts.p0 = (int32_t)n;
      a.ts.p1 = (int32_t)args[1];
      a.ts.ptr0 = (uint64_t)bufs[0].ptr;
      a.ts.ptr1 = (uint64_t)bufs[1].ptr;
      a.ts.ptr2 = (uint64_t)bufs[2].ptr;
    } break;
  }
  int slot = -1;
  for (int s = 0; s < c->tmax; ++s)
    if (c->trees[s].hstatus == H_FREE) { slot = s; break; }
  if (slot < 0) return fail(c, TREES_E_NOMEM, "no free tree slot");
  const int64_t base = arena_alloc(c, bound);
  if (base < 0) return fail(c, TREES_E_NOMEM, "task-vector budget exhausted");
  c->frozen = true;
  a.slot = slot;
  a.ts.base = base;
  a.ts.cap = (int32_t)bound;
  HostTree &t = c->trees[slot];
  t.hstatus = H_STAGED;
  t.prog = prog;
  t.kind = P.kind;
  t.base = base;
  t.cap = bound;
  t.order = c->order++;
  // the kernels' per-tree parameter: nqueens n, or postorder's node count
  // (its visit counter sits at log[n])
  const bool with_n = P.kind == TREES_PROG_NQUEENS || P.kind == TREES_PROG_POSTORDER ||
                      P.kind == TREES_PROG_PREORDER || P.kind == TREES_PROG_FFT;
  // (SSSP: its bucket width)
  const uint32_t param = with_n ? (uint32_t)args[0]
                         : (P.kind == TREES_PROG_SSSP_CSR && nargs >= 4) ? (uint32_t)args[3] : 0u;
  t.tp = (uint32_t)P.tbase | (param << 8);
  a.ts.tp = t.tp;
  if (c->async_on) {
    // publish into the admission ring: the running kernel adopts the tree at
    // its next epoch boundary (and initialises its buffers there)
    c->ring_adm[c->ring_tail % (uint32_t)c->tmax] = a;
    __atomic_store_n(&c->ring->tail, c->ring_tail + 1, __ATOMIC_RELEASE);
    c->ring_tail++;
    t.hstatus = H_LIVE;
    memset(&t.st, 0, sizeof(t.st));
    t.st.e = 1; t.st.old = 1; t.st.status = TS_LIVE; t.st.tasks = 0; t.st.peak = 1;
    t.st.done_gepoch = -1; t.st.start_gepoch = -1;
  } else {
    stage(c, a);
  }
  c->tslots = std::max(c->tslots, slot + 1);
  c->ntrees++;
  *out_tree = ((uint64_t)t.gen << 32) | (uint32_t)slot;
  return TREES_OK;
}

trees_status trees_run(trees_ctx *c, int64_t max_epochs, uint32_t flags, trees_run_stats *out) {
  if (!c) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  if (flags & ~(uint32_t)TREES_RUN_ASYNC) return fail(c, TREES_E_INVALID, "unknown trees_run flags");
  auto t0 = std::chrono::steady_clock::now();
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, TREES_E_DEVICE, "hipSetDevice failed");
  if (out) memset(out, 0, sizeof(*out));
  if (c->async_on) {
    // a blocking call closes the asynchronous run: its kernel finishes every
    // live and submitted tree, then returns
    if (flags & TREES_RUN_ASYNC) return fail(c, TREES_E_STATE, "an asynchronous run is already active");
    TRY(finish_async(c, true));
    if (out) {
      out->global_epochs = (uint64_t)c->hdr_host->run_epochs;
      out->tasks = c->async_tasks;
      out->stop_reason = c->hdr_host->stop_reason;
      int live = 0;
      for (int i = 0; i < c->tslots; ++i) live += c->trees[i].hstatus == H_LIVE || c->trees[i].hstatus == H_STAGED;
      out->live = live;
      out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - c->async_t0).count();
      out->grid = c->last_grid;
      out->api_blocks_per_cu = c->last_api_bpc;
      out->sched = TREES_SCHED_PERSISTENT;
      out->wg_size = c->wg;
    }
    if (c->hdr_host->stop_reason == 4) return fail(c, TREES_E_DEVICE, "persistent barrier timed out");
    return TREES_OK;
  }
  *(volatile int32_t *)c->abort_flag = 0;
  trees_status s = flush_admissions(c);
  if (s) return s;
  std::vector<int> before;
  for (int i = 0; i < c->tslots; ++i)
    if (c->trees[i].hstatus == H_LIVE) before.push_back(i);
  if (flags & TREES_RUN_ASYNC) {
    if (c->sched != TREES_SCHED_PERSISTENT && c->sched != TREES_SCHED_AUTO)
      return fail(c, TREES_E_INVALID, "an asynchronous run needs the PERSISTENT (or AUTO) scheduler");
    TRY(start_async(c, max_epochs));
    if (out) {
      out->live = (int32_t)before.size();
      out->grid = c->last_grid;
      out->api_blocks_per_cu = c->last_api_bpc;
      out->sched = TREES_SCHED_PERSISTENT;
      out->wg_size = c->wg;
      out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return TREES_OK;
  }
  uint64_t gepochs = 0;
  int32_t stop_reason = 1;
  // AUTO: the shape the tuner chose for this device and workload class (read
  // once from the tuned file), else the graph form at the context's shape
  int sched = c->sched;
  const int wg0 = c->wg, bpc0 = c->bpc, chunk0 = c->chunk;
  if (sched == TREES_SCHED_AUTO) {
    if (!c->tuned_done) {
      c->tuned_ok = read_tuned(tuned_path(nullptr), c->devname, workload_class(c), &c->tuned);
      c->tuned_done = true;
    }
    sched = TREES_SCHED_GRAPH;
    if (c->tuned_ok) {
      sched = c->tuned.sched;
      c->wg = c->tuned.wg_size;
      c->bpc = c->tuned.blocks_per_cu;
      if (c->tuned.graph_chunk > 0) c->chunk = c->tuned.graph_chunk;
    }
  }
  s = run_sched(c, sched, max_epochs, before, &gepochs, &stop_reason);
  c->wg = wg0; c->bpc = bpc0; c->chunk = chunk0;   // (AUTO's shape holds for this run only)
  if (s) return s;
  if (out) {
    out->global_epochs = gepochs;
    uint64_t tasks = 0;
    int live = 0;
    for (int i : before) {
      HostTree &t = c->trees[i];
      if (t.hstatus == H_DONE) tasks += (uint64_t)t.st.tasks;
      else if (t.hstatus == H_LIVE) ++live;
    }
    out->tasks = tasks;
    out->live = live;
    out->stop_reason = stop_reason;
    out->grid = (sched == TREES_SCHED_PLAIN) ? 0 : c->last_grid;
    out->api_blocks_per_cu = c->last_api_bpc;
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    out->sched = sched;
    out->wg_size = c->last_wg;
  }
  if (stop_reason == 4) return fail(c, TREES_E_DEVICE, "persistent barrier timed out");
  return TREES_OK;
}

static HostTree *find_tree(trees_ctx *c, uint64_t id, int *slot) {
  const int s = (int)(uint32_t)id;
  const uint32_t gen = (uint32_t)(id >> 32);
  if (s < 0 || s >= c->tmax) return nullptr;
  HostTree &t = c->trees[s];
  if (t.hstatus == H_FREE || t.gen != gen) return nullptr;
  *slot = s;
  return &t;
}

// While an asynchronous run is active: take in its completions, and collect
// the run if its kernel has ended by itself.
static trees_status async_progress(trees_ctx *c) {
  if (!c->async_on) return TREES_OK;
  drain_completions(c);
  if (hipStreamQuery(c->stream) != hipErrorNotReady) return finish_async(c, false);
  return TREES_OK;
}

trees_status trees_results(trees_ctx *c, uint64_t tree, int64_t *out_value, trees_tree_stats *out) {
  if (!c) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  int slot;
  HostTree *t = find_tree(c, tree, &slot);
  if (!t) return fail(c, TREES_E_INVALID, "unknown tree id");
  if (t->hstatus == H_LIVE) TRY(async_progress(c));
  if (t->hstatus != H_DONE) {
    if (out) { memset(out, 0, sizeof(*out)); out->status = TREES_E_PENDING; }
    return TREES_E_PENDING;
  }
  const TreeState &st = t->st;
  if (out_value) *out_value = st.result;
  if (out) {
    out->status = st.err;
    out->epochs = (uint32_t)st.epochs;
    out->tasks = (uint64_t)st.tasks;
    out->launched = (uint64_t)st.launched;
    out->peak_entries = (uint64_t)st.peak;
    out->start_epoch = st.start_gepoch;
    out->done_epoch = st.done_gepoch;
  }
  const trees_status rc = st.err;
  arena_free(c, t->base, t->cap);
  t->hstatus = H_FREE;
  t->gen++;
  c->ntrees--;
  return rc;
}

trees_status trees_poll(trees_ctx *c, uint64_t *ids, int32_t cap, int32_t *n) {
  if (!c || !n || cap < 0 || (cap > 0 && !ids)) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  *n = 0;
  TRY(async_progress(c));
  int k = 0;
  while (k < cap && !c->finished.empty()) {
    const uint64_t id = c->finished.front();
    c->finished.pop_front();
    int slot;
    HostTree *t = find_tree(c, id, &slot);
    if (!t || t->hstatus != H_DONE) continue;   // already released by trees_results
    ids[k++] = id;
  }
  *n = k;
  return TREES_OK;
}

trees_status trees_trace(trees_ctx *c, uint64_t tree, trees_epoch_rec *out, int32_t cap, int32_t *n) {
  if (!c || !n) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  if (c->async_on) return fail(c, TREES_E_STATE, "trees_trace: an asynchronous run is active");
  int slot;
  HostTree *t = find_tree(c, tree, &slot);
  if (!t) return fail(c, TREES_E_INVALID, "unknown tree id");
  static_assert(sizeof(TraceRec) == sizeof(trees_epoch_rec), "trace record layout");
  if (!c->dc.trace) return fail(c, TREES_E_STATE, "context created without TREES_F_TRACE");
  const int total = std::min<int>(t->st.ntrace, kTraceMax);
  const int m = std::min<int>(cap, total);
  if (m > 0)
    HIPCHK(c, hipMemcpy(out, c->dc.trace + (size_t)slot * kTraceMax, sizeof(TraceRec) * m, hipMemcpyDeviceToHost));
  *n = total;
  return TREES_OK;
}

trees_status trees_abort(trees_ctx *c) {
  if (!c || !c->abort_flag) return TREES_E_INVALID;
  __atomic_store_n(c->abort_flag, 1, __ATOMIC_SEQ_CST);
  return TREES_OK;
}

trees_status trees_set_schedule(trees_ctx *c, int32_t sched, int32_t wg, int32_t bpc, int32_t chunk) {
  if (!c) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  if (c->async_on) return fail(c, TREES_E_STATE, "trees_set_schedule: an asynchronous run is active");
  if (sched < 0 || sched > TREES_SCHED_AUTO) return fail(c, TREES_E_INVALID, "bad scheduler");
  if (wg && wg != 256 && wg != 512 && wg != 1024) return fail(c, TREES_E_INVALID, "bad wg_size");
  c->sched = sched;
  if (wg) c->wg = wg;
  c->bpc = bpc;
  if (chunk > 0) c->chunk = chunk;
  return TREES_OK;
}

trees_status trees_tv_bound(int32_t kind, const int64_t *args, int32_t nargs, int64_t *entries) {
  if (!entries) return TREES_E_INVALID;
  return tv_bound(kind, args, nargs, entries, nullptr);
}

trees_status trees_profile_mask(trees_ctx *c, uint32_t mask) {
  if (!c) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->profile) return fail(c, TREES_E_STATE, "context created without TREES_F_PROFILE");
  c->prof_mask = mask & 0x7FFu;
  return TREES_OK;
}

trees_status trees_kernel_times(trees_ctx *c, trees_ktime *out, int32_t n) {
  if (!c || !out) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  if (!c->profile) return fail(c, TREES_E_STATE, "context created without TREES_F_PROFILE");
  for (int k = 0; k < n && k < 11; ++k) out[k] = c->ktime[k];
  return TREES_OK;
}

trees_status trees_debug_phases(trees_ctx *c, double *us, int32_t n) {
  if (!c || !us) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  if (c->async_on) return fail(c, TREES_E_STATE, "trees_debug_phases: an asynchronous run is active");
  HIPCHK(c, hipMemcpy(c->hdr_host, c->dc.hdr, sizeof(SchedHdr), hipMemcpyDeviceToHost));
  for (int k = 0; k < n && k < 8; ++k) us[k] = (double)c->hdr_host->phase[k] * 1e6 / c->clock_hz;
  return TREES_OK;
}

trees_status trees_epoch_times(trees_ctx *c, double *us, int32_t cap, int32_t *n) {
  if (!c || !n) return TREES_E_INVALID;
  std::lock_guard<std::mutex> g(c->mu);
  if (c->async_on) return fail(c, TREES_E_STATE, "trees_epoch_times: an asynchronous run is active");
  HIPCHK(c, hipMemcpy(c->hdr_host, c->dc.hdr, sizeof(SchedHdr), hipMemcpyDeviceToHost));
  const int ne = (int)std::min<int64_t>(c->hdr_host->run_epochs, kEpochStamps);
  int64_t prev = c->hdr_host->stamp0;
  for (int e = 0; e < ne && e < cap; ++e) {
    us[e] = (double)(c->hdr_host->stamp[e] - prev) * 1e6 / c->clock_hz;
    prev = c->hdr_host->stamp[e];
  }
  *n = ne;
  return TREES_OK;
}

trees_status trees_tuned_shape(const char *path, const char *device, const char *wclass, trees_shape *out) {
  if (!device || !wclass || !out) return TREES_E_INVALID;
  return read_tuned(tuned_path(path), device, wclass, out) ? TREES_OK : TREES_E_INVALID;
}

trees_status trees_workload_class(const trees_ctx *c, char *buf, int32_t cap) {
  if (!c || !buf || cap <= 0) return TREES_E_INVALID;
  const std::string w = workload_class(c);
  const size_t n = std::min<size_t>(w.size(), (size_t)cap - 1);
  memcpy(buf, w.data(), n);
  buf[n] = 0;
  return TREES_OK;
}

trees_status trees_wl_workspace_bytes(int32_t V, int32_t sssp, uint64_t *bytes) {
  if (!bytes || V < 1) return TREES_E_INVALID;
  *bytes = wl_layout(V, sssp != 0).total;
  return TREES_OK;
}

trees_status trees_wl_bfs(trees_ctx *c, int32_t V, int32_t source, const int32_t *row_ptr, const int32_t *col_idx,
                          int32_t *depth, void *ws, uint64_t ws_bytes, trees_wl_stats *out) {
  return wl_run(c, false, V, source, row_ptr, col_idx, nullptr, depth, ws, ws_bytes, out);
}

trees_status trees_wl_sssp(trees_ctx *c, int32_t V, int32_t source, const int32_t *row_ptr, const int32_t *col_idx,
                           const int32_t *weights, int32_t *dist, void *ws, uint64_t ws_bytes, trees_wl_stats *out) {
  return wl_run(c, true, V, source, row_ptr, col_idx, weights, dist, ws, ws_bytes, out);
}

trees_status trees_wl_bfs_noalloc(trees_ctx *c, int32_t V, int32_t source, const int32_t *row_ptr,
                                  const int32_t *col_idx, int32_t *depth, trees_wl_stats *out) {
  if (!c) return TREES_E_INVALID;
  if (V > kWlScratchMaxV) return fail(c, TREES_E_INVALID, "wl_bfs_noalloc: V above 2^22, the fixed workspace's limit");
  void *ws = wl_scratch_ptr(c->device);
  if (!ws) return fail(c, TREES_E_STATE, "wl_bfs_noalloc: no fixed workspace on this device");
  return wl_run(c, false, V, source, row_ptr, col_idx, nullptr, depth, ws, kWlScratchBytes, out);
}

int64_t trees_free_entries(const trees_ctx *c) { return c ? c->free_ent : 0; }

int32_t trees_num_trees(const trees_ctx *c) { return c ? c->ntrees : 0; }

}  // extern "C"
