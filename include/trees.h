/*
 * libtrees -- the TREES epoch runtime (Hechtman, Hilton and Sorin, "TREES: A
 * CPU/GPU Task-Parallel Runtime with Explicit Epoch Synchronization") for
 * AMD Instinct MI355X (gfx950).
 *
 * A program is a set of task types whose bodies use fork / join / emit
 * (Section 4.3.2).  The runtime keeps every task in a task vector in HBM and
 * runs the program as a sequence of bulk-synchronous epochs (Section 4.3):
 * Phase 1 picks the next epoch's range of task-vector entries, Phase 2 runs
 * every task of the range in parallel on the GPU, Phase 3 pushes the ranges
 * created by forks and joins.  Many independent task trees may share the
 * epochs of one context.
 *
 * Conventions of the whole interface:
 *  - every function returns a trees_status (0 = success, < 0 = error) unless
 *    stated otherwise; no C++ exception crosses this boundary;
 *  - "device pointer" means memory of the context's GPU (hipMalloc'd or a
 *    PyTorch CUDA/HIP tensor's data pointer); the caller owns it;
 *  - trees_last_error() returns a message for the last failed call.
 */
#ifndef TREES_H
#define TREES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct trees_ctx trees_ctx;
typedef int32_t trees_status;

enum {
  TREES_OK = 0,
  TREES_E_INVALID = -1,   /* bad argument or program */
  TREES_E_NOMEM = -2,     /* the tree's task-vector arena does not fit in the budget now */
  TREES_E_OVERFLOW = -3,  /* a tree needed more task-vector entries than reserved */
  TREES_E_PENDING = -4,   /* the tree has not finished yet */
  TREES_E_DEVICE = -5,    /* a HIP runtime call failed */
  TREES_E_ABORTED = -6,   /* the run stopped on trees_abort or its epoch budget */
  TREES_E_STATE = -7,     /* call not allowed in the context's current state */
  TREES_E_ENCODING = -8,  /* a task-vector entry held a code outside its epoch's window */
  TREES_E_STACK = -9      /* a tree exceeded the per-tree stack depth (128 records) */
};

/* Scheduler: how epochs are sequenced.
 *  PLAIN      one kernel launch per epoch of one tree, Phases 1 and 3 on the
 *             host after copying back nextFreeCore and the join count
 *             (Sections 5.2.2-5.2.4); trees run one after another.
 *  GRAPH      all live trees share each epoch; Phases 1 and 3 run on the
 *             device; a captured chain of `graph_chunk` epoch launches is
 *             replayed until no tree is live.
 *  PERSISTENT all live trees share each epoch inside one co-resident
 *             (cooperative) launch with a device grid barrier per epoch.
 *  AUTO       the launch shape (scheduler, work-group size, work-groups per
 *             CU, graph chunk) that a tuner recorded for this device and the
 *             context's workload class in the tuned file (trees_tuned_shape);
 *             without such a record, GRAPH at the context's own shape.  The
 *             file is read once, at the context's first AUTO run. */
typedef enum {
  TREES_SCHED_PLAIN = 0,
  TREES_SCHED_GRAPH = 1,
  TREES_SCHED_PERSISTENT = 2,
  TREES_SCHED_AUTO = 3
} trees_sched;

enum {
  TREES_F_TRACE = 1u,   /* record per-epoch (CEN, range, valid, forks, joins) per tree */
  TREES_F_DEBUG = 2u,
  TREES_F_PROFILE = 4u, /* time every epoch launch with HIP events (trees_kernel_times) */
  TREES_F_NOMAP = 8u    /* merge continuations merge serially in their own lane (the paper's
                         * naive mergesort) instead of registering a data-parallel map job
                         * (Section 4.2) that a co-operative merge-path launch runs before
                         * the next epoch */
};

/* trees_run flags */
enum {
  TREES_RUN_ASYNC = 1u  /* start a persistent run and return at once (see trees_run) */
};

typedef struct {
  uint32_t struct_size;   /* sizeof(trees_config) */
  int32_t device;         /* HIP device ordinal */
  void *stream;           /* hipStream_t to run on; NULL = a stream owned by the context */
  void *arena_base;       /* device pointer to the task-vector budget; NULL = the library allocates */
  uint64_t arena_bytes;   /* budget in bytes (28 bytes per task-vector entry) */
  int32_t max_trees;      /* tree slots; 0 = 4096 */
  int32_t sched;          /* trees_sched */
  int32_t wg_size;        /* 256, 512 or 1024; 0 = 256 (the paper's work-group size, Section 5.1.1) */
  int32_t blocks_per_cu;  /* work-groups per CU for GRAPH/PERSISTENT grids; 0 = automatic: the
                           * co-resident count (the runtime's occupancy figure bounded by the
                           * kernel's own register and LDS use; 3/4 of it for a kernel that
                           * uses scratch) */
  int32_t graph_chunk;    /* epochs per captured graph; 0 = 8 */
  uint32_t flags;         /* TREES_F_* */
  double timeout_s;       /* PERSISTENT barrier spin limit in seconds; 0 = 60; also how long an
                           * asynchronous run may stay idle (no live tree) before it ends */
} trees_config;

/* Built-in task programs (their task bodies are compiled into the library). */
typedef enum {
  TREES_PROG_FIB_I32 = 1,   /* naive Fibonacci, 32-bit sums (Section 6.2) */
  TREES_PROG_FIB_I64 = 2,   /* naive Fibonacci, 64-bit sums */
  TREES_PROG_MSORT_U32 = 3, /* split-in-halves merge sort of uint32 keys (Section 6.4) */
  TREES_PROG_NQUEENS = 4,   /* N-queens solution count, one task per partial placement (Section 6.5) */
  TREES_PROG_BFS_CSR = 5,   /* task-per-vertex breadth-first search over CSR (Section 6.3) */
  TREES_PROG_POSTORDER = 6, /* postorder traversal of a binary tree (Figure 2, Section 5.3) */
  TREES_PROG_SSSP_CSR = 7,  /* single-source shortest paths by relaxation over CSR (Section 6.3) */
  TREES_PROG_PREORDER = 8,  /* preorder traversal of a binary tree (Figure 2) */
  TREES_PROG_FFT = 9        /* radix-2 FFT of complex fp32 data (Section 6.2) */
} trees_builtin;

typedef struct {
  void *ptr;       /* device pointer, caller-owned */
  uint64_t bytes;
} trees_buf;

typedef struct {
  int32_t status;          /* TREES_OK, TREES_E_PENDING or the tree's error */
  uint32_t epochs;         /* epochs the tree executed (its critical path, Section 4.4.1) */
  uint64_t tasks;          /* valid task executions, join continuations included (its work) */
  uint64_t launched;       /* lanes launched over all its epochs (valid + invalid entries) */
  uint64_t peak_entries;   /* high-water mark of nextFreeCore (its space, Section 4.4.2) */
  int64_t start_epoch;     /* global epoch of its first epoch (batched schedulers) */
  int64_t done_epoch;      /* global epoch in which it finished */
} trees_tree_stats;

typedef struct {
  uint64_t global_epochs;  /* epochs executed by this run */
  uint64_t tasks;          /* valid tasks of trees that finished in this run */
  int32_t stop_reason;     /* 1 drained, 2 epoch budget, 3 abort, 4 barrier timeout,
                            * 5 an asynchronous run idle for timeout_s */
  int32_t live;            /* trees still live after the run */
  double seconds;          /* host wall time of the run */
  int32_t grid;            /* work-groups of the batched launch (0 for PLAIN) */
  int32_t api_blocks_per_cu; /* co-resident work-groups per CU of that kernel */
  int32_t sched;           /* the scheduler that ran (AUTO resolved) */
  int32_t wg_size;         /* its work-group size */
} trees_run_stats;

/* A launch shape: what the tuner chooses and AUTO applies. */
typedef struct {
  int32_t sched;           /* TREES_SCHED_PLAIN, _GRAPH or _PERSISTENT */
  int32_t wg_size;         /* 256, 512 or 1024 */
  int32_t blocks_per_cu;   /* 0 = automatic */
  int32_t graph_chunk;     /* 0 = the context's */
} trees_shape;

typedef struct {
  int32_t epoch, cen, b, e, launched, valid, forks, joins, nfc;
} trees_epoch_rec;

/* Create a context on cfg->device.  *out receives the context.  Allocates the
 * task vector (unless cfg->arena_base is given), the per-tree descriptors,
 * stacks and scheduler state in device memory.  Errors: INVALID, DEVICE,
 * NOMEM. */
trees_status trees_create(const trees_config *cfg, trees_ctx **out);

/* Destroy a context and free what the library allocated (not caller buffers). */
void trees_destroy(trees_ctx *ctx);

/* Message describing the last error of ctx (or of trees_create when ctx is NULL). */
const char *trees_last_error(const trees_ctx *ctx);

/* Register a built-in program.  Its task types receive a slice of the
 * context's global type ids 1..NumTaskTypes (the encoding of Section 5.1.2
 * needs NumTaskTypes fixed before the first epoch), so every program must be
 * registered before the first trees_submit (else STATE).  Registering a kind
 * twice returns the same id.  *out_prog receives the program id. */
trees_status trees_register_program(trees_ctx *ctx, int32_t kind, int32_t *out_prog);

/* Submit one task tree: its root task is placed in entry 0 of a fresh arena of
 * the task vector and runs in epoch 0 (Section 5.2.1).
 *   FIB_I32 / FIB_I64: args = {n}, 0 <= n <= 43; no buffers.
 *   NQUEENS:           args = {n}, 1 <= n <= 14; no buffers.
 *   MSORT_U32:         args = {N}, 0 <= N < 2^31; bufs = {keys[N] (sorted in place), tmp[N]}
 *                      (the pointers may be NULL when N = 0).
 *   BFS_CSR:           args = {V, source}; bufs = {row_ptr[V+1], col_idx[E], depth[V] (out)}
 *                      int32 CSR; depth receives hop counts, -1 = unreachable.
 *   SSSP_CSR:          args = {V, source[, max_entries[, delta]]}; bufs = {row_ptr[V+1], col_idx[E],
 *                      weights[E], dist[V] (out)} int32, weights >= 0 and every distance
 *                      below 2^31 - 1.  visit(v) lowers the distance of each out-neighbour
 *                      it improves (atomic min) and forks a visit of it; dist receives the
 *                      shortest distances, 2^31 - 1 = unreachable.  A vertex is visited once
 *                      per improvement, so the task count depends on the schedule: the arena
 *                      holds max_entries entries (default 8 V) and a run that needs more
 *                      ends the tree with OVERFLOW (max_entries 0: the default).  A visit
 *                      forked by a distance that has since dropped returns at once (a later
 *                      visit relaxes the arcs).  delta > 0 (< 2^24) sets a bucket width: a
 *                      visit forked with distance d runs only in an epoch whose CEN satisfies
 *                      d < (CEN + 1) * delta, and until then forks itself unchanged (fewer
 *                      repeated relaxations for more, cheap, waiting tasks; the arena must
 *                      then hold the waiting copies too).
 *   POSTORDER:         args = {n, root}, 1 <= n < 2^24, -1 <= root < n (-1: the empty tree);
 *                      bufs = {left[n], right[n], log[n+1] (out)} int32; left/right hold each
 *                      node's children, -1 = none.  postorder(node) forks postorder(right),
 *                      postorder(left) and joins a visit of node; a visit appends the node to
 *                      log (log[n] counts the visits; the library zeroes it at the next
 *                      trees_run, before the tree's first epoch).  Nodes
 *                      must form a tree under root (each reachable node has one parent).
 *                      The arena holds 2n+1 entries (every postorder task, null children
 *                      included).
 *   PREORDER:          args and bufs as POSTORDER.  preorder(node) appends node to log, then
 *                      forks preorder(right), preorder(left); nothing joins, so a node is
 *                      visited in the epoch of its depth (the log goes level by level).
 *   FFT:               args = {log2 N}, 0 <= log2 N <= 20; bufs = {x[N], y[N] (out)}, complex
 *                      fp32 interleaved (re, im), not overlapping.  y receives the DFT of x,
 *                      y[k] = sum_j x[j] exp(-2 pi i jk / N) (no scaling), by recursive radix-2
 *                      decimation in time: FFT(lo, o, ls) transforms x[o + j 2^ls], j < n =
 *                      N / 2^ls, into y[lo, lo + n); n <= 64 is a leaf (a wavefront runs its
 *                      butterflies), otherwise it forks the even and odd halves and joins a
 *                      combine of n/2 butterflies with twiddles exp(-2 pi i k / n), which the
 *                      work-groups expand co-operatively.  x is not modified.  The arena holds
 *                      2 max(1, N/64) - 1 entries.
 * A program's output buffers must not overlap its input buffers (INVALID
 * otherwise; msort's keys and tmp must not overlap either).
 * The arena is sized to the exact task-vector bound of the tree, rounded up to
 * a multiple of 64 entries (arenas start on 64-entry boundaries); if it does
 * not fit in the free budget the call returns NOMEM and changes nothing (the
 * caller may retry once other trees have been collected).  Buffers must stay
 * alive and unmodified until trees_results returns OK for the tree.  The tree
 * becomes live at the next trees_run.  *out_tree receives its id.
 * While an asynchronous run is active (trees_run with TREES_RUN_ASYNC) the
 * call may come from any host thread: the tree is published into a lock-free
 * admission ring in host-mapped memory, which the running kernel reads at
 * every epoch boundary; the kernel then places the root (Section 5.2.1),
 * initialises the BFS depth / SSSP distance / visit counter on the device
 * and runs the tree from the next epoch on, beside the trees already live.
 * The caller's writes to the payload must have completed (its stream
 * synchronised) before the call. */
trees_status trees_submit(trees_ctx *ctx, int32_t prog, const int64_t *args, int32_t nargs,
                          const trees_buf *bufs, int32_t nbufs, uint64_t *out_tree);

/* Run epochs until no tree is live, trees_abort is called, or max_epochs
 * epochs have run (< 0: no limit).  Each epoch is Phase 1, 2 and 3 of
 * Section 4.3 over every live tree; a tree ends when its stack of pending
 * ranges is empty (Section 4.3.3).  Blocking.  A tree that is stopped by the
 * budget keeps its state and continues at the next trees_run.  out may be
 * NULL.  flags: 0 or TREES_RUN_ASYNC.
 *
 * TREES_RUN_ASYNC (PERSISTENT or AUTO scheduler; INVALID otherwise) launches
 * the persistent kernel and returns at once: trees_submit may then be called
 * concurrently (trees join the shared epochs at the next epoch boundary),
 * and finished trees come back through a completion ring that trees_poll
 * and trees_results read, without stopping the kernel.  With no tree live,
 * the kernel waits for submissions in slices of 2 ms (empty epochs, not
 * counted) and ends by itself after timeout_s idle (stop_reason 5), on
 * trees_abort, or at max_epochs.  The next blocking trees_run closes the run:
 * the kernel finishes every live and submitted tree, then returns; that call
 * reports the whole asynchronous run in *out (max_epochs is not used).
 * STATE if an asynchronous run is already active.  While one is active,
 * trees_trace, trees_epoch_times, trees_debug_phases, trees_set_schedule
 * and the worklist calls return STATE. */
trees_status trees_run(trees_ctx *ctx, int64_t max_epochs, uint32_t flags, trees_run_stats *out);

/* Result of one tree.  Returns PENDING while it is live, its error if it
 * failed, OK otherwise.  *out_value receives the value the root task emitted
 * into its own entry (Section 4.3.2, emit; fib: F(n); nqueens: the count;
 * msort and BFS: 0, their output is in the caller's buffers).  OK and errors release the tree's slot and arena: the id
 * is invalid afterwards.  Either output pointer may be NULL. */
trees_status trees_results(trees_ctx *ctx, uint64_t tree, int64_t *out_value,
                           trees_tree_stats *out_stats);

/* Ids of finished trees (their results ready), each reported once, oldest
 * first: at most cap ids into ids, their number in *n.  During an
 * asynchronous run it takes in the completion ring first.  Trees already
 * released by trees_results are skipped. */
trees_status trees_poll(trees_ctx *ctx, uint64_t *ids, int32_t cap, int32_t *n);

/* Per-epoch records of a tree run with TREES_F_TRACE (at most 256 epochs).
 * Copies up to cap records into out and stores the count in *n.  Call before
 * trees_results releases the tree. */
trees_status trees_trace(trees_ctx *ctx, uint64_t tree, trees_epoch_rec *out, int32_t cap,
                         int32_t *n);

/* Device time of epoch launches measured with HIP events recorded on the
 * context's stream around each launch (needs TREES_F_PROFILE).  out[k] for
 * k = 1..5 accumulates the plain scheduler's per-epoch launches of program
 * kind k (trees_builtin); out[0] accumulates batched launches (one graph
 * replay or one persistent launch each); out[6] and out[7] the plain
 * scheduler's map phase (Section 4.2): its partition-pass and merge-pass
 * launches; out[8], out[9] and out[10] the plain scheduler's traversal
 * (POSTORDER, PREORDER), SSSP_CSR and FFT epochs.  Copies min(n, 11) entries. */
typedef struct {
  double ms;           /* summed launch durations */
  uint64_t launches;   /* number of timed launches */
} trees_ktime;
trees_status trees_kernel_times(trees_ctx *ctx, trees_ktime *out, int32_t n);

/* Choose which launches trees_kernel_times covers: bit k set = time the
 * launches that accumulate in out[k] (all eleven by default).  Each timed
 * launch carries two HIP events, which cost host time per launch, so a
 * throughput measurement times only the launches it reports.  STATE if the
 * context was created without TREES_F_PROFILE. */
trees_status trees_profile_mask(trees_ctx *ctx, uint32_t mask);

/* Device-clock duration of each epoch of the last GRAPH or PERSISTENT run,
 * in microseconds, measured from the device's constant-rate clock where the
 * last work-group of each epoch builds the next work list (it includes the
 * epoch's barrier and any map phase).  Copies up to cap values (at most 256)
 * and stores the number of epochs in *n. */
trees_status trees_epoch_times(trees_ctx *ctx, double *us, int32_t cap, int32_t *n);

/* Debug (TREES_F_DEBUG): summed work-group time, in microseconds, spent in
 * each phase of the batched epoch sweep since the context was created:
 * 0 locate, 1 fetch + bodies, 2 fork allocation, 3 child and own writes,
 * 4 BFS arc expansion, 5 per-tree bookkeeping, 6 between chunks and the
 * barrier, 7 barrier (including the scan and map phases).  Copies min(n, 8). */
trees_status trees_debug_phases(trees_ctx *ctx, double *us, int32_t n);

/* Request that a running trees_run stop at the next epoch boundary.  Safe to
 * call from another host thread. */
trees_status trees_abort(trees_ctx *ctx);

/* Change the scheduler and launch shape for later runs (used by the tuner). */
trees_status trees_set_schedule(trees_ctx *ctx, int32_t sched, int32_t wg_size,
                                int32_t blocks_per_cu, int32_t graph_chunk);

/* Exact task-vector entries a tree of `kind` with `args` can occupy at once.
 * Admission charges this rounded up to a multiple of 64.  Host-only. */
trees_status trees_tv_bound(int32_t kind, const int64_t *args, int32_t nargs, int64_t *entries);

/* The tuned shape for a device name (hipDeviceProp_t::name) and a workload
 * class, read from the tuned file at `path` (NULL: $TREES_TUNE_FILE, else
 * $HOME/.cache/trees/tuned.txt).  The file holds one shape per line:
 * device TAB class TAB "sched wg_size blocks_per_cu graph_chunk"; the last
 * line for a (device, class) pair wins and lines that do not parse are
 * skipped.  OK and *out filled if a shape was found, INVALID otherwise.
 * Host-only. */
trees_status trees_tuned_shape(const char *path, const char *device, const char *wclass, trees_shape *out);

/* The workload class of a context, as the tuned file keys it: the kinds of
 * its registered programs (trees_builtin numbers), ascending, joined by '+'
 * ("2+4" for FIB_I64 and NQUEENS).  Copies at most cap bytes, NUL included. */
trees_status trees_workload_class(const trees_ctx *ctx, char *buf, int32_t cap);

/* ---------------------------------------------------------------------------
 * Native worklist BFS and SSSP: the hand-managed formulation that Section 6.3
 * compares TREES with.  Each iteration is one kernel over an input worklist
 * of vertices; every vertex relaxes its out-arcs (BFS: a head at depth -1 is
 * claimed by compare-and-swap to level + 1; SSSP: a head's distance is lowered
 * by an atomic min) and pushes each head it claims or improves to the output
 * worklist through one atomically advanced tail counter (an SSSP head at most
 * once per iteration).  After each kernel the host reads back that one count;
 * the lists swap and the next kernel covers the old output list, until an
 * iteration pushes nothing.  The kernels run on the context's stream with its
 * work-group size and the host polls host-mapped memory for the count, as the
 * PLAIN scheduler does for its epoch counters.
 *
 * Workspace: caller-owned device memory of at least trees_wl_workspace_bytes
 * bytes, 256-byte aligned, not overlapping the output; it holds the two
 * worklists (V int32 each), the SSSP push stamps (V int32) and 256 bytes of
 * counters, and may be reused between calls (not concurrently).
 * Errors: INVALID (bad sizes, null pointers, workspace too small or
 * misaligned, output overlapping it), STATE (an asynchronous trees_run is
 * active), DEVICE.  Blocking: returns when the last iteration has finished.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t iterations;      /* relaxation kernels launched (the last pushes nothing) */
  int32_t pad;
  uint64_t pushed;         /* vertices pushed to output worklists, all iterations */
  double seconds;          /* host wall time of the call */
} trees_wl_stats;

/* Workspace bytes for a graph of V vertices (sssp != 0: with the stamps). */
trees_status trees_wl_workspace_bytes(int32_t V, int32_t sssp, uint64_t *bytes);

/* BFS from source: depth[V] (out) receives hop counts, -1 = unreachable.
 * int32 CSR row_ptr[V + 1], col_idx[E] (device pointers). */
trees_status trees_wl_bfs(trees_ctx *ctx, int32_t V, int32_t source, const int32_t *row_ptr,
                          const int32_t *col_idx, int32_t *depth, void *ws, uint64_t ws_bytes,
                          trees_wl_stats *out);

/* SSSP from source with int32 weights[E] >= 0 (every distance below 2^31 - 1):
 * dist[V] (out) receives shortest distances, 2^31 - 1 = unreachable. */
trees_status trees_wl_sssp(trees_ctx *ctx, int32_t V, int32_t source, const int32_t *row_ptr,
                           const int32_t *col_idx, const int32_t *weights, int32_t *dist, void *ws,
                           uint64_t ws_bytes, trees_wl_stats *out);

/* trees_wl_bfs for callers that cannot allocate memory at call time (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the worklists and counters live in a fixed array of device
 * memory inside the library (32 MiB + 256 B on every GPU it runs on, held
 * until the process ends) instead of a caller's workspace.  Graphs of at most
 * 2^22 vertices (INVALID above).  The call allocates nothing: no device, host
 * or pinned memory.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (each call initialises what it reads), so
 * calls that overlap on one GPU -- from different contexts or threads --
 * race; calls through one context are serialised.  Results, statistics and
 * other errors as trees_wl_bfs. */
trees_status trees_wl_bfs_noalloc(trees_ctx *ctx, int32_t V, int32_t source, const int32_t *row_ptr,
                                  const int32_t *col_idx, int32_t *depth, trees_wl_stats *out);

/* Free task-vector entries of the budget (for admission decisions). */
int64_t trees_free_entries(const trees_ctx *ctx);

/* Number of submitted trees not yet released by trees_results. */
int32_t trees_num_trees(const trees_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TREES_H */
