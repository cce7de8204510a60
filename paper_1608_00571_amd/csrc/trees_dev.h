// Device-side state of the TREES runtime, shared by the host library and the
// HIP kernels.  All layouts are plain structs in HBM.
//
// Task vector (Section 5.1.2): structure-of-arrays, one slot per TVM core.
//   code[i]  = epoch * NumTaskTypes + type   (0 = invalid / finished)
//   a0..a3[i] = task arguments (int32)
//   r[i]     = the value an emitting task leaves in its own entry (int64)
// Each tree owns a contiguous arena [base, base + cap) of the task vector;
// all indices stored inside the task vector are arena-relative.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace trees {

constexpr int kMapTile = 4096;     // map phase inside the persistent kernel: merged keys per tile
// standalone map launches (plain and graph forms): work-group size and
// keys per tile (8 a lane)
constexpr int kMapWG = 1024;
constexpr int kMapLaunchTile = 8192;
constexpr int kMapBlocksPerCU = 16;   // plain form: merge work-groups per CU at most (one tile each)
constexpr int kChunkItems = 1024;  // work items per work-group chunk of an epoch
constexpr int kMaxTypes = 31;     // global task-type ids 1..NTT, NTT <= 31
constexpr int kStackMax = 128;    // stack records per tree
constexpr int kTraceMax = 256;    // per-epoch trace records per tree
constexpr int kLeaf = 64;         // merge-sort ranges of <= 64 keys are leaves

// Operations a task type can run.
enum Op : int32_t {
  OP_NONE = 0,
  OP_FIB32 = 1, OP_SUM32 = 2,
  OP_FIB64 = 3, OP_SUM64 = 4,
  OP_MS = 5, OP_MERGE = 6,
  OP_Q = 7, OP_QSUM = 8,
  OP_VISIT = 9,
  OP_POST = 10, OP_PVISIT = 11,
  OP_SVISIT = 12,
  OP_PRE = 13,
  OP_FFT = 14, OP_COMB = 15,
  OP_COUNT = 16
};
constexpr uint32_t opbit(int op) { return 1u << op; }
constexpr uint32_t OPS_FIB = opbit(OP_FIB32) | opbit(OP_SUM32) | opbit(OP_FIB64) | opbit(OP_SUM64);
constexpr uint32_t OPS_NQ = opbit(OP_Q) | opbit(OP_QSUM);
constexpr uint32_t OPS_MS = opbit(OP_MS) | opbit(OP_MERGE);
constexpr uint32_t OPS_BFS = opbit(OP_VISIT);
constexpr uint32_t OPS_PO = opbit(OP_POST) | opbit(OP_PVISIT) | opbit(OP_PRE);   // tree traversals
constexpr uint32_t OPS_SSSP = opbit(OP_SVISIT);
constexpr uint32_t OPS_GRAPH = OPS_BFS | OPS_SSSP;   // arcs
constexpr uint32_t OPS_FFT = opbit(OP_FFT) | opbit(OP_COMB);
constexpr uint32_t OPS_EXPAND = OPS_GRAPH | OPS_FFT;   // kernels with the co-operative expansion
constexpr uint32_t OPS_ALL = OPS_FIB | OPS_NQ | OPS_MS | OPS_BFS | OPS_PO | OPS_SSSP | OPS_FFT;
constexpr int kFftLeafLog = 6;      // FFT tasks of at most 2^6 points are leaves (one wavefront)
constexpr int kFftMaxLog = 20;      // largest FFT: 2^20 points (a chunk's butterflies stay below 2^31)

// Tree status values (TreeState::status).
enum : int32_t { TS_FREE = 0, TS_LIVE = 1, TS_DONE = 2, TS_PAUSED = 3 };
// Error flags raised by kernels (TreeHot::flags, atomic OR).
enum : int32_t { TF_OVERFLOW = 1, TF_ENCODING = 2, TF_STACK = 4 };

// Immutable per-tree descriptor (written at submit).
struct TreeStatic {
  int64_t base;      // arena offset in task-vector entries
  int32_t cap;       // arena capacity in entries
  int32_t tbase;     // global type id of the program's first type
  int32_t kind;      // trees_builtin
  int32_t p0, p1;    // fib n | nqueens n | msort N | bfs, sssp V, source | traversal n, root | fft log2 N
  uint32_t tp;       // tbase | parameter << 8 (nqueens n, traversal n, fft log2 N, sssp bucket
                     // width), as the work list carries it
  // msort: keys, tmp; bfs: row_ptr, col_idx, depth; sssp: row_ptr, col_idx,
  // dist, weights; postorder, preorder: left, right, log; fft: x, y
  uint64_t ptr0, ptr1, ptr2, ptr3;
};

// Per-tree counters updated with device-scope atomics during an epoch.
// One 64-byte block per tree so trees never share a line.
struct alignas(64) TreeHot {
  int32_t nfc;        // nextFreeCore, arena-relative
  int32_t flags;      // TF_* error bits
  uint64_t done;      // items finished this epoch (low 32) | joins (high 32)
  int32_t valid;      // valid tasks executed this epoch
  int32_t pad[11];
};

// Per-tree scheduler state.  Written only by the work-group that finishes
// the tree's epoch, read across the epoch barrier.
struct alignas(128) TreeState {
  int32_t cen, b, e, old;    // current epoch number and range, oldNextFreeCore
  int32_t sp;                // stack depth
  int32_t status;            // TS_*
  int32_t err;               // 0 or a trees_status error code
  int32_t epochs;            // epochs executed
  int64_t tasks;             // valid task executions, counted per epoch
  int64_t launched;          // lanes launched over all epochs
  int64_t result;            // r[root] once done
  int64_t done_gepoch;       // global epoch at completion
  int64_t start_gepoch;      // global epoch of the first executed epoch (-1: not started)
  int32_t peak;              // high-water mark of nfc
  int32_t ntrace;            // trace records written
  int32_t pad[8];
};

struct TraceRec {
  int32_t epoch, cen, b, e, launched, valid, forks, joins, nfc;
};

// Scheduler header.  The barrier words sit on their own cache lines.
struct SchedHdr {
  uint32_t S;           // items in the current work list
  int32_t L;            // work-list entries
  int32_t stop;         // non-zero: kernels exit at the next epoch boundary
  int32_t live;         // live trees after the last scan
  int64_t gepoch;       // global epochs executed by this context
  int64_t run_epochs;   // epochs executed in the current run
  int64_t max_epochs;   // budget of the current run (< 0: none)
  int32_t done_count;   // trees finished in the current epoch (done_list length)
  int32_t stop_reason;  // 1 = drained, 2 = epoch budget, 3 = abort, 4 = timeout
  int32_t tslots;       // slots [0, tslots) may hold trees
  uint32_t mapJ;        // map jobs registered by the last epoch (raw count)
  int32_t initN;        // asynchronous run: adopted trees whose buffers the next epoch initialises
  uint32_t adm_head;    // asynchronous run: admission records adopted so far
  uint32_t ctail;       // asynchronous run: completion records written so far
  uint32_t ctail_pub;   // asynchronous run: completion records published to the host
  int64_t idle_t0;      // asynchronous run: device clock when no tree was left live (0: busy)
  uint32_t pub_seq;     // captured chains published to the host mirror (HdrMirror::seq)
  int32_t pad0[7];
  alignas(128) uint32_t arrive;   // barrier arrivals of the last work-group of each group
  int32_t pad1[31];
  struct alignas(128) Grp { uint32_t n; int32_t pad[31]; } grp[8];   // per-group arrivals (blockIdx % 8)
  int32_t wsel;                   // which of the two work-list buffers is current
  int32_t pad4[31];
  // Appends to the next epoch's work list: (entries << kWlShift) | items.
  // A tree's Phase 3 appends its next range; the end-of-epoch scan reads
  // the total and clears it.
  alignas(128) uint64_t wl_next;
  int32_t pad9[30];
  alignas(128) uint32_t gen;      // barrier generation
  int32_t pad2[31];
  alignas(128) uint64_t map_ctr;  // (jobs << 38) | units, appended during an epoch
  uint32_t map_arrive;            // work-groups done with the map launch
  int32_t pad3[29];
  alignas(128) uint32_t chunk_ctr;  // next chunk of the current epoch to hand out
  int32_t pad5[31];
  alignas(128) uint32_t arc_jobs;   // arc jobs published this epoch
  uint32_t arc_tiles;               // their tiles
  uint32_t arc_segs;                // their segment records
  int32_t pad6[29];
  alignas(128) uint32_t arc_next;   // next arc tile to hand out in the arc phase
  int32_t pad7[31];
  alignas(128) uint32_t arc_arrive; // work-groups done with the arc launch (graph form)
  int32_t arc_phase;                // 1: the epoch's arc phase is pending (the scan waits for it)
  int32_t pad8[30];
  int64_t stamp0;                 // device clock when the run's first work list was built
  int64_t stamp[256];             // device clock at the end of each epoch of the run
  uint64_t phase[8];              // debug: summed work-group time per chunk phase (device clock)
};
constexpr int kEpochStamps = 256;

// A map counter packs the job count (high 26 bits) and the job units (low
// 38 bits) so one atomic add per work-group reserves both, and job indices
// and unit offsets grow in the same order.
constexpr int kMapShift = 38;
// The work-list append counter: entries in the high 24 bits, items in the
// low 40 (entry indices and item offsets grow in the same order).
constexpr int kWlShift = 40;
constexpr uint64_t kWlItemMask = (1ull << kWlShift) - 1;
constexpr uint64_t kMapUnitMask = (1ull << kMapShift) - 1;

// Counters used by the plain scheduler (double-buffered by epoch parity, so
// the host never has to clear them: epoch k clears the other parity).
struct PlainCounters {
  uint64_t fj[2];      // forks (low 32 bits) | joins (high 32 bits): one atomic per work-group
  int32_t valid[2];
  int32_t flags[2];
  uint64_t map[2];
  alignas(128) uint32_t ticket;   // work-groups of the epoch that have finished (own line)
};

// Arc phase (BFS VISIT, Tenet 2 across work-groups, batched forms).  A chunk
// whose VISIT items have more than kArcLocal arcs does not expand them: it
// publishes them as a job of tiles and leaves its retirement to the job.
// After the epoch's chunks, every work-group claims tiles; the work-group
// that finishes a job's last tile retires the owner chunk's items.  The
// owner records, for each of its tiles, the job and the items the tile's
// arcs come from.
constexpr int kArcJobs = 8192;      // jobs per epoch (beyond: the owner expands locally)
constexpr int kArcTile = 2048;      // arcs per tile (larger jobs use larger tiles)
constexpr int kArcTilesMax = 64;    // tiles per job of arcs
constexpr int kBflyTilesMax = 1024; // tiles per job with FFT butterflies (cheap, uniform units)
constexpr int kArcTilesAll = 1 << 18;   // tiles per epoch
constexpr int kArcSegPool = 1 << 16;    // segment records per epoch
constexpr int kArcLocal = 16384;    // chunks with at most this many arcs expand locally
struct alignas(64) ArcJob {
  int32_t tot;       // arcs of the job
  int32_t tile;      // arcs per tile
  int32_t ntiles;
  int32_t nseg;      // segments (trees) of the owner's chunk
  uint32_t tbase;    // global number of the job's first tile
  uint32_t done;     // tiles expanded
  uint32_t sbase;    // first segment record of the job in the pool
  int32_t pad[9];
};
// Per job: item arrays pre, row, seg, dv (kChunkItems each, lane-major order
// of the owner chunk; dv: an SSSP item's distance, -1 for BFS, -(ls + 2) for
// an FFT combine of level ls, whose row is its first output).  Per segment, a record in the pool's seven planes: slot,
// cen, tb, tp, items (retired by the job), range (the segment's items this
// epoch) and jv (joins | valid << 16).
constexpr int kArcItemWords = 4 * kChunkItems;

// Host-visible copy of one epoch's counters (host-mapped, coherent memory),
// written after the epoch; `seq` is written last and names the launch, so
// the host can wait on it instead of on the stream.
struct PlainMirror {
  uint64_t fj;
  uint64_t map;
  int32_t valid;
  int32_t flags;
  uint32_t seq;
  uint32_t pad;
};

// Host-visible copy of the header's first 64 bytes (S .. adm_head), written
// at the end of each captured chain of epochs; `seq` is written last and
// counts the chains, so the host polls it instead of copying the header back
// and synchronising the stream.
struct HdrMirror {
  int32_t hdr[16];
  uint32_t seq;
  uint32_t pad[15];
};
static_assert(offsetof(SchedHdr, ctail) == sizeof(HdrMirror::hdr), "the mirrored part of the header");

// ---------------------------------------------------------------------------
// Asynchronous runs (TREES_RUN_ASYNC): trees submitted while a persistent
// run is in flight arrive through an admission ring in host-mapped memory,
// and finished trees leave through a completion ring beside it.  Each ring
// has one slot per tree slot, so neither can overflow: a record is written
// only for a tree slot that is in use, and a slot is reused only after the
// host has consumed its completion.
// ---------------------------------------------------------------------------
struct Completion {
  int32_t slot, err, epochs, peak;
  int64_t tasks, launched, result, start_gepoch, done_gepoch;
  int64_t pad;
};

struct alignas(64) AsyncRing {
  uint32_t tail;        // host: admission records published
  uint32_t head;        // device: admission records adopted (for the host's information)
  uint32_t ctail;       // device: completion records published
  int32_t close;        // host: end the run once no tree is live and nothing waits
  int32_t pad[12];
};

// One staged submission, applied on the device by the admission kernel
// (or, in an asynchronous run, adopted from the admission ring).
struct Admit {
  int32_t slot, root_code, a0, a1, a2, a3;
  TreeStatic ts;
};

// Everything a kernel needs, passed by value.
struct DevCtx {
  int32_t *code, *a0, *a1, *a2, *a3;
  int64_t *r;
  const TreeStatic *ts;
  TreeState *st;
  TreeHot *hot;
  int32_t *t_len, *t_cen, *t_b;   // next-epoch range per tree (finisher -> scan)
  int4 *stack;                    // [slot * kStackMax + k] = {cen, b, e, cend}
  TraceRec *trace;                // [slot * kTraceMax + k] or null
  // Work list, two buffers of tmax + 1 entries each (hdr->wsel: the
  // current one; the epoch's Phase 3 appends the next epoch's to the other)
  int32_t *wl_tree;               // work list: tree slot
  uint32_t *wl_off;               // exclusive prefix of range lengths (L+1 entries)
  int32_t *wl_b;                  // arena-relative range start
  int32_t *wl_cen;                // epoch number of the entry
  uint32_t *wl_tb;                // arena base / 64 (arenas are 64-entry aligned)
  uint32_t *wl_tp;                // the tree's first type id | program parameter << 8 (nqueens n)
  int32_t *done_list;             // trees finished in this epoch
  int32_t tmax;
  int32_t pad3;
  SchedHdr *hdr;
  PlainCounters *plain;
  PlainMirror *mirror;            // device address of the host-mapped mirror
  const volatile int32_t *abort_flag;  // host-pinned, set by trees_abort
  int32_t ntt;
  int32_t trace_on;
  int32_t debug;
  int32_t pad;
  int64_t timeout_ticks;          // spin limit at the grid barrier (100 MHz clock ticks)
  // map jobs (data-parallel merges registered by MERGE continuations)
  int32_t *mj_lo, *mj_hi;         // key range [lo, hi); the halves split at lo + (hi - lo) / 2
  const uint32_t **mj_src;        // buffer holding the two sorted halves
  uint32_t **mj_dst;              // buffer receiving the merged range
  uint64_t *mj_off;               // first unit (output key) of the job
  uint32_t *part_job;             // per tile boundary: job containing the boundary unit
  int64_t *part_ia;               // per tile boundary: first-half keys before it (merge path)
  int32_t mj_cap;                 // 0: map disabled, merges run serially in their lane
  int32_t part_cap;               // tile boundaries the partition arrays hold
  ArcJob *arc_job;                // [kArcJobs]
  int32_t *arc_item;              // [kArcJobs * kArcItemWords]
  int32_t *arc_seg;               // [7 * kArcSegPool]: the segment record planes
  int4 *arc_tile;                 // [kArcTilesAll]: {job, first item, last item, -}
  // asynchronous runs (async_mode != 0 only in the persistent launch of one)
  AsyncRing *ring;                // device address of the host-mapped ring header
  const Admit *ring_adm;          // [tmax] admission records (host-mapped)
  Completion *ring_done;          // [tmax] completion records (host-mapped)
  int32_t *init_slot;             // [tmax] adopted trees whose buffers need initialising
  int32_t async_mode;
  int32_t pad4;
  int64_t slice_ticks;            // idle wait for a submission before an empty epoch
  int64_t idle_ticks;             // idle time after which the run ends by itself
  const DevCtx *self;             // a copy of this struct in device memory (for out-of-line code)
  uint8_t op_of_type[kMaxTypes + 1];
};


// Arguments of one plain-scheduler epoch (one tree, host-driven).
struct PlainArgs {
  int32_t slot, cen, b, e, nfc0, par;
  uint32_t seq;   // launch number published in the mirror
  uint32_t tb;    // the tree's arena base / 64
  uint32_t tp;    // its first type id | program parameter << 8 (nqueens n)
  uint32_t nwg;   // work-groups of the launch (the last to finish publishes); set by the launcher
};


// ---------------------------------------------------------------------------
// Native worklist BFS / SSSP (the hand-managed comparison of Section 6.3)
// ---------------------------------------------------------------------------
constexpr int kWlChunk = 1024;   // worklist entries per work-group
// The allocation-free worklist BFS keeps its workspace (256 B of counters
// and two worklists of V int32, 256-byte aligned sections) in a fixed device
// array: graphs of up to 2^22 vertices.
constexpr int32_t kWlScratchMaxV = 1 << 22;
constexpr size_t kWlScratchBytes = 256 + 2 * (size_t)kWlScratchMaxV * 4;

// Control words of one worklist run (in the caller's workspace, 256 B).
struct alignas(128) WlCtl {
  uint32_t tail[2];      // output-list counters, by iteration parity
  uint32_t pad0[30];
  uint32_t ticket;       // work-groups of the iteration that have finished
  uint32_t pad1[31];
};

// Host-mapped copy of an iteration's output count; `seq` is written last.
struct WlMirror {
  uint32_t count;
  uint32_t seq;
};

struct WlArgs {
  const int32_t *row;      // CSR row pointers [V + 1]
  const int32_t *col;      // CSR heads [E]
  const int32_t *w;        // SSSP arc weights [E] (null for BFS)
  int32_t *val;            // BFS depth / SSSP distance [V]
  const int32_t *in;       // input worklist
  int32_t *out;            // output worklist
  int32_t *stamp;          // SSSP: iteration that last pushed each vertex [V]
  WlCtl *ctl;
  WlMirror *mir;           // device address of the host-mapped mirror
  uint32_t n_in;           // entries of the input list
  int32_t level;           // iteration number (BFS: the depth of the input vertices)
  int32_t par;             // iteration parity (which tail counter this iteration advances)
  uint32_t seq;            // launch number published in the mirror
  uint32_t nwg;            // work-groups of the launch
  int32_t pad;
};

}  // namespace trees
