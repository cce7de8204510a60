"""TREES epoch runtime for AMD Instinct MI355X -- Python binding.

A thin ctypes layer over ``libtrees.so`` (the C ABI declared in
``include/trees.h``).  Every step of the epoch path runs in the library's
HIP kernels; this module only marshals arguments.  PyTorch supplies device
memory (the task-vector arena and the payload tensors) and nothing else.

The library must be built (``python -m paper_1608_00571_amd.build``); there
is no fallback: importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrees.so")

# status codes
OK, E_INVALID, E_NOMEM, E_OVERFLOW, E_PENDING, E_DEVICE, E_ABORTED, E_STATE, E_ENCODING, E_STACK = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "OVERFLOW", -4: "PENDING", -5: "DEVICE",
                -6: "ABORTED", -7: "STATE", -8: "ENCODING", -9: "STACK"}

# schedulers
PLAIN, GRAPH, PERSISTENT, AUTO = 0, 1, 2, 3
SCHEDS = {"plain": PLAIN, "graph": GRAPH, "persistent": PERSISTENT, "auto": AUTO}

# built-in programs
FIB_I32, FIB_I64, MSORT_U32, NQUEENS, BFS_CSR, POSTORDER, SSSP_CSR, PREORDER, FFT = range(1, 10)
PROGRAMS = {"fib32": FIB_I32, "fib64": FIB_I64, "msort": MSORT_U32, "nqueens": NQUEENS, "bfs": BFS_CSR,
            "postorder": POSTORDER, "sssp": SSSP_CSR, "preorder": PREORDER, "fft": FFT}
SSSP_UNREACHED = 2**31 - 1   # distance of a vertex the source does not reach

F_TRACE, F_DEBUG, F_PROFILE, F_NOMAP = 1, 2, 4, 8
RUN_ASYNC = 1
BYTES_PER_ENTRY = 28


class TreesError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("arena_base", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_uint64), ("max_trees", ctypes.c_int32),
                ("sched", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("graph_chunk", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("timeout_s", ctypes.c_double)]


class _Buf(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("bytes", ctypes.c_uint64)]


class _TreeStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("epochs", ctypes.c_uint32), ("tasks", ctypes.c_uint64),
                ("launched", ctypes.c_uint64), ("peak_entries", ctypes.c_uint64),
                ("start_epoch", ctypes.c_int64), ("done_epoch", ctypes.c_int64)]


class _RunStats(ctypes.Structure):
    _fields_ = [("global_epochs", ctypes.c_uint64), ("tasks", ctypes.c_uint64),
                ("stop_reason", ctypes.c_int32), ("live", ctypes.c_int32), ("seconds", ctypes.c_double),
                ("grid", ctypes.c_int32), ("api_blocks_per_cu", ctypes.c_int32),
                ("sched", ctypes.c_int32), ("wg_size", ctypes.c_int32)]


class _Shape(ctypes.Structure):
    _fields_ = [("sched", ctypes.c_int32), ("wg_size", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("graph_chunk", ctypes.c_int32)]


class _WlStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("pad", ctypes.c_int32), ("pushed", ctypes.c_uint64),
                ("seconds", ctypes.c_double)]


class _KTime(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", ctypes.c_uint64)]


REC_DTYPE = np.dtype([(n, np.int32) for n in
                      ("epoch", "cen", "b", "e", "launched", "valid", "forks", "joins", "nfc")])

_lib = None


def lib():
    """Load libtrees.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1608_00571_amd.build`")
        # torch carries its own ROCm runtime beside the system one this
        # library links; torch's must be loaded first (loaded the other way
        # round, a context's hipSetDevice fails once torch has used the GPU)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        L.trees_create.restype = i32
        L.trees_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(vp)]
        L.trees_destroy.argtypes = [vp]
        L.trees_last_error.restype = ctypes.c_char_p
        L.trees_last_error.argtypes = [vp]
        L.trees_register_program.restype = i32
        L.trees_register_program.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.trees_submit.restype = i32
        L.trees_submit.argtypes = [vp, i32, ctypes.POINTER(i64), i32, ctypes.POINTER(_Buf), i32,
                                   ctypes.POINTER(u64)]
        L.trees_run.restype = i32
        L.trees_run.argtypes = [vp, i64, ctypes.c_uint32, ctypes.POINTER(_RunStats)]
        L.trees_results.restype = i32
        L.trees_results.argtypes = [vp, u64, ctypes.POINTER(i64), ctypes.POINTER(_TreeStats)]
        L.trees_poll.restype = i32
        L.trees_poll.argtypes = [vp, ctypes.POINTER(u64), i32, ctypes.POINTER(i32)]
        L.trees_trace.restype = i32
        L.trees_trace.argtypes = [vp, u64, vp, i32, ctypes.POINTER(i32)]
        L.trees_abort.restype = i32
        L.trees_abort.argtypes = [vp]
        L.trees_set_schedule.restype = i32
        L.trees_set_schedule.argtypes = [vp, i32, i32, i32, i32]
        L.trees_tv_bound.restype = i32
        L.trees_tv_bound.argtypes = [i32, ctypes.POINTER(i64), i32, ctypes.POINTER(i64)]
        L.trees_profile_mask.restype = i32
        L.trees_profile_mask.argtypes = [vp, ctypes.c_uint32]
        L.trees_kernel_times.restype = i32
        L.trees_kernel_times.argtypes = [vp, ctypes.POINTER(_KTime), i32]
        L.trees_epoch_times.restype = i32
        L.trees_epoch_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)]
        L.trees_debug_phases.restype = i32
        L.trees_debug_phases.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32]
        L.trees_free_entries.restype = i64
        L.trees_free_entries.argtypes = [vp]
        L.trees_num_trees.restype = i32
        L.trees_num_trees.argtypes = [vp]
        L.trees_tuned_shape.restype = i32
        L.trees_tuned_shape.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(_Shape)]
        L.trees_workload_class.restype = i32
        L.trees_workload_class.argtypes = [vp, ctypes.c_char_p, i32]
        L.trees_wl_workspace_bytes.restype = i32
        L.trees_wl_workspace_bytes.argtypes = [i32, i32, ctypes.POINTER(u64)]
        L.trees_wl_bfs.restype = i32
        L.trees_wl_bfs.argtypes = [vp, i32, i32, vp, vp, vp, vp, u64, ctypes.POINTER(_WlStats)]
        L.trees_wl_bfs_noalloc.restype = i32
        L.trees_wl_bfs_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, ctypes.POINTER(_WlStats)]
        L.trees_wl_sssp.restype = i32
        L.trees_wl_sssp.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, u64, ctypes.POINTER(_WlStats)]
        _lib = L
    return _lib


EXPORTED = ("trees_create", "trees_destroy", "trees_last_error", "trees_register_program",
            "trees_submit", "trees_run", "trees_results", "trees_trace", "trees_abort",
            "trees_set_schedule", "trees_tv_bound", "trees_free_entries", "trees_num_trees",
            "trees_kernel_times", "trees_profile_mask", "trees_epoch_times", "trees_debug_phases",
            "trees_tuned_shape", "trees_workload_class", "trees_wl_workspace_bytes", "trees_wl_bfs",
            "trees_wl_sssp", "trees_wl_bfs_noalloc", "trees_poll")


@dataclass
class TreeStats:
    status: int
    epochs: int
    tasks: int
    launched: int
    peak_entries: int
    start_epoch: int
    done_epoch: int


@dataclass
class RunStats:
    global_epochs: int
    tasks: int
    stop_reason: int
    live: int
    seconds: float
    grid: int = 0
    api_blocks_per_cu: int = 0
    sched: int = 0
    wg_size: int = 0


def tuned_shape(device: str, wclass: str, path: str | None = None):
    """The tuned file's (sched, wg_size, blocks_per_cu, graph_chunk) for a
    device name and workload class, or None (what AUTO reads)."""
    out = _Shape()
    rc = lib().trees_tuned_shape(path.encode() if path else None, device.encode(), wclass.encode(),
                                 ctypes.byref(out))
    if rc:
        return None
    return (int(out.sched), int(out.wg_size), int(out.blocks_per_cu), int(out.graph_chunk))


@dataclass
class WlStats:
    iterations: int
    pushed: int
    seconds: float


def wl_workspace_bytes(V: int, sssp: bool = False) -> int:
    out = ctypes.c_uint64(0)
    rc = lib().trees_wl_workspace_bytes(V, 1 if sssp else 0, ctypes.byref(out))
    if rc:
        raise TreesError(rc, "trees_wl_workspace_bytes")
    return int(out.value)


def tv_bound(kind: int, args) -> int:
    a = (ctypes.c_int64 * len(args))(*args)
    out = ctypes.c_int64(0)
    rc = lib().trees_tv_bound(kind, a, len(args), ctypes.byref(out))
    if rc:
        raise TreesError(rc, "trees_tv_bound")
    return int(out.value)


def _ptr_bytes(t):
    """(device pointer, bytes) of a torch tensor; must live on the GPU."""
    if not t.is_cuda:
        raise TreesError(E_INVALID, "payload tensors must be on the GPU")
    if not t.is_contiguous():
        raise TreesError(E_INVALID, "payload tensors must be contiguous")
    return t.data_ptr(), t.numel() * t.element_size()


class Context:
    """One TREES context on one GPU: a task-vector budget, up to `max_trees`
    tree slots and a scheduler."""

    def __init__(self, arena_bytes: int = 1 << 30, *, max_trees: int = 4096, sched="persistent",
                 wg: int = 256, blocks_per_cu: int = 0, graph_chunk: int = 8, trace: bool = False,
                 profile: bool = False, nomap: bool = False, debug: bool = False, device: int = 0,
                 timeout_s: float = 0.0):
        import torch
        self._torch = torch
        L = lib()
        self.device = device
        # the task-vector arena is a torch allocation; the library carves it up
        nbytes = (arena_bytes // BYTES_PER_ENTRY) * BYTES_PER_ENTRY + 1024
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{device}")
        cfg = _Config()
        cfg.struct_size = ctypes.sizeof(_Config)
        cfg.device = device
        cfg.stream = None
        cfg.arena_base = self.arena.data_ptr()
        cfg.arena_bytes = arena_bytes
        cfg.max_trees = max_trees
        cfg.sched = SCHEDS[sched] if isinstance(sched, str) else int(sched)
        cfg.wg_size = wg
        cfg.blocks_per_cu = blocks_per_cu
        cfg.graph_chunk = graph_chunk
        cfg.flags = ((F_TRACE if trace else 0) | (F_PROFILE if profile else 0) | (F_NOMAP if nomap else 0)
                     | (F_DEBUG if debug else 0))
        cfg.timeout_s = timeout_s
        h = ctypes.c_void_p(0)
        rc = L.trees_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc:
            raise TreesError(rc, L.trees_last_error(None).decode())
        self.h = h
        self._async = False
        self._keep = {}   # tree id -> payload tensors kept alive until results
        self._progs = {}

    # -- plumbing ---------------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc:
            raise TreesError(rc, f"{what}: {lib().trees_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None):
            # an asynchronous run ends at its next epoch boundary (trees_destroy
            # also requests it); then the device may be synchronised
            if self._async:
                lib().trees_abort(self.h)
            self._torch.cuda.synchronize(self.device)
            lib().trees_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the C ABI ------------------------------------------------------------
    def register(self, kind: int) -> int:
        if kind in self._progs:
            return self._progs[kind]
        out = ctypes.c_int32(0)
        self._check(lib().trees_register_program(self.h, kind, ctypes.byref(out)), "register_program")
        self._progs[kind] = out.value
        return out.value

    def submit(self, prog: int, args, bufs=(), ready: bool = False) -> int:
        """trees_submit.  During an asynchronous run the payload must be on the
        device already: unless `ready`, the current stream is synchronised
        first."""
        if bufs and self._async and not ready:
            self._torch.cuda.current_stream(self.device).synchronize()
        a = (ctypes.c_int64 * max(1, len(args)))(*args)
        pb = [_ptr_bytes(t) for t in bufs]
        b = (_Buf * max(1, len(pb)))(*[_Buf(p, n) for p, n in pb])
        out = ctypes.c_uint64(0)
        rc = lib().trees_submit(self.h, prog, a, len(args), b, len(pb), ctypes.byref(out))
        if rc == E_NOMEM:
            raise TreesError(rc, "task-vector budget or tree slots exhausted")
        self._check(rc, "submit")
        self._keep[out.value] = tuple(bufs)
        return out.value

    def try_submit(self, prog: int, args, bufs=(), ready: bool = False):
        """submit(), but returns None instead of raising when the tree does not fit now."""
        try:
            return self.submit(prog, args, bufs, ready)
        except TreesError as e:
            if e.status == E_NOMEM:
                return None
            raise

    def run(self, max_epochs: int = -1, asynchronous: bool = False) -> RunStats:
        """trees_run.  asynchronous=True starts a persistent run and returns at
        once (submit, poll and results work while it runs); the next blocking
        run() closes it and reports the whole run."""
        self._torch.cuda.current_stream(self.device).synchronize()
        st = _RunStats()
        self._check(lib().trees_run(self.h, max_epochs, RUN_ASYNC if asynchronous else 0, ctypes.byref(st)), "run")
        self._async = asynchronous
        return RunStats(int(st.global_epochs), int(st.tasks), int(st.stop_reason), int(st.live),
                        float(st.seconds), int(st.grid), int(st.api_blocks_per_cu), int(st.sched),
                        int(st.wg_size))

    def results(self, tree: int):
        """(value, TreeStats); raises TreesError(PENDING) if the tree is live,
        or the tree's error.  Releases the tree's slot and arena."""
        v = ctypes.c_int64(0)
        s = _TreeStats()
        rc = lib().trees_results(self.h, tree, ctypes.byref(v), ctypes.byref(s))
        stats = TreeStats(int(s.status), int(s.epochs), int(s.tasks), int(s.launched),
                          int(s.peak_entries), int(s.start_epoch), int(s.done_epoch))
        if rc == E_PENDING:
            raise TreesError(rc, "tree still running")
        self._keep.pop(tree, None)
        if rc:
            raise TreesError(rc, f"tree failed: {lib().trees_last_error(self.h).decode()}")
        return int(v.value), stats

    def poll(self, tree: int):
        """results() or None while the tree is live."""
        try:
            return self.results(tree)
        except TreesError as e:
            if e.status == E_PENDING:
                return None
            raise

    def poll_finished(self, cap: int = 4096) -> list:
        """Ids of trees that have finished since the last call (trees_poll)."""
        arr = (ctypes.c_uint64 * cap)()
        n = ctypes.c_int32(0)
        self._check(lib().trees_poll(self.h, arr, cap, ctypes.byref(n)), "poll")
        return [int(arr[i]) for i in range(n.value)]

    def trace(self, tree: int) -> np.ndarray:
        out = np.zeros(256, dtype=REC_DTYPE)
        n = ctypes.c_int32(0)
        self._check(lib().trees_trace(self.h, tree, out.ctypes.data, 256, ctypes.byref(n)), "trace")
        return out[: min(n.value, 256)].copy()

    def profile_mask(self, kinds):
        """Time only the launches of the given kernel_times() kinds."""
        m = 0
        for k in kinds:
            m |= 1 << k
        self._check(lib().trees_profile_mask(self.h, m), "profile_mask")

    def kernel_times(self):
        """{kind: (ms, launches)}: HIP-event timed epoch launches; kind 0 =
        batched launches, kinds 1..5 = the plain scheduler's epochs per
        program kind, 6 and 7 = its map phase (partition pass, merge pass),
        8, 9 and 10 = its traversal (postorder, preorder), sssp and fft epochs."""
        arr = (_KTime * 11)()
        self._check(lib().trees_kernel_times(self.h, arr, 11), "kernel_times")
        return {k: (float(arr[k].ms), int(arr[k].launches)) for k in range(11)}

    def epoch_times(self) -> np.ndarray:
        """Per-epoch device-clock durations (us) of the last batched run."""
        out = (ctypes.c_double * 256)()
        n = ctypes.c_int32(0)
        self._check(lib().trees_epoch_times(self.h, out, 256, ctypes.byref(n)), "epoch_times")
        return np.array(out[: min(n.value, 256)])

    def debug_phases(self) -> np.ndarray:
        """Summed work-group time (us) per sweep phase (TREES_F_DEBUG)."""
        out = (ctypes.c_double * 8)()
        self._check(lib().trees_debug_phases(self.h, out, 8), "debug_phases")
        return np.array(out[:8])

    def abort(self):
        self._check(lib().trees_abort(self.h), "abort")

    def set_schedule(self, sched, wg: int = 0, blocks_per_cu: int = 0, graph_chunk: int = 0):
        s = SCHEDS[sched] if isinstance(sched, str) else int(sched)
        self._check(lib().trees_set_schedule(self.h, s, wg, blocks_per_cu, graph_chunk), "set_schedule")

    def wl_bfs(self, V: int, source: int, row_ptr, col_idx, depth, ws) -> WlStats:
        """Native worklist BFS (Section 6.3's comparison): depth (int32 [V],
        out) gets hop counts; ws: a device workspace of wl_workspace_bytes(V)."""
        self._torch.cuda.current_stream(self.device).synchronize()
        st = _WlStats()
        rp, ci, d, w = (_ptr_bytes(t)[0] for t in (row_ptr, col_idx, depth, ws))
        self._check(lib().trees_wl_bfs(self.h, V, source, rp, ci, d, w, _ptr_bytes(ws)[1], ctypes.byref(st)),
                    "wl_bfs")
        return WlStats(int(st.iterations), int(st.pushed), float(st.seconds))

    def wl_bfs_noalloc(self, V: int, source: int, row_ptr, col_idx, depth) -> WlStats:
        """wl_bfs with its workspace in the library's fixed device array (no
        allocation in the call; V <= 2^22)."""
        self._torch.cuda.current_stream(self.device).synchronize()
        st = _WlStats()
        rp, ci, d = (_ptr_bytes(t)[0] for t in (row_ptr, col_idx, depth))
        self._check(lib().trees_wl_bfs_noalloc(self.h, V, source, rp, ci, d, ctypes.byref(st)), "wl_bfs_noalloc")
        return WlStats(int(st.iterations), int(st.pushed), float(st.seconds))

    def wl_sssp(self, V: int, source: int, row_ptr, col_idx, weights, dist, ws) -> WlStats:
        """Native worklist SSSP: dist (int32 [V], out) gets shortest distances."""
        self._torch.cuda.current_stream(self.device).synchronize()
        st = _WlStats()
        rp, ci, wt, d, w = (_ptr_bytes(t)[0] for t in (row_ptr, col_idx, weights, dist, ws))
        self._check(lib().trees_wl_sssp(self.h, V, source, rp, ci, wt, d, w, _ptr_bytes(ws)[1],
                                        ctypes.byref(st)), "wl_sssp")
        return WlStats(int(st.iterations), int(st.pushed), float(st.seconds))

    @property
    def workload_class(self) -> str:
        """The registered program kinds as the tuned file keys them ("2+4")."""
        buf = ctypes.create_string_buffer(128)
        self._check(lib().trees_workload_class(self.h, buf, 128), "workload_class")
        return buf.value.decode()

    @property
    def free_entries(self) -> int:
        return int(lib().trees_free_entries(self.h))

    @property
    def num_trees(self) -> int:
        return int(lib().trees_num_trees(self.h))
