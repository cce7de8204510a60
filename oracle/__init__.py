"""TREES CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product path (the HIP
library and its Python binding) never imports it and shares no code with it;
both sides meet only in the seeded generators of ``inputs/``.

Thin ctypes wrapper over ``trees_oracle.c``:

* plain sequential evaluators (the results the method must reach):
  :func:`fib_iter`, :func:`fib_rec`, :func:`nqueens_rec`, :func:`sort_u32`,
  :func:`msort_rec`, :func:`bfs_queue`, :func:`dijkstra`, :func:`dft`;
* the epoch-semantics emulator (Task Vector Machine, Section 4.3, in the
  TREES representation of Sections 5.1.2-5.2.4): :func:`fib`,
  :func:`nqueens`, :func:`msort`, :func:`bfs`, :func:`sssp`, :func:`postorder`, :func:`preorder`,
  :func:`fft`,
  :func:`run_batch`, plus checkpoint / resume at an epoch boundary.

Every function here is pinned by ``tests/test_oracle_*.py`` against closed
forms, textbook counts, library routines, brute force on tiny inputs and the
worked example of Section 5.3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trees_oracle.c")
LIB_PATH = os.path.join(_HERE, "libtrees_oracle.so")

FIB32, FIB64, MSORT, NQUEENS, BFS, POSTORDER, SSSP, PREORDER, FFT = 1, 2, 3, 4, 5, 6, 7, 8, 9
FFT_LEAF = 64   # FFT tasks of at most this many points are leaves
UNREACHED = 2**31 - 1   # SSSP distance of a vertex the source does not reach
E_OVERFLOW, E_ENCODING = -3, -8

REC_DTYPE = np.dtype([(n, np.int32) for n in
                      ("epoch", "cen", "b", "e", "launched", "valid", "forks", "joins", "nfc")])


class _Stats(ctypes.Structure):
    _fields_ = [("result", ctypes.c_int64), ("epochs", ctypes.c_int64), ("tasks", ctypes.c_int64),
                ("launched", ctypes.c_int64), ("peak", ctypes.c_int64),
                ("tasks_by_type", ctypes.c_int64 * 2), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


def build_lib() -> str:
    """Compile the oracle with gcc (plain C, -O2)."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_lib()
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.orc_fib_iter.restype = i64
        L.orc_fib_iter.argtypes = [i32]
        L.orc_fib_rec.restype = i64
        L.orc_fib_rec.argtypes = [i32, ctypes.POINTER(i64)]
        L.orc_nqueens_rec.restype = i64
        L.orc_nqueens_rec.argtypes = [i32]
        L.orc_sort_u32.argtypes = [vp, i64]
        L.orc_msort_rec.argtypes = [vp, vp, i64]
        L.orc_bfs_queue.argtypes = [i32, vp, vp, i32, vp]
        L.orc_dijkstra.argtypes = [i32, vp, vp, vp, i32, vp]
        L.orc_dft.argtypes = [i64, vp, vp]
        L.orc_set_delta.argtypes = [vp, i32]
        L.orc_new.restype = vp
        L.orc_new.argtypes = [i32, i32, i32, vp, vp, vp, vp, i64]
        L.orc_free.argtypes = [vp]
        L.orc_keep_records.argtypes = [vp, i32]
        L.orc_step.restype = i32
        L.orc_step.argtypes = [vp]
        L.orc_run.restype = i32
        L.orc_run.argtypes = [vp, i64]
        L.orc_run_batch.restype = i64
        L.orc_run_batch.argtypes = [ctypes.POINTER(vp), i32]
        L.orc_get_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
        L.orc_num_records.restype = i64
        L.orc_num_records.argtypes = [vp]
        L.orc_get_records.argtypes = [vp, vp]
        L.orc_nfc.restype = i64
        L.orc_nfc.argtypes = [vp]
        L.orc_stack_depth.restype = i32
        L.orc_stack_depth.argtypes = [vp]
        L.orc_num_visits.restype = i64
        L.orc_num_visits.argtypes = [vp]
        L.orc_snapshot_size.restype = i64
        L.orc_snapshot_size.argtypes = [vp]
        L.orc_snapshot.restype = i64
        L.orc_snapshot.argtypes = [vp, vp]
        L.orc_restore.restype = vp
        L.orc_restore.argtypes = [vp, vp, vp, vp, vp]
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# Plain sequential evaluators
# ----------------------------------------------------------------------------
def fib_iter(n: int) -> int:
    return int(lib().orc_fib_iter(n))


def fib_rec(n: int) -> tuple[int, int]:
    """(F(n), number of calls) by naive recursion."""
    calls = ctypes.c_int64(0)
    v = lib().orc_fib_rec(n, ctypes.byref(calls))
    return int(v), int(calls.value)


def nqueens_rec(n: int) -> int:
    return int(lib().orc_nqueens_rec(n))


def sort_u32(keys: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    lib().orc_sort_u32(a.ctypes.data, a.shape[0])
    return a


def msort_rec(keys: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    t = np.empty_like(a)
    lib().orc_msort_rec(a.ctypes.data, t.ctypes.data, a.shape[0])
    return a


def dijkstra(V: int, row_ptr: np.ndarray, col_idx: np.ndarray, weights: np.ndarray, source: int) -> np.ndarray:
    """Shortest distances from `source` over non-negative int32 arc weights
    (the plain definition SSSP reaches); UNREACHED for unreachable vertices."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    w = np.ascontiguousarray(weights, dtype=np.int32)
    d = np.empty(V, dtype=np.int32)
    lib().orc_dijkstra(V, rp.ctypes.data, ci.ctypes.data, w.ctypes.data, source, d.ctypes.data)
    return d


def dft(x: np.ndarray) -> np.ndarray:
    """The DFT of x (complex, fp64) by its defining sum, O(n^2)."""
    xx = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(xx)
    lib().orc_dft(xx.shape[0], xx.ctypes.data, y.ctypes.data)
    return y


def bfs_queue(V: int, row_ptr: np.ndarray, col_idx: np.ndarray, source: int) -> np.ndarray:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    d = np.empty(V, dtype=np.int32)
    lib().orc_bfs_queue(V, rp.ctypes.data, ci.ctypes.data, source, d.ctypes.data)
    return d


# ----------------------------------------------------------------------------
# Epoch emulator
# ----------------------------------------------------------------------------
@dataclass
class Run:
    status: int
    result: int
    epochs: int
    tasks: int
    launched: int
    peak: int
    tasks_by_type: tuple
    records: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


class Emulator:
    """One task tree under the epoch semantics.  Payload arrays are kept
    alive by this object; the C side writes into them in place."""

    def __init__(self, kind: int, p0: int = 0, p1: int = 0, ptrs=(None, None, None, None),
                 cap: int = 0, records: bool = False, _handle=None):
        self._keep = [p for p in ptrs if p is not None]
        addr = [p.ctypes.data if p is not None else None for p in ptrs]
        L = lib()
        self.kind = kind
        self.h = _handle if _handle is not None else L.orc_new(kind, p0, p1, *addr, cap)
        if records:
            L.orc_keep_records(self.h, 1)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_free(h)
            self.h = None

    def step(self) -> int:
        return int(lib().orc_step(self.h))

    def run(self, max_epochs: int = -1) -> int:
        return int(lib().orc_run(self.h, max_epochs))

    @property
    def nfc(self) -> int:
        return int(lib().orc_nfc(self.h))

    @property
    def stack_depth(self) -> int:
        return int(lib().orc_stack_depth(self.h))

    def stats(self) -> Run:
        s = _Stats()
        L = lib()
        L.orc_get_stats(self.h, ctypes.byref(s))
        n = int(L.orc_num_records(self.h))
        recs = None
        if n:
            recs = np.empty(n, dtype=REC_DTYPE)
            L.orc_get_records(self.h, recs.ctypes.data)
        return Run(int(s.status), int(s.result), int(s.epochs), int(s.tasks), int(s.launched),
                   int(s.peak), tuple(int(x) for x in s.tasks_by_type), recs,
                   {"nvisit": int(L.orc_num_visits(self.h))})

    def snapshot(self) -> bytes:
        L = lib()
        buf = ctypes.create_string_buffer(int(L.orc_snapshot_size(self.h)))
        n = L.orc_snapshot(self.h, buf)
        return buf.raw[:n]

    @classmethod
    def restore(cls, kind: int, snap: bytes, ptrs=(None, None, None, None), records=False):
        buf = ctypes.create_string_buffer(snap, len(snap))
        addr = [p.ctypes.data if p is not None else None for p in ptrs]
        h = lib().orc_restore(buf, *addr)
        return cls(kind, ptrs=ptrs, records=records, _handle=h)


def fib(n: int, width: int = 64, records: bool = False, cap: int = 0) -> Run:
    em = Emulator(FIB64 if width == 64 else FIB32, n, cap=cap, records=records)
    em.run()
    return em.stats()


def nqueens(n: int, records: bool = False, cap: int = 0) -> Run:
    em = Emulator(NQUEENS, n, cap=cap, records=records)
    em.run()
    return em.stats()


def msort(keys: np.ndarray, records: bool = False, cap: int = 0) -> tuple[np.ndarray, Run]:
    a = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    t = np.zeros_like(a)
    em = Emulator(MSORT, a.shape[0], ptrs=(a, t, None, None), cap=cap, records=records)
    em.run()
    return a, em.stats()


def bfs(V: int, row_ptr: np.ndarray, col_idx: np.ndarray, source: int, records: bool = False,
        cap: int = 0) -> tuple[np.ndarray, Run]:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    d = np.empty(V, dtype=np.int32)
    em = Emulator(BFS, V, source, ptrs=(rp, ci, d, None), cap=cap, records=records)
    em.run()
    return d, em.stats()


def sssp(V: int, row_ptr: np.ndarray, col_idx: np.ndarray, weights: np.ndarray, source: int,
         records: bool = False, cap: int = 0, delta: int = 0) -> tuple[np.ndarray, Run]:
    """The relaxation program in the epoch emulator: distances (UNREACHED
    for unreachable vertices) and the statistics of this one schedule (task
    counts depend on the order of relaxations inside an epoch).  delta > 0:
    a visit whose distance is at least (CEN + 1) * delta waits an epoch."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    w = np.ascontiguousarray(weights, dtype=np.int32)
    d = np.empty(V, dtype=np.int32)
    em = Emulator(SSSP, V, source, ptrs=(rp, ci, w, d), cap=cap, records=records)
    if delta:
        lib().orc_set_delta(em.h, delta)
    em.run()
    return d, em.stats()


def postorder(left, right, root: int, records: bool = True) -> tuple[np.ndarray, np.ndarray, Run]:
    """Figure 2's postorder traversal; returns (visit order, epoch of each
    node's visit, run statistics)."""
    L_ = np.ascontiguousarray(left, dtype=np.int32)
    R_ = np.ascontiguousarray(right, dtype=np.int32)
    n = L_.shape[0]
    log = np.full(max(n, 1), -1, dtype=np.int32)
    ep = np.full(max(n, 1), -1, dtype=np.int32)
    em = Emulator(POSTORDER, root, ptrs=(L_, R_, log, ep), records=records)
    em.run()
    st = em.stats()
    return log[: st.extra["nvisit"]], ep[:n], st


def preorder(left, right, root: int, records: bool = True) -> tuple[np.ndarray, np.ndarray, Run]:
    """Figure 2's preorder traversal; returns (visit order, epoch of each
    node's visit, run statistics)."""
    L_ = np.ascontiguousarray(left, dtype=np.int32)
    R_ = np.ascontiguousarray(right, dtype=np.int32)
    n = L_.shape[0]
    log = np.full(max(n, 1), -1, dtype=np.int32)
    ep = np.full(max(n, 1), -1, dtype=np.int32)
    em = Emulator(PREORDER, root, ptrs=(L_, R_, log, ep), records=records)
    em.run()
    st = em.stats()
    return log[: st.extra["nvisit"]], ep[:n], st


def fft(x: np.ndarray, records: bool = False) -> tuple[np.ndarray, Run]:
    """The FFT program (radix-2 decimation in time, leaves of FFT_LEAF points
    by the defining sum) in the epoch emulator, fp64; len(x) a power of two."""
    xx = np.ascontiguousarray(x, dtype=np.complex128)
    n = xx.shape[0]
    m = n.bit_length() - 1
    assert n >= 1 and n == 1 << m, "fft: the length must be a power of two"
    y = np.zeros_like(xx)
    em = Emulator(FFT, m, ptrs=(xx, y, None, None), records=records)
    em.run()
    return y, em.stats()


def run_batch(emulators: list[Emulator]) -> int:
    """Run trees together in shared global epochs; returns the global epoch count."""
    arr = (ctypes.c_void_p * len(emulators))(*[e.h for e in emulators])
    return int(lib().orc_run_batch(arr, len(emulators)))
