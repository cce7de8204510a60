"""Seeded synthetic inputs for the TREES workloads.

Shared by the CPU oracle (``oracle/``) and the GPU path.  Nothing here
computes any part of the task-parallel method: this module only draws
random numbers (SplitMix64, counter-based; see ``gen.c``) and builds the
workloads the method runs on:

* uniform uint32 sort keys;
* R-MAT graphs (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), E = 16 V directed
  arcs, vertex ids relabelled by a seeded permutation, CSR built by a stable
  counting sort, self-loops and duplicate arcs kept;
* the 4096-tree fib / N-queens batch mix and the 64-graph BFS batch;
* Poisson request traces for the serving loop.

All draws derive from one master seed, so every input is reproducible.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

MASTER_SEED = 1608005710
_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
LIB_PATH = os.path.join(_HERE, "libtrees_inputs.so")

# R-MAT cumulative quadrant thresholds a, a+b, a+b+c as 32-bit integers.
RMAT_PROBS = (0.57, 0.19, 0.19, 0.05)
RMAT_THRESHOLDS = (57 * 2**32 // 100, 76 * 2**32 // 100, 95 * 2**32 // 100)
EDGE_FACTOR = 16


def build_lib() -> str:
    """Compile gen.c into a shared library beside it (gcc, OpenMP)."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_lib()
        L = ctypes.CDLL(LIB_PATH)
        u64, i64, i32, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.tin_mix.restype = u64
        L.tin_mix.argtypes = [u64]
        L.tin_draw.restype = u64
        L.tin_draw.argtypes = [u64, u64]
        L.tin_uniform.restype = i64
        L.tin_uniform.argtypes = [u64, u64, i64, i64]
        L.tin_keys_u32.argtypes = [u64, i64, vp]
        L.tin_permutation.argtypes = [u64, i64, vp]
        L.tin_binary_tree.argtypes = [u64, i64, vp, vp]
        L.tin_rmat_edges.argtypes = [i32, i64, u64, vp, vp, vp]
        L.tin_relabel.argtypes = [i64, vp, vp]
        L.tin_csr.argtypes = [i64, i64, vp, vp, vp, vp]
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# SplitMix64 in pure Python (the same definition as gen.c; used for the
# small scalar draws and to cross-check the C library in the tests).
# ----------------------------------------------------------------------------
def mix64(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def draw(seed: int, i: int) -> int:
    return mix64((seed + (i + 1) * _GAMMA) & _M64)


def uniform(seed: int, i: int, lo: int, hi: int) -> int:
    return lo + (((draw(seed, i) >> 32) * (hi - lo + 1)) >> 32)


def unit(seed: int, i: int) -> float:
    """Uniform double in [0, 1) from the top 53 bits of one draw."""
    return (draw(seed, i) >> 11) * (1.0 / 9007199254740992.0)


def item_seed(config: int, item: int) -> int:
    """Seed of item `item` of workload `config`."""
    return mix64(MASTER_SEED ^ ((config << 32) & _M64) ^ item)


def sub_seed(seed: int, tag: int) -> int:
    return mix64(seed ^ ((tag * _GAMMA) & _M64))


def permutation(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    lib().tin_permutation(seed, n, out.ctypes.data)
    return out


# ----------------------------------------------------------------------------
# Sort keys
# ----------------------------------------------------------------------------
def arc_weights(E: int, seed: int, lo: int = 1, hi: int = 100) -> np.ndarray:
    """int32 arc weights uniform on [lo, hi]: weight i = lo + (high 32 bits
    of draw(seed, i)) * (hi - lo + 1) >> 32, the scalar `uniform` rule."""
    k = keys_u32(E, seed).astype(np.uint64)
    return (lo + ((k * np.uint64(hi - lo + 1)) >> np.uint64(32))).astype(np.int32)


def complex_signal(n: int, seed: int) -> np.ndarray:
    """n complex64 values whose real and imaginary parts are uniform on
    [-1, 1) in steps of 2^-23 (exact in fp32 and fp64): part t of value i is
    (draw(seed, 2i + t) >> 40) * 2^-23 - 1."""
    k = keys_u32(2 * n, seed) >> np.uint32(8)
    v = (k.astype(np.float64) * 2.0 ** -23 - 1.0).astype(np.float32)
    return (v[0::2] + 1j * v[1::2]).astype(np.complex64)


def sssp_graph(scale: int, seed: int, lo: int = 1, hi: int = 100) -> tuple[Graph, np.ndarray]:
    """An R-MAT graph (as for BFS) with arc weights uniform on [lo, hi]."""
    g = rmat(scale, seed)
    return g, arc_weights(g.col_idx.shape[0], sub_seed(seed, 77), lo, hi)


def binary_tree(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """(left, right) child arrays of a random binary tree of n nodes rooted
    at node 0 (-1 = no child): node v hangs below a uniform earlier node, on a
    uniform side, redrawn while that slot is taken."""
    left = np.empty(max(n, 0), dtype=np.int32)
    right = np.empty(max(n, 0), dtype=np.int32)
    if n:
        lib().tin_binary_tree(seed, n, left.ctypes.data, right.ctypes.data)
    return left, right


def postorder_tree(n: int = 1 << 22) -> tuple[np.ndarray, np.ndarray]:
    """The postorder workload: a random binary tree of n nodes."""
    return binary_tree(n, item_seed(6, 0))


def keys_u32(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    if n:
        lib().tin_keys_u32(seed, n, out.ctypes.data)
    return out


def msort_keys(n: int = 1 << 24) -> np.ndarray:
    """The merge-sort workload: n uniform uint32 keys."""
    return keys_u32(n, item_seed(2, 0))


# ----------------------------------------------------------------------------
# Graphs
# ----------------------------------------------------------------------------
@dataclass
class Graph:
    V: int
    row_ptr: np.ndarray  # int32[V+1]
    col_idx: np.ndarray  # int32[E]
    source: int

    @property
    def E(self) -> int:
        return int(self.col_idx.shape[0])


def pick_source(seed: int, row_ptr: np.ndarray) -> int:
    """First vertex with out-degree >= 1 in a seeded random probe sequence."""
    V = row_ptr.shape[0] - 1
    deg = np.diff(row_ptr)
    if not (deg > 0).any():
        return 0
    k = 0
    while True:
        v = uniform(seed, k, 0, V - 1)
        if deg[v] > 0:
            return int(v)
        k += 1


def rmat(scale: int, seed: int, edge_factor: int = EDGE_FACTOR) -> Graph:
    """Directed R-MAT graph with 2^scale vertices and edge_factor * V arcs."""
    V = 1 << scale
    E = edge_factor * V
    L = lib()
    src = np.empty(E, dtype=np.int32)
    dst = np.empty(E, dtype=np.int32)
    thr = np.array(RMAT_THRESHOLDS, dtype=np.uint32)
    L.tin_rmat_edges(scale, E, sub_seed(seed, 1), thr.ctypes.data, src.ctypes.data, dst.ctypes.data)
    perm = permutation(sub_seed(seed, 2), V)
    L.tin_relabel(E, perm.ctypes.data, src.ctypes.data)
    L.tin_relabel(E, perm.ctypes.data, dst.ctypes.data)
    row_ptr = np.empty(V + 1, dtype=np.int32)
    col_idx = np.empty(E, dtype=np.int32)
    L.tin_csr(V, E, src.ctypes.data, dst.ctypes.data, row_ptr.ctypes.data, col_idx.ctypes.data)
    del src, dst
    return Graph(V, row_ptr, col_idx, pick_source(sub_seed(seed, 3), row_ptr))


def csr_from_arcs(V: int, arcs, source: int) -> Graph:
    """Small hand-made graphs (tests): arcs is a list of (u, v)."""
    arcs = list(arcs)
    src = np.array([a for a, _ in arcs], dtype=np.int32)
    dst = np.array([b for _, b in arcs], dtype=np.int32)
    order = np.argsort(src, kind="stable")
    row_ptr = np.zeros(V + 1, dtype=np.int32)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return Graph(V, row_ptr, dst[order].astype(np.int32), int(source))


def bfs_batch_scales(ngraphs: int = 64, lo: int = 16, hi: int = 22) -> list[int]:
    """Scales of the 64-graph BFS batch (uniform in [lo, hi])."""
    return [uniform(item_seed(4, g), 0, lo, hi) for g in range(ngraphs)]


def bfs_batch_graph(g: int, scale: int) -> Graph:
    return rmat(scale, item_seed(4, g))


def sssp_batch_graph(g: int, scale: int, lo: int = 1, hi: int = 100) -> tuple[Graph, np.ndarray]:
    """Graph g of the weighted batch: the BFS batch's graph g with arc
    weights uniform on [lo, hi]."""
    G = bfs_batch_graph(g, scale)
    return G, arc_weights(G.E, item_seed(7, g), lo, hi)


# ----------------------------------------------------------------------------
# Tree batches and request traces
# ----------------------------------------------------------------------------
def batch_mix(ntrees: int = 4096, fib_range=(10, 28), nq_range=(6, 11)) -> list[tuple[str, int]]:
    """Half fib(n), half N-queens(n) trees, submitted in a seeded random order."""
    items = []
    for k in range(ntrees):
        s = item_seed(3, k)
        if k < ntrees // 2:
            items.append(("fib", uniform(s, 0, *fib_range)))
        else:
            items.append(("nqueens", uniform(s, 0, *nq_range)))
    order = permutation(item_seed(3, 1 << 31), ntrees)
    return [items[int(j)] for j in order]


@dataclass
class Request:
    rid: int
    t_arrive: float  # seconds from the start of the trace
    kind: str  # "fib" | "msort" | "bfs"
    size: int  # fib n, msort N, or R-MAT scale
    seed: int  # payload seed (msort keys, R-MAT graph)


def serving_trace(nreq: int, rate: float, trace_seed: int = 0,
                  fib_range=(12, 30), msort_log2=(10, 22), bfs_scale=(12, 20),
                  mix=(0.4, 0.4, 0.2)) -> list[Request]:
    """Poisson arrivals (exponential gaps at `rate` per second) of a 40/40/20
    fib / merge-sort / BFS mix.  Merge-sort sizes are log-uniform."""
    out = []
    t = 0.0
    base = item_seed(5, trace_seed)
    for k in range(nreq):
        s = sub_seed(base, k)
        t += -math.log(1.0 - unit(s, 0)) / rate
        u = unit(s, 1)
        if u < mix[0]:
            out.append(Request(k, t, "fib", uniform(s, 2, *fib_range), s))
        elif u < mix[0] + mix[1]:
            lo, hi = msort_log2
            n = int(math.floor(2.0 ** (lo + (hi - lo) * unit(s, 2))))
            out.append(Request(k, t, "msort", n, s))
        else:
            out.append(Request(k, t, "bfs", uniform(s, 2, *bfs_scale), s))
    return out


def request_payload(req: Request):
    """Materialise the payload of a request: keys for msort, a graph for BFS."""
    if req.kind == "msort":
        return keys_u32(req.size, sub_seed(req.seed, 7))
    if req.kind == "bfs":
        return rmat(req.size, sub_seed(req.seed, 8))
    return None
