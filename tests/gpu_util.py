"""Helpers for the GPU parity tests: run task trees through the C ABI (via
the ctypes binding) and fetch what the oracle is compared with."""
from __future__ import annotations

import numpy as np

SCHEDS = ["plain", "graph", "persistent"]

KIND_OF = {"fib32": 1, "fib64": 2, "msort": 3, "nqueens": 4, "bfs": 5, "postorder": 6, "sssp": 7, "preorder": 8,
           "fft": 9}


def to_dev_u32(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to("cuda")


def to_dev_i32(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda")


def from_dev_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def register_all(ctx, jobs):
    """Every program must be registered before the first submit."""
    for k in sorted({j.kind for j in jobs}):
        ctx.register(KIND_OF[k])


class Job:
    """One tree: its spec, payload tensors and, after collect(), its outputs."""

    def __init__(self, kind: str, n=None, keys=None, graph=None, bintree=None, weights=None, cap=None,
                 signal=None, delta=0):
        # bintree (postorder): (left, right, root) int32 child arrays, -1 = none
        # weights (sssp): int32 arc weights in the graph's CSR order; cap: the
        # tree's task-vector entries (default 8 V)
        self.kind, self.n, self.keys, self.graph, self.bintree = kind, n, keys, graph, bintree
        self.weights, self.cap = weights, cap
        self.signal = signal   # fft: complex64 input, a power-of-two length
        self.delta = delta     # sssp: bucket width (0: the plain program)
        self.tree = None
        self.value = None
        self.stats = None
        self.trace = None
        self.out = None
        self.bufs = ()

    def submit(self, ctx):
        import torch
        import paper_1608_00571_amd as T
        prog = ctx.register(KIND_OF[self.kind])
        if self.kind in ("fib32", "fib64", "nqueens"):
            self.tree = ctx.submit(prog, [self.n])
        elif self.kind == "msort":
            k = to_dev_u32(self.keys)
            tmp = torch.empty_like(k)
            self.bufs = (k, tmp)
            self.tree = ctx.submit(prog, [self.keys.shape[0]], [k, tmp])
        elif self.kind == "bfs":
            g = self.graph
            rp, ci = to_dev_i32(g.row_ptr), to_dev_i32(g.col_idx)
            if ci.numel() == 0:
                ci = torch.zeros(1, dtype=torch.int32, device="cuda")
            d = torch.empty(g.V, dtype=torch.int32, device="cuda")
            self.bufs = (rp, ci, d)
            self.tree = ctx.submit(prog, [g.V, g.source], [rp, ci, d])
        elif self.kind == "sssp":
            g = self.graph
            rp, ci, w = to_dev_i32(g.row_ptr), to_dev_i32(g.col_idx), to_dev_i32(self.weights)
            if ci.numel() == 0:
                ci = torch.zeros(1, dtype=torch.int32, device="cuda")
                w = torch.zeros(1, dtype=torch.int32, device="cuda")
            d = torch.empty(g.V, dtype=torch.int32, device="cuda")
            self.bufs = (rp, ci, w, d)
            args = [g.V, g.source] + ([self.cap or 0, self.delta] if (self.cap or self.delta) else [])
            self.tree = ctx.submit(prog, args, [rp, ci, w, d])
        elif self.kind == "fft":
            x = np.ascontiguousarray(self.signal, dtype=np.complex64)
            xt = torch.from_numpy(x.view(np.float32).copy()).to("cuda")
            y = torch.full_like(xt, float("nan"))
            self.bufs = (xt, y)
            self.tree = ctx.submit(prog, [x.shape[0].bit_length() - 1], [xt, y])
        elif self.kind in ("postorder", "preorder"):
            left, right, root = self.bintree
            lt, rt = to_dev_i32(left), to_dev_i32(right)
            log = torch.full((left.shape[0] + 1,), -7, dtype=torch.int32, device="cuda")
            self.bufs = (lt, rt, log)
            self.tree = ctx.submit(prog, [left.shape[0], root], [lt, rt, log])
        else:
            raise ValueError(self.kind)
        return self.tree

    def collect(self, ctx, trace=False):
        if trace:
            self.trace = ctx.trace(self.tree)
        self.value, self.stats = ctx.results(self.tree)
        if self.kind == "msort":
            self.out = from_dev_u32(self.bufs[0])
        elif self.kind == "bfs":
            self.out = self.bufs[2].cpu().numpy()
        elif self.kind == "sssp":
            self.out = self.bufs[3].cpu().numpy()
        elif self.kind in ("postorder", "preorder"):
            self.out = self.bufs[2].cpu().numpy()   # visit log, then the visit count
        elif self.kind == "fft":
            self.out = self.bufs[1].cpu().numpy().view(np.complex64)
            assert np.array_equal(self.bufs[0].cpu().numpy().view(np.complex64),
                                  np.asarray(self.signal, dtype=np.complex64)), "fft: the input was modified"
        return self


def oracle_run(job: Job):
    """The oracle's emulation of the same tree: (Run, output array or None)."""
    import oracle
    if job.kind == "fib32":
        return oracle.fib(job.n, width=32, records=True), None
    if job.kind == "fib64":
        return oracle.fib(job.n, width=64, records=True), None
    if job.kind == "nqueens":
        return oracle.nqueens(job.n, records=True), None
    if job.kind == "msort":
        out, r = oracle.msort(job.keys, records=True)
        return r, out
    if job.kind == "bfs":
        g = job.graph
        d, r = oracle.bfs(g.V, g.row_ptr, g.col_idx, g.source, records=True)
        return r, d
    if job.kind == "postorder":
        left, right, root = job.bintree
        log, _, r = oracle.postorder(left, right, root, records=True)
        return r, log
    if job.kind == "fft":
        y, r = oracle.fft(np.asarray(job.signal, dtype=np.complex128), records=True)
        return r, y
    if job.kind == "preorder":
        left, right, root = job.bintree
        log, ep, r = oracle.preorder(left, right, root, records=True)
        return r, (log, ep)
    raise ValueError(job.kind)


def check_postorder_log(job: Job, want_log: np.ndarray):
    """The GPU's visit log holds each visited node once, the same nodes as the
    oracle's, and every node after its children (the order of visits within
    one epoch is not unique, so the logs are not compared entry by entry)."""
    left, right, _ = job.bintree
    n = left.shape[0]
    cnt = int(job.out[n])
    assert cnt == len(want_log), f"postorder: {cnt} visits, oracle {len(want_log)}"
    log = job.out[:cnt]
    assert np.array_equal(np.sort(log), np.sort(want_log)), "postorder: visited nodes differ"
    pos = np.full(n, -1, dtype=np.int64)
    pos[log] = np.arange(cnt)
    for child in (left, right):
        has = (pos >= 0) & (child >= 0)
        assert np.all(pos[child[has]] < pos[has]), "postorder: a node visited before its child"


def check_sssp(job: Job):
    """Distances equal Dijkstra's exactly.  The task count of the relaxation
    program depends on the order of relaxations inside an epoch, so the
    statistics are checked against what every schedule must satisfy: each
    reached vertex is visited at least once, a vertex h arcs from the source
    is first visited in epoch h, every fork goes one level deeper (epoch i
    runs at CEN i) and nothing joins."""
    import oracle
    g = job.graph
    want = oracle.dijkstra(g.V, g.row_ptr, g.col_idx, job.weights, g.source)
    bad = np.flatnonzero(job.out != want)
    assert bad.size == 0, f"sssp: {bad.size} distances differ, first at {bad[:5]}: " \
        f"got {job.out[bad[:5]]} want {want[bad[:5]]}"
    hops = oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source)
    s = job.stats
    reached = int(np.count_nonzero(want != oracle.UNREACHED))
    assert s.tasks >= reached, f"sssp: {s.tasks} visits for {reached} reached vertices"
    assert s.epochs >= int(hops.max()) + 1
    if job.delta:   # a vertex at distance d is relaxed no earlier than epoch d // delta
        assert s.epochs >= int(want[want != oracle.UNREACHED].max()) // job.delta + 1
    assert s.launched >= s.tasks
    if job.trace is not None and len(job.trace) == s.epochs and s.epochs <= 256:
        t = job.trace
        assert np.array_equal(t["cen"], np.arange(s.epochs)), "sssp: an epoch not at its depth"
        assert int(t["joins"].sum()) == 0
        assert int(t["valid"].sum()) == s.tasks
        assert int(t["forks"].sum()) == s.tasks - 1


def check_preorder_log(job: Job, want):
    """The GPU's visit log holds the oracle's visited nodes once each, in
    nondecreasing visit epoch (a node's epoch is its depth; the order within
    an epoch is not unique)."""
    want_log, want_ep = want
    n = job.bintree[0].shape[0]
    cnt = int(job.out[n])
    assert cnt == len(want_log), f"preorder: {cnt} visits, oracle {len(want_log)}"
    log = job.out[:cnt]
    assert np.array_equal(np.sort(log), np.sort(want_log)), "preorder: visited nodes differ"
    assert np.all(np.diff(want_ep[log]) >= 0), "preorder: a node visited before a shallower one"


def fft_tolerance(n: int) -> float:
    """Norm-wise relative error bound of a radix-2 FFT in fp32 against the
    exact DFT: log2(n) * eta / (1 - log2(n) * eta), eta = mu + gamma_4 (sqrt 2 + mu)
    (Higham, Accuracy and Stability of Numerical Algorithms, Thm 24.2), with
    the twiddle error mu taken as 4u and u = 2^-24; about 10 u log2 n."""
    u = 2.0 ** -24
    mu = 4 * u
    eta = mu + (4 * u / (1 - 4 * u)) * (np.sqrt(2) + mu)
    t = max(1, int(n).bit_length() - 1) * eta
    return t / (1 - t)


def check_fft(job: Job, want_y: np.ndarray):
    got = job.out.astype(np.complex128)
    assert np.all(np.isfinite(got)), "fft: outputs not written"
    err = np.linalg.norm(got - want_y) / max(np.linalg.norm(want_y), 1e-30)
    tol = fft_tolerance(want_y.shape[0])
    assert err <= tol, f"fft {want_y.shape[0]}: relative error {err:.3e} above {tol:.3e}"


def assert_matches_oracle(job: Job, check_trace=True):
    if job.kind == "sssp":
        return check_sssp(job)
    want, out = oracle_run(job)
    s = job.stats
    got = (job.value if job.kind not in ("msort", "bfs", "postorder", "preorder", "fft") else want.result,
           s.epochs, s.tasks,
           s.launched, s.peak_entries)
    exp = (want.result, want.epochs, want.tasks, want.launched, want.peak)
    assert got == exp, f"{job.kind} {job.n}: got {got} want {exp}"
    if job.kind == "postorder":
        check_postorder_log(job, out)
    elif job.kind == "preorder":
        check_preorder_log(job, out)
    elif job.kind == "fft":
        check_fft(job, out)
    elif out is not None:
        assert np.array_equal(job.out, out), f"{job.kind}: output differs"
    if check_trace and job.trace is not None and want.records is not None:
        n = min(len(job.trace), 256)
        w = want.records[:n]
        for f in ("epoch", "cen", "b", "e", "launched", "valid", "forks", "joins", "nfc"):
            assert np.array_equal(job.trace[f][:n], w[f]), f"{job.kind} {job.n}: trace field {f} differs"
