"""Continuous-batching serving loop over one TREES context.

Requests (fib, merge sort, BFS task programs) arrive over time.  The loop
admits each one as soon as its task-vector arena fits in the context's
budget -- FIFO, with a bounded skip-ahead past requests that do not fit yet
-- and runs the device in short bursts of shared epochs.  Requests admitted
while others are on the device join the next global epoch, so their work
overlaps; finished trees are collected after every burst and their arenas
return to the budget.  Latency is measured from a request's arrival to the
burst after which its result was collected.

Payloads: a merge-sort request brings its keys in pinned host memory
(uploaded asynchronously at admission); BFS requests query graphs of a
device-resident pool (uploaded once per graph, shared by every request on
that graph); a request's output stays on the device until it is read.

Every step of the epoch path runs in libtrees; this module only decides
what to submit and when.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import BFS_CSR, FIB_I64, MSORT_U32, Context, TreesError

KIND = {"fib": FIB_I64, "msort": MSORT_U32, "bfs": BFS_CSR}


@dataclass
class Job:
    """One request as the serving loop sees it."""
    rid: int
    t_arrive: float
    kind: str
    args: list
    host_payload: object = None      # msort: uint32 keys (numpy); bfs: (row_ptr, col_idx)
    graph_key: object = None         # bfs: the pool graph the request queries
    tree: int | None = None
    dev: tuple = ()
    t_admit: float = 0.0
    t_done: float = 0.0
    value: int = 0
    stats: object = None
    out_dev: object = None           # msort: sorted keys; bfs: depths (device tensors)
    bytes_payload: int = 0
    pinned: object = None            # msort: the keys in pinned host memory

    @property
    def out(self) -> np.ndarray | None:
        """The request's output on the host (copied on first use)."""
        if self.out_dev is None:
            return None
        a = self.out_dev.cpu().numpy()
        return a.view(np.uint32) if self.kind == "msort" else a


@dataclass
class ServeResult:
    jobs: list
    seconds: float
    bursts: int
    max_inflight: int
    epochs: int
    latencies: np.ndarray = field(default_factory=lambda: np.zeros(0))

    def pct(self, q: float) -> float:
        return float(np.percentile(self.latencies, q)) if len(self.latencies) else 0.0


class Server:
    """Serves jobs through one context.  `burst` epochs run per device call."""

    def __init__(self, arena_bytes: int, *, sched: str = "graph", burst: int = 8, skip_ahead: int = 8,
                 payload_budget: int = 16 << 30, wg: int = 512, max_trees: int = 4096):
        import torch
        self.torch = torch
        self.ctx = Context(arena_bytes, sched=sched, wg=wg, graph_chunk=burst, max_trees=max_trees)
        self.progs = {k: self.ctx.register(v) for k, v in KIND.items()}
        self.burst = burst
        self.skip_ahead = skip_ahead
        self.payload_budget = payload_budget
        self.payload_used = 0
        self.graphs = {}   # graph_key -> (row_ptr, col_idx) on the device

    def close(self):
        self.ctx.close()

    # -- admission ------------------------------------------------------------
    def _graph(self, j: Job):
        key = j.graph_key if j.graph_key is not None else ("job", j.rid)
        g = self.graphs.get(key)
        if g is None:
            rp, ci = j.host_payload
            g = (self.torch.from_numpy(rp).to("cuda"), self.torch.from_numpy(ci).to("cuda"))
            if j.graph_key is not None:
                self.graphs[key] = g
        return g

    def _upload(self, j: Job):
        torch = self.torch
        if j.kind == "msort":
            src = j.pinned if j.pinned is not None else torch.from_numpy(j.host_payload.view(np.int32))
            k = src.to("cuda", non_blocking=True)
            j.dev = (k, torch.empty_like(k))
        elif j.kind == "bfs":
            rp, ci = self._graph(j)
            j.dev = (rp, ci, torch.empty(rp.shape[0] - 1, dtype=torch.int32, device="cuda"))

    def _try_admit(self, j: Job, now: float) -> bool:
        if self.payload_used + j.bytes_payload > self.payload_budget:
            return False
        if j.kind != "fib" and not j.dev:
            self._upload(j)
        t = self.ctx.try_submit(self.progs[j.kind], j.args, j.dev)
        if t is None:
            return False
        j.tree = t
        j.t_admit = now
        self.payload_used += j.bytes_payload
        return True

    def _collect(self, j: Job, now: float) -> bool:
        r = self.ctx.poll(j.tree)
        if r is None:
            return False
        j.value, j.stats = r
        j.t_done = now
        if j.kind == "msort":
            j.out_dev = j.dev[0]
        elif j.kind == "bfs":
            j.out_dev = j.dev[2]
        j.dev = ()
        self.payload_used -= j.bytes_payload
        return True

    # -- the loop ----------------------------------------------------------------
    def serve(self, jobs: list[Job], realtime: bool = True) -> ServeResult:
        """Serve `jobs` (sorted by arrival).  realtime=False admits every job
        at time 0 (a closed batch: the saturation throughput)."""
        torch = self.torch
        waiting = collections.deque(jobs)
        pending: list[Job] = []
        inflight: dict[int, Job] = {}
        done = []
        bursts = epochs = max_inflight = 0
        t0 = time.perf_counter()
        while waiting or pending or inflight:
            now = time.perf_counter() - t0
            while waiting and (not realtime or waiting[0].t_arrive <= now):
                pending.append(waiting.popleft())
            # FIFO admission with bounded skip-ahead past jobs that do not fit
            admitted, skipped = [], 0
            for j in pending:
                if skipped > self.skip_ahead:
                    break
                if self._try_admit(j, now):
                    admitted.append(j)
                    inflight[j.tree] = j
                else:
                    skipped += 1
            if admitted:
                ids = {id(j) for j in admitted}
                pending = [j for j in pending if id(j) not in ids]
            elif pending and not inflight:
                raise TreesError(-2, f"request {pending[0].rid} does not fit in an empty context")
            if inflight:
                max_inflight = max(max_inflight, len(inflight))
                torch.cuda.current_stream().synchronize()   # payload copies before the device reads them
                rs = self.ctx.run(self.burst)
                bursts += 1
                epochs += rs.global_epochs
                now = time.perf_counter() - t0
                for t in [t for t, j in inflight.items() if self._collect(j, now)]:
                    done.append(inflight.pop(t))
            elif waiting and realtime:
                gap = waiting[0].t_arrive - (time.perf_counter() - t0)
                if gap > 0:
                    time.sleep(min(gap, 0.001))
        total = time.perf_counter() - t0
        lat = np.array([j.t_done - (0.0 if not realtime else j.t_arrive) for j in done])
        return ServeResult(done, total, bursts, max_inflight, epochs, lat)


def make_jobs(requests, graph_pool: dict, keys_for, pin: bool = True) -> list[Job]:
    """Turn request descriptions into jobs.  graph_pool maps an R-MAT scale
    to a host graph (requests on one scale query the same pool graph);
    keys_for(req) returns the request's uint32 keys, which arrive in pinned
    host memory when `pin`."""
    import torch
    jobs = []
    for r in requests:
        if r.kind == "fib":
            jobs.append(Job(r.rid, r.t_arrive, "fib", [r.size]))
        elif r.kind == "msort":
            keys = keys_for(r)
            pinned = torch.from_numpy(keys.view(np.int32)).pin_memory() if pin else None
            jobs.append(Job(r.rid, r.t_arrive, "msort", [r.size], keys, bytes_payload=8 * r.size,
                            pinned=pinned))
        else:
            g = graph_pool[r.size]
            # the graph is pool-resident; a request holds its depth array
            jobs.append(Job(r.rid, r.t_arrive, "bfs", [g.V, g.source], (g.row_ptr, g.col_idx),
                            graph_key=("rmat", r.size), bytes_payload=4 * g.V))
    return jobs
