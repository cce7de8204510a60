"""Continuous-batching serving loop over one TREES context.

Requests (fib, merge sort, BFS task programs) arrive over time.  The loop
admits each one as soon as its task-vector arena and working buffers fit in
the budget -- FIFO, with a bounded skip-ahead past requests that do not fit
yet -- and collects finished ones as soon as the device reports them.

Two modes:
  * "async" (default): one asynchronous persistent run (trees_run with
    TREES_RUN_ASYNC).  A request is submitted the moment it arrives and
    fits; the running kernel adopts it at the next epoch boundary, so its
    work shares epochs with the requests already on the device.  Finished
    trees come back through the completion ring (trees_poll) while the
    kernel keeps running.
  * "bursts": the host runs the device in bursts of `burst` shared epochs
    (blocking trees_run calls), admitting and collecting between bursts.
    Kept as the comparison point: a request that arrives during a burst
    waits for its end.

Latency is measured from a request's arrival to the moment the loop sees it
finished.  Payloads (merge-sort keys, each BFS request's own graph) are on
the device before serving starts -- a request names device-resident data --
and each request owns its output buffers.  Every step of the epoch path runs
in libtrees; this module only decides what to submit and when.
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
    host_payload: object = None      # msort: uint32 keys (numpy); bfs: the Graph
    tree: int | None = None
    dev: tuple = ()                  # device buffers handed to trees_submit
    t_admit: float = 0.0
    t_done: float = 0.0
    value: int = 0
    stats: object = None
    out_dev: object = None           # msort: sorted keys; bfs: depths (device tensors)
    bytes_payload: int = 0           # device bytes the request holds while admitted

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
    """Serves jobs through one context (see the module docstring for the
    two modes)."""

    def __init__(self, arena_bytes: int, *, mode: str = "async", sched: str = "persistent", burst: int = 8,
                 skip_ahead: int = 8, payload_budget: int = 16 << 30, wg: int = 1024, max_trees: int = 4096,
                 timeout_s: float = 60.0):
        import torch
        if mode not in ("async", "bursts"):
            raise ValueError(mode)
        self.torch = torch
        self.mode = mode
        self.ctx = Context(arena_bytes, sched="persistent" if mode == "async" else sched, wg=wg,
                           graph_chunk=burst, max_trees=max_trees, timeout_s=timeout_s)
        self.progs = {k: self.ctx.register(v) for k, v in KIND.items()}
        self.burst = burst
        self.skip_ahead = skip_ahead
        self.payload_budget = payload_budget
        self.payload_used = 0

    def close(self):
        self.ctx.close()

    # -- admission ------------------------------------------------------------
    def _try_admit(self, j: Job, now: float) -> bool:
        if self.payload_used + j.bytes_payload > self.payload_budget:
            return False
        t = self.ctx.try_submit(self.progs[j.kind], j.args, j.dev, ready=True)
        if t is None:
            return False
        j.tree = t
        j.t_admit = now
        self.payload_used += j.bytes_payload
        return True

    def _finish(self, j: Job, r, now: float):
        j.value, j.stats = r
        j.t_done = now
        if j.kind == "msort":
            j.out_dev = j.dev[0]
        elif j.kind == "bfs":
            j.out_dev = j.dev[2]
        self.payload_used -= j.bytes_payload

    def _admit_pending(self, pending, inflight, now):
        """FIFO admission with bounded skip-ahead past jobs that do not fit."""
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
            pending[:] = [j for j in pending if id(j) not in ids]
        elif pending and not inflight:
            raise TreesError(-2, f"request {pending[0].rid} does not fit in an empty context")
        return len(admitted)

    # -- the loop ----------------------------------------------------------------
    def serve(self, jobs: list[Job], realtime: bool = True) -> ServeResult:
        """Serve `jobs` (sorted by arrival).  realtime=False admits every job
        at time 0 (a closed batch: the saturation throughput)."""
        self.torch.cuda.synchronize()   # the payloads are on the device
        if self.mode == "async":
            return self._serve_async(jobs, realtime)
        return self._serve_bursts(jobs, realtime)

    def _serve_async(self, jobs, realtime):
        waiting = collections.deque(jobs)
        pending: list[Job] = []
        inflight: dict[int, Job] = {}
        done = []
        max_inflight = 0
        self.ctx.run(asynchronous=True)
        t0 = time.perf_counter()
        try:
            while waiting or pending or inflight:
                now = time.perf_counter() - t0
                while waiting and (not realtime or waiting[0].t_arrive <= now):
                    pending.append(waiting.popleft())
                busy = 0
                if pending:
                    busy += self._admit_pending(pending, inflight, now)
                max_inflight = max(max_inflight, len(inflight))
                if inflight:
                    fin = self.ctx.poll_finished()
                    if fin:
                        now = time.perf_counter() - t0
                        for t in fin:
                            j = inflight.pop(t, None)
                            if j is not None:
                                self._finish(j, self.ctx.results(t), now)
                                done.append(j)
                        busy += len(fin)
                if not busy:
                    if waiting and not inflight and not pending and realtime:
                        gap = waiting[0].t_arrive - (time.perf_counter() - t0)
                        if gap > 0:
                            time.sleep(min(gap, 5e-4))
                    else:
                        time.sleep(2e-5)
        finally:
            rs = self.ctx.run()   # closes the asynchronous run
        total = time.perf_counter() - t0
        lat = np.array([j.t_done - (0.0 if not realtime else j.t_arrive) for j in done])
        return ServeResult(done, total, 1, max_inflight, int(rs.global_epochs), lat)

    def _serve_bursts(self, jobs, realtime):
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
            if pending:
                self._admit_pending(pending, inflight, now)
            if inflight:
                max_inflight = max(max_inflight, len(inflight))
                rs = self.ctx.run(self.burst)
                bursts += 1
                epochs += rs.global_epochs
                now = time.perf_counter() - t0
                for t in self.ctx.poll_finished():
                    j = inflight.pop(t, None)
                    if j is not None:
                        self._finish(j, self.ctx.results(t), now)
                        done.append(j)
            elif waiting and realtime:
                gap = waiting[0].t_arrive - (time.perf_counter() - t0)
                if gap > 0:
                    time.sleep(min(gap, 0.001))
        total = time.perf_counter() - t0
        lat = np.array([j.t_done - (0.0 if not realtime else j.t_arrive) for j in done])
        return ServeResult(done, total, bursts, max_inflight, epochs, lat)


def make_jobs(requests, payload_for) -> list[Job]:
    """Turn request descriptions into jobs with their payloads on the device.
    payload_for(req) returns the request's host payload: uint32 keys for
    msort, its own Graph for BFS (None for fib).  A request's admission bytes
    are the device buffers it holds: keys + merge buffer, or graph + depths."""
    import torch
    jobs = []
    for r in requests:
        if r.kind == "fib":
            jobs.append(Job(r.rid, r.t_arrive, "fib", [r.size]))
            continue
        p = payload_for(r)
        if r.kind == "msort":
            k = torch.from_numpy(np.ascontiguousarray(p).view(np.int32)).to("cuda")
            jobs.append(Job(r.rid, r.t_arrive, "msort", [r.size], p, dev=(k, torch.empty_like(k)),
                            bytes_payload=8 * r.size))
        else:
            rp = torch.from_numpy(p.row_ptr).to("cuda")
            ci = torch.from_numpy(p.col_idx).to("cuda")
            if ci.numel() == 0:
                ci = torch.zeros(1, dtype=torch.int32, device="cuda")
            d = torch.empty(p.V, dtype=torch.int32, device="cuda")
            jobs.append(Job(r.rid, r.t_arrive, "bfs", [p.V, p.source], p, dev=(rp, ci, d),
                            bytes_payload=4 * (p.V + 1) + 4 * p.E + 4 * p.V))
    return jobs
