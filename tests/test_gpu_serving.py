"""Serving: requests that arrive while others run are admitted into shared
epochs; every result and tree statistic equals the oracle's run of that
request alone.  The asynchronous mode submits into a running persistent
kernel; the burst mode runs the device in bursts of shared epochs."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


def make(n, rate, seed, **sizes):
    from paper_1608_00571_amd.serving import make_jobs
    reqs = inputs.serving_trace(n, rate, seed, **sizes)
    return make_jobs(reqs, inputs.request_payload)


def small_jobs(n, rate, seed):
    return make(n, rate, seed, fib_range=(5, 20), msort_log2=(6, 15), bfs_scale=(6, 11))


def check(jobs):
    """Each served request against the oracle's run of it alone: fib value,
    tasks, epochs, peak and lanes; msort output, tasks, epochs and peak;
    BFS depths (the request's own graph), tasks and epochs."""
    import oracle
    for j in jobs:
        s = j.stats
        if j.kind == "fib":
            r = oracle.fib(j.args[0])
            assert (j.value, s.tasks, s.epochs, s.peak_entries, s.launched) == \
                   (r.result, r.tasks, r.epochs, r.peak, r.launched), f"fib request {j.rid}"
        elif j.kind == "msort":
            out, r = oracle.msort(j.host_payload)
            assert np.array_equal(j.out, out), f"msort request {j.rid}"
            assert (s.tasks, s.epochs, s.peak_entries) == (r.tasks, r.epochs, r.peak), f"msort request {j.rid}"
        else:
            g = j.host_payload
            d, r = oracle.bfs(g.V, g.row_ptr, g.col_idx, g.source)
            assert np.array_equal(j.out, d), f"bfs request {j.rid}"
            assert (s.tasks, s.epochs) == (r.tasks, r.epochs), f"bfs request {j.rid}"


@pytest.mark.parametrize("mode", ["async", "bursts"])
@pytest.mark.parametrize("realtime", [False, True])
def test_serving_results_equal_alone(mode, realtime):
    from paper_1608_00571_amd.serving import Server
    jobs = small_jobs(120, 4000.0, 3)
    srv = Server(64 << 20, mode=mode, sched="graph", burst=3, payload_budget=1 << 30, timeout_s=20.0)
    try:
        res = srv.serve(jobs, realtime=realtime)
    finally:
        srv.close()
    assert len(res.jobs) == len(jobs)
    check(res.jobs)
    # continuous batching: several requests were on the device together
    assert res.max_inflight > 1


@pytest.mark.parametrize("mode", ["async", "bursts"])
def test_serving_admission_by_budget(mode):
    """A budget that holds only a few trees at once: requests wait for
    arenas to free up, and all still complete correctly."""
    from paper_1608_00571_amd.serving import Server
    import paper_1608_00571_amd as T
    jobs = small_jobs(40, 1e6, 4)
    biggest = max(T.tv_bound({"fib": T.FIB_I64, "msort": T.MSORT_U32, "bfs": T.BFS_CSR}[j.kind], j.args)
                  for j in jobs)
    srv = Server((biggest * 2 + 64) * T.BYTES_PER_ENTRY, mode=mode, sched="graph", burst=2,
                 payload_budget=1 << 30, timeout_s=20.0)
    try:
        res = srv.serve(jobs, realtime=False)
    finally:
        srv.close()
    assert len(res.jobs) == len(jobs)
    check(res.jobs)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("realtime", [False, True])
def test_serving_stated_sizes(realtime):
    """The serving configuration at its stated sizes: 120 requests drawn
    40/40/20 from fib(12..30), msort of 2^10..2^22 keys (log-uniform) and
    R-MAT BFS of scale 12..20, each BFS request on its own seeded graph;
    admission within a 64 GiB budget (32 GiB of task-vector arena, 32 GiB
    of request buffers); the asynchronous persistent form at the work-group
    size the bench serves with.  Every request against its oracle run."""
    import torch
    from paper_1608_00571_amd.serving import Server
    jobs = make(120, 3000.0, 11)
    kinds = {j.kind for j in jobs}
    assert kinds == {"fib", "msort", "bfs"}
    assert max(j.args[0] for j in jobs if j.kind == "fib") >= 25
    srv = Server(32 << 30, mode="async", payload_budget=32 << 30, wg=1024, timeout_s=30.0)
    try:
        res = srv.serve(jobs, realtime=realtime)
    finally:
        srv.close()
    assert len(res.jobs) == len(jobs)
    check(res.jobs)
    assert res.max_inflight > 1
    del jobs, res
    torch.cuda.empty_cache()
