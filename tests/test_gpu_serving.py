"""Serving: requests that arrive while others run are admitted into shared
epochs; every result equals the oracle's run of that request alone."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


def small_jobs(n, rate, seed):
    from paper_1608_00571_amd.serving import make_jobs
    reqs = inputs.serving_trace(n, rate, seed, fib_range=(5, 20), msort_log2=(6, 15), bfs_scale=(6, 11))
    pool = {sc: inputs.rmat(sc, 900 + sc) for sc in range(6, 12)}
    keys = {r.rid: inputs.keys_u32(r.size, inputs.sub_seed(r.seed, 7)) for r in reqs if r.kind == "msort"}
    return pool, make_jobs(reqs, pool, lambda r: keys[r.rid])


def check(jobs, pool):
    import oracle
    for j in jobs:
        if j.kind == "fib":
            r = oracle.fib(j.args[0])
            assert (j.value, j.stats.tasks, j.stats.epochs, j.stats.peak_entries, j.stats.launched) == \
                   (r.result, r.tasks, r.epochs, r.peak, r.launched)
        elif j.kind == "msort":
            out, r = oracle.msort(j.host_payload)
            assert np.array_equal(j.out, out)
            assert (j.stats.tasks, j.stats.epochs, j.stats.peak_entries) == (r.tasks, r.epochs, r.peak)
        else:
            g = pool[j.args[0].bit_length() - 1]
            d, r = oracle.bfs(g.V, g.row_ptr, g.col_idx, g.source)
            assert np.array_equal(j.out, d)
            assert (j.stats.tasks, j.stats.epochs) == (r.tasks, r.epochs)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
@pytest.mark.parametrize("realtime", [False, True])
def test_serving_results_equal_alone(sched, realtime):
    from paper_1608_00571_amd.serving import Server
    pool, jobs = small_jobs(120, 4000.0, 3)
    srv = Server(64 << 20, sched=sched, burst=3, payload_budget=1 << 30)
    try:
        res = srv.serve(jobs, realtime=realtime)
    finally:
        srv.close()
    assert len(res.jobs) == len(jobs)
    check(res.jobs, pool)
    # continuous batching: several requests were on the device together
    assert res.max_inflight > 1


def test_serving_admission_by_budget():
    """A budget that holds only a few trees at once: requests wait for
    arenas to free up, and all still complete correctly."""
    from paper_1608_00571_amd.serving import Server
    pool, jobs = small_jobs(40, 1e6, 4)
    import paper_1608_00571_amd as T
    biggest = max(T.tv_bound({"fib": T.FIB_I64, "msort": T.MSORT_U32, "bfs": T.BFS_CSR}[j.kind], j.args)
                  for j in jobs)
    srv = Server((biggest * 2 + 64) * T.BYTES_PER_ENTRY, sched="graph", burst=2, payload_budget=1 << 30)
    try:
        res = srv.serve(jobs, realtime=False)
    finally:
        srv.close()
    assert len(res.jobs) == len(jobs)
    check(res.jobs, pool)
