"""Asynchronous runs (trees_run with TREES_RUN_ASYNC): trees submitted while
the persistent kernel runs -- from this thread or from others -- are adopted
at an epoch boundary and finish with exactly the result and statistics of
their oracle run alone; the kernel does not stop between submissions; an
idle run waits in empty epochs that are not counted, ends by itself after
its idle limit, and stops on abort with its trees resumable."""
import threading
import time

import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import Job, assert_matches_oracle

pytestmark = pytest.mark.gpu


def make_ctx(**kw):
    import paper_1608_00571_amd as T
    kw.setdefault("timeout_s", 20.0)
    kw.setdefault("wg", 512)
    return T.Context(256 << 20, sched="persistent", **kw)


def register(ctx):
    import paper_1608_00571_amd as T
    for k in (T.FIB_I64, T.NQUEENS, T.MSORT_U32, T.BFS_CSR, T.SSSP_CSR, T.POSTORDER):
        ctx.register(k)


def mixed_jobs(seed, n):
    """Small trees of every kind the serving mix uses, plus SSSP and postorder
    (their buffers are initialised on the device at adoption)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        k = i % 6
        if k == 0:
            jobs.append(Job("fib64", int(rng.integers(0, 24))))
        elif k == 1:
            jobs.append(Job("nqueens", int(rng.integers(4, 9))))
        elif k == 2:
            jobs.append(Job("msort", keys=inputs.keys_u32(int(rng.integers(0, 70000)), seed * 100 + i)))
        elif k == 3:
            jobs.append(Job("bfs", graph=inputs.rmat(int(rng.integers(6, 13)), seed * 100 + i)))
        elif k == 4:
            g = inputs.rmat(int(rng.integers(6, 11)), seed * 100 + i)
            jobs.append(Job("sssp", graph=g, weights=inputs.arc_weights(g.E, seed + i)))
        else:
            left, right = inputs.binary_tree(int(rng.integers(1, 3000)), seed * 100 + i)
            jobs.append(Job("postorder", bintree=(left, right, 0)))
    return jobs


def collect_all(ctx, jobs, deadline_s=60.0):
    by_id = {j.tree: j for j in jobs}
    left = set(by_id)
    t0 = time.time()
    while left:
        for t in ctx.poll_finished():
            if t in left:
                by_id[t].collect(ctx)
                left.discard(t)
        assert time.time() - t0 < deadline_s, f"{len(left)} trees still pending"
        time.sleep(0.0005)


def test_submit_while_running():
    import torch
    jobs0 = mixed_jobs(1, 12)
    late = mixed_jobs(2, 36)
    with make_ctx() as ctx:
        register(ctx)
        for j in jobs0:
            j.submit(ctx)
        rs = ctx.run(asynchronous=True)
        assert rs.sched == 2 and rs.grid > 0
        # submissions in waves while the kernel runs; each wave's buffers are
        # on the device (the binding synchronises the stream) before submit
        for w in range(6):
            wave = late[w * 6:(w + 1) * 6]
            for j in wave:
                j.submit(ctx)
            time.sleep(0.003)
        collect_all(ctx, jobs0 + late)
        fin = ctx.run()   # closes the run
    assert fin.stop_reason == 1 and fin.live == 0
    for j in jobs0 + late:
        assert_matches_oracle(j, check_trace=False)
    # trees submitted later started later: the kernel kept running across
    # the waves (global epochs kept counting in one run)
    starts = [j.stats.start_epoch for j in late]
    assert max(starts) > 0
    assert fin.global_epochs >= max(j.stats.done_epoch for j in jobs0 + late)
    assert fin.tasks == sum(j.stats.tasks for j in jobs0 + late)


def test_device_initialises_buffers_of_adopted_trees():
    """BFS depth, SSSP distance and the postorder visit counter of a tree
    adopted mid-run hold junk at submit; the kernel initialises them."""
    import torch

    import paper_1608_00571_amd as T
    g = inputs.rmat(11, 7)
    w = inputs.arc_weights(g.E, 8)
    left, right = inputs.binary_tree(4000, 9)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    wt = torch.from_numpy(w).cuda()
    depth = torch.full((g.V,), 1234, dtype=torch.int32, device="cuda")
    dist = torch.full((g.V,), -5, dtype=torch.int32, device="cuda")
    lt, rt = torch.from_numpy(left).cuda(), torch.from_numpy(right).cuda()
    log = torch.full((4001,), 77, dtype=torch.int32, device="cuda")
    with make_ctx() as ctx:
        register(ctx)
        ctx.run(asynchronous=True)
        time.sleep(0.01)   # the kernel idles in empty epochs first
        ids = [ctx.submit(ctx.register(T.BFS_CSR), [g.V, g.source], [rp, ci, depth]),
               ctx.submit(ctx.register(T.SSSP_CSR), [g.V, g.source], [rp, ci, wt, dist]),
               ctx.submit(ctx.register(T.POSTORDER), [4000, 0], [lt, rt, log])]
        stats = []
        for t in ids:
            t0 = time.time()
            while True:
                r = ctx.poll(t)
                if r is not None:
                    stats.append(r[1])
                    break
                assert time.time() - t0 < 30
                time.sleep(0.0005)
        fin = ctx.run()
    assert np.array_equal(depth.cpu().numpy(), oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source))
    assert np.array_equal(dist.cpu().numpy(), oracle.dijkstra(g.V, g.row_ptr, g.col_idx, w, g.source))
    lg = log.cpu().numpy()
    assert lg[4000] == 4000 and sorted(lg[:4000].tolist()) == list(range(4000))
    # the empty epochs spent waiting are not counted
    assert fin.global_epochs == max(s.done_epoch for s in stats) + 1


def test_submit_from_several_threads():
    jobs = mixed_jobs(3, 48)
    with make_ctx() as ctx:
        register(ctx)
        ctx.run(asynchronous=True)
        errs = []

        def worker(part):
            try:
                for j in part:
                    j.submit(ctx)
                    time.sleep(0.001)
            except Exception as e:   # surfaced below
                errs.append(e)
        ths = [threading.Thread(target=worker, args=(jobs[i::3],)) for i in range(3)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        assert not errs, errs
        collect_all(ctx, jobs)
        ctx.run()
    for j in jobs:
        assert_matches_oracle(j, check_trace=False)


def test_idle_limit_then_staged():
    """An asynchronous run with nothing to do ends by itself after timeout_s;
    a later submission is staged and runs at the next (blocking) run."""
    import paper_1608_00571_amd as T
    with make_ctx(timeout_s=1.0) as ctx:
        register(ctx)
        ctx.run(asynchronous=True)
        time.sleep(2.0)
        j = Job("fib64", 20)
        j.submit(ctx)        # the run has ended: the tree is staged
        rs = ctx.run()       # a plain blocking persistent run
        assert rs.stop_reason == 1
        j.collect(ctx)
    assert_matches_oracle(j, check_trace=False)


def test_abort_then_resume():
    import paper_1608_00571_amd as T
    jobs = [Job("fib64", 30), Job("nqueens", 10)]
    with make_ctx() as ctx:
        register(ctx)
        for j in jobs:
            j.submit(ctx)
        ctx.run(asynchronous=True)
        time.sleep(0.002)
        ctx.abort()
        fin = ctx.run()      # collects the aborted run
        assert fin.stop_reason in (1, 3)
        rs = ctx.run()       # resumes whatever was left live
        for j in jobs:
            j.collect(ctx)
    for j in jobs:
        assert_matches_oracle(j, check_trace=False)


def test_async_argument_errors():
    import paper_1608_00571_amd as T
    with T.Context(64 << 20, sched="graph") as ctx:
        ctx.register(T.FIB_I64)
        with pytest.raises(T.TreesError) as e:
            ctx.run(asynchronous=True)
        assert e.value.status == T.E_INVALID
    with make_ctx() as ctx:
        register(ctx)
        ctx.run(asynchronous=True)
        with pytest.raises(T.TreesError) as e:
            ctx.run(asynchronous=True)
        assert e.value.status == T.E_STATE
        with pytest.raises(T.TreesError) as e:
            ctx.epoch_times()
        assert e.value.status == T.E_STATE
        ctx.run()
