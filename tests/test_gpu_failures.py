"""Failure handling and resumption through the C ABI: an epoch budget pauses
every tree at an epoch boundary and a later run (under any scheduler)
finishes it with the oracle's result and statistics; an abort from another
thread stops a run the same way; a budget that is full refuses admission
until a tree is collected; bad arguments and late registration are refused."""
import threading

import numpy as np
import pytest

import oracle
from tests.gpu_util import Job, assert_matches_oracle, register_all

pytestmark = pytest.mark.gpu


def ctx(sched, arena=64 << 20, **kw):
    import paper_1608_00571_amd as T
    return T.Context(arena, sched=sched, timeout_s=20.0, **kw)


@pytest.mark.parametrize("first,second", [("persistent", "graph"), ("graph", "plain"),
                                          ("plain", "persistent")])
def test_epoch_budget_pauses_and_resumes(first, second):
    import paper_1608_00571_amd as T
    jobs = [Job("fib64", 18), Job("nqueens", 7), Job("fib64", 3)]
    with ctx(first, trace=True) as c:
        register_all(c, jobs)
        for j in jobs:
            j.submit(c)
        rs = c.run(max_epochs=5)
        assert rs.stop_reason == 2 and rs.live >= 1
        with pytest.raises(T.TreesError) as e:
            c.results(jobs[0].tree)
        assert e.value.status == T.E_PENDING
        c.set_schedule(second)
        c.run()
        for j in jobs:
            j.collect(c, trace=True)
    for j in jobs:
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
def test_abort_from_another_thread_then_resume(sched):
    """The abort lands at an epoch boundary (or after the run ended, if the
    run was faster than the other thread): either way every tree finishes
    correctly after a further run."""
    import time
    jobs = [Job("fib64", 32) for _ in range(8)]
    with ctx(sched, arena=2 << 30) as c:
        register_all(c, jobs)
        for j in jobs:
            j.submit(c)
        out = {}

        def runner():
            out["rs"] = c.run()

        t = threading.Thread(target=runner)
        t.start()
        time.sleep(0.002)
        c.abort()
        t.join(60)
        assert not t.is_alive()
        rs = out["rs"]
        assert rs.stop_reason in (1, 3)
        if rs.stop_reason == 3:
            assert rs.live >= 1
            c.run()
        for j in jobs:
            j.collect(c, trace=False)
    for j in jobs:
        assert_matches_oracle(j, check_trace=False)


def test_admission_refused_until_collected():
    import paper_1608_00571_amd as T
    need = T.tv_bound(T.FIB_I64, [20])
    per = ((need + 63) // 64) * 64
    with ctx("persistent", arena=(per * 2 + 10) * T.BYTES_PER_ENTRY) as c:
        p = c.register(T.FIB_I64)
        a = c.submit(p, [20])
        b = c.submit(p, [20])
        assert c.try_submit(p, [20]) is None          # the budget holds two arenas
        c.run()
        assert c.results(a)[0] == oracle.fib(20).result
        d = c.submit(p, [20])                          # a's arena came back
        c.run()
        assert c.results(b)[0] == oracle.fib(20).result
        assert c.results(d)[0] == oracle.fib(20).result
        assert c.num_trees == 0


def test_bad_arguments_and_late_registration():
    import paper_1608_00571_amd as T
    with ctx("plain") as c:
        pq = c.register(T.NQUEENS)
        for bad in ([0], [15], []):
            with pytest.raises(T.TreesError) as e:
                c.submit(pq, bad)
            assert e.value.status == T.E_INVALID
        pf = c.register(T.FIB_I64)
        t = c.submit(pf, [10])
        with pytest.raises(T.TreesError) as e:
            c.register(T.MSORT_U32)                     # the type ids are frozen at the first submit
        assert e.value.status == T.E_STATE
        c.run()
        assert c.results(t)[0] == 55
        with pytest.raises(T.TreesError):
            c.results(t)                                # released: the id is stale


def test_overlapping_buffers_refused():
    """Output buffers that overlap a tree's inputs (or msort's keys and tmp)
    are refused at submit with INVALID; nothing is admitted."""
    import torch

    import paper_1608_00571_amd as T
    with ctx("plain") as c:
        pm, pb = c.register(T.MSORT_U32), c.register(T.BFS_CSR)
        keys = torch.zeros(4096, dtype=torch.int32, device="cuda")
        rp = torch.zeros(101, dtype=torch.int32, device="cuda")
        ci = torch.zeros(16, dtype=torch.int32, device="cuda")
        for prog, args, bufs in [(pm, [2048], [keys[:2048], keys[1024:3072]]),
                                 (pb, [100, 0], [rp, ci, rp[:100]]),
                                 (pb, [10, 0], [rp, ci, ci[:10]])]:
            with pytest.raises(T.TreesError) as e:
                c.submit(prog, args, bufs)
            assert e.value.status == T.E_INVALID
        assert c.num_trees == 0
        t = c.submit(pm, [2048], [keys[:2048], keys[2048:]])   # adjacent, not overlapping: admitted
        c.run()
        c.results(t)


@pytest.mark.parametrize("kind", ["postorder", "preorder"])
def test_traversal_log_cleared_after_pending_fill(kind):
    """A traversal's visit counter (log[n]) is cleared inside trees_run, after
    the caller's own pending work on the log: a fill of the log that is still
    queued on the caller's stream at submit (behind a device-side sleep)
    lands before the clear, so the tree still logs every node once.  A
    submit refused for lack of budget leaves the log untouched."""
    import torch

    import inputs
    import paper_1608_00571_amd as T
    left, right = inputs.binary_tree(5000, 11)
    n = left.shape[0]
    lt = torch.from_numpy(left).cuda()
    rt = torch.from_numpy(right).cuda()
    with ctx("graph", arena=(2 * n + 1 + 64) * T.BYTES_PER_ENTRY) as c:
        p = c.register(T.POSTORDER if kind == "postorder" else T.PREORDER)
        log = torch.empty(n + 1, dtype=torch.int32, device="cuda")
        torch.cuda._sleep(20_000_000)   # keeps the fill below queued past the submit
        log.fill_(-7)
        t = c.submit(p, [n, 0], [lt, rt, log])
        # a second tree does not fit: refused, and its log keeps its contents
        log2 = torch.full((n + 1,), 5, dtype=torch.int32, device="cuda")
        assert c.try_submit(p, [n, 0], [lt, rt, log2]) is None
        c.run()
        c.results(t)
        torch.cuda.synchronize()
        out = log.cpu().numpy()
        assert int(out[n]) == n
        assert sorted(out[:n].tolist()) == list(range(n))
        assert np.all(log2.cpu().numpy() == 5)


def test_library_loaded_before_torch_uses_the_gpu():
    """The library loaded before torch has touched the GPU (a host-only call
    first), then torch allocates, then a context runs a tree: the binding
    loads torch's runtime ahead of the library, so this order works too.
    Run in a fresh process, where nothing has loaded either yet."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1608_00571_amd as T\n"
        "need = T.tv_bound(T.FIB_I64, [15])\n"
        "import torch\n"
        "x = torch.zeros(16, device='cuda')\n"
        "with T.Context((need + 4096) * T.BYTES_PER_ENTRY, sched='graph', timeout_s=20.0) as c:\n"
        "    p = c.register(T.FIB_I64)\n"
        "    t = c.submit(p, [15])\n"
        "    c.run()\n"
        "    v, st = c.results(t)\n"
        "assert v == 610, v\n"
        "print('ok', v)\n" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "ok 610" in r.stdout
