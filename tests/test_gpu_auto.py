"""The AUTO scheduler follows the tuned file: the shape a tuner recorded for
this device and the context's workload class is the one that runs (the run
statistics report it), and every tree still matches its oracle run."""
import pytest

import oracle

pytestmark = pytest.mark.gpu


def run_batch(ctx):
    import paper_1608_00571_amd as T
    pf, pq = ctx.register(T.FIB_I64), ctx.register(T.NQUEENS)
    specs = [("fib", 14), ("nqueens", 7), ("fib", 19), ("nqueens", 6), ("fib", 1)]
    ids = [ctx.submit(pf if k == "fib" else pq, [n]) for k, n in specs]
    rs = ctx.run()
    for (k, n), t in zip(specs, ids):
        v, st = ctx.results(t)
        o = oracle.fib(n) if k == "fib" else oracle.nqueens(n)
        assert (v, st.epochs, st.tasks, st.peak_entries, st.launched) == \
            (o.result, o.epochs, o.tasks, o.peak, o.launched), (k, n)
    return rs


@pytest.mark.parametrize("shape", [("graph", 512, 2, 4), ("persistent", 256, 0, 8), ("plain", 1024, 0, 8),
                                   ("persistent", 1024, 1, 8)])
def test_auto_follows_tuned_shape(tmp_path, monkeypatch, shape):
    import torch

    import paper_1608_00571_amd as T
    from paper_1608_00571_amd import autotune as A
    path = tmp_path / "tuned.txt"
    monkeypatch.setenv("TREES_TUNE_FILE", str(path))
    with T.Context(64 << 20, sched="auto", wg=256) as ctx:
        ctx.register(T.FIB_I64)
        ctx.register(T.NQUEENS)
        assert ctx.workload_class == "2+4"
        A.write_tuned(torch.cuda.get_device_name(0), ctx.workload_class, A.Shape(*shape))
        # a shape for another class must not be taken
        A.write_tuned(torch.cuda.get_device_name(0), "5", A.Shape("plain", 256, 0, 8))
        rs = run_batch(ctx)
        assert rs.sched == A.SCHED_ID[shape[0]], rs
        assert rs.wg_size == shape[1], rs
        if shape[0] != "plain" and shape[2] > 0:
            assert rs.grid <= shape[2] * torch.cuda.get_device_properties(0).multi_processor_count


def test_auto_without_a_tuned_shape_runs_graph(tmp_path, monkeypatch):
    import paper_1608_00571_amd as T
    monkeypatch.setenv("TREES_TUNE_FILE", str(tmp_path / "absent.txt"))
    with T.Context(64 << 20, sched="auto", wg=512) as ctx:
        rs = run_batch(ctx)
    assert rs.sched == T.GRAPH and rs.wg_size == 512
