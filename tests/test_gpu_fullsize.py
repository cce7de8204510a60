"""GPU parity at the benchmark's full sizes, in the launch configurations
bench.py times: the default line (fib(32) with 64-bit sums and a merge sort
of 2^24 keys under the plain scheduler, 1024 lanes) and the batch of 4096
fib / N-queens trees (graph and persistent forms, 512 lanes).  Every tree's
result and statistics equal the oracle's emulation; the sort's output is the
oracle's, key for key."""
import functools

import numpy as np
import pytest

import inputs
from tests.gpu_util import Job, assert_matches_oracle, register_all

pytestmark = pytest.mark.gpu


def make_ctx(sched, arena, **kw):
    import paper_1608_00571_amd as T
    return T.Context(arena, sched=sched, timeout_s=60.0, **kw)


def test_default_line_full_size():
    """fib(32) int64 (10,573,732 tasks, 63 epochs) and msort of 2^24 keys
    (786,430 tasks, 37 epochs, merges in the map phase), run back to back
    under the plain scheduler at 1024 lanes, as in the default bench line;
    the per-epoch traces are compared too."""
    fib = Job("fib64", 32)
    srt = Job("msort", keys=inputs.keys_u32(1 << 24, inputs.item_seed(2, 0)))
    with make_ctx("plain", 4 << 30, wg=1024, trace=True) as ctx:
        register_all(ctx, [fib, srt])
        for j in (fib, srt):
            j.submit(ctx)
            ctx.run()
            j.collect(ctx, trace=True)
    assert_matches_oracle(fib)
    assert_matches_oracle(srt)


@functools.lru_cache(maxsize=None)
def expected(kind, n):
    import oracle
    r = oracle.fib(n) if kind == "fib64" else oracle.nqueens(n)
    return r.result, r.tasks, r.epochs, r.peak, r.launched


@pytest.mark.parametrize("sched", ["graph", "persistent"])
def test_tree_batch_full_size(sched):
    """The 4096 trees of the batch configuration (fib(10..28), N-queens(6..11),
    seeded order) in shared epochs: each tree's value, epochs, tasks, peak
    entries and launched lanes equal its own oracle run."""
    import paper_1608_00571_amd as T
    mix = [("fib64" if k == "fib" else "nqueens", n) for k, n in inputs.batch_mix(4096)]
    kind_of = {"fib64": T.FIB_I64, "nqueens": T.NQUEENS}
    arena = (sum(T.tv_bound(kind_of[k], [n]) + 64 for k, n in mix) + 4096) * T.BYTES_PER_ENTRY
    with make_ctx(sched, arena, wg=512, max_trees=4096) as ctx:
        progs = {k: ctx.register(v) for k, v in kind_of.items()}
        ids = [ctx.submit(progs[k], [n]) for k, n in mix]
        rs = ctx.run()
        got = [ctx.results(t) for t in ids]
    for (k, n), (value, st) in zip(mix, got):
        want = expected(k, n)
        assert (value, st.tasks, st.epochs, st.peak_entries, st.launched) == want, (k, n)
    assert rs.global_epochs == max(expected(k, n)[2] for k, n in mix)
    assert np.isfinite(rs.seconds)
