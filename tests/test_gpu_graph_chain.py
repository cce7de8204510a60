"""Captured chains (the graph form): a chain holds graph_chunk epochs, each
with its map launches, and ends with a node that publishes the header to
host-mapped memory for the host to poll.  Runs of one context under chains of
1 to 8 epochs (the runs end at different positions inside their last chain),
re-captured between runs when the work-group size or the chain length
changes; every result, tree statistic and trace against the oracle's run of
the tree alone."""
import pytest

import inputs
from tests.gpu_util import Job, assert_matches_oracle, register_all

pytestmark = pytest.mark.gpu


def mix(seed):
    return [Job("fib64", 14 + seed % 3), Job("nqueens", 6),
            Job("msort", keys=inputs.keys_u32(5000 + 37 * seed, 300 + seed)),
            Job("msort", keys=inputs.keys_u32(65, 400 + seed))]


def test_chain_lengths_and_recapture():
    import paper_1608_00571_amd as T
    shapes = [(256, 1), (256, 2), (512, 3), (1024, 4), (512, 5), (256, 6), (1024, 7), (512, 8), (512, 8)]
    done = []
    with T.Context(256 << 20, sched="graph", wg=shapes[0][0], graph_chunk=shapes[0][1], trace=True,
                   timeout_s=20.0) as ctx:
        register_all(ctx, mix(0))
        for k, (wg, chunk) in enumerate(shapes):
            ctx.set_schedule("graph", wg=wg, graph_chunk=chunk)
            jobs = mix(k)
            for j in jobs:
                j.submit(ctx)
            rs = ctx.run()
            for j in jobs:
                j.collect(ctx, trace=True)
            assert rs.stop_reason == 1
            assert rs.global_epochs == max(j.stats.epochs for j in jobs)
            done.append(jobs)
    for jobs in done:
        for j in jobs:
            assert_matches_oracle(j)


def test_budget_inside_a_chain_then_resume():
    """An epoch budget that ends the run in the middle of a chain: the chain's
    remaining epoch launches find the run stopped and return, the header the
    host reads says so, and a further run finishes every tree."""
    import paper_1608_00571_amd as T
    jobs = mix(5)
    with T.Context(256 << 20, sched="graph", wg=512, graph_chunk=8, trace=True, timeout_s=20.0) as ctx:
        register_all(ctx, jobs)
        for j in jobs:
            j.submit(ctx)
        rs = ctx.run(max_epochs=3)
        assert rs.stop_reason == 2 and rs.global_epochs == 3 and rs.live >= 1
        rs = ctx.run()
        assert rs.stop_reason == 1
        for j in jobs:
            j.collect(ctx, trace=True)
    for j in jobs:
        assert_matches_oracle(j)
