"""GPU parity: every program, under every scheduler, through the C ABI,
element by element against the CPU oracle (results, per-tree statistics and
the per-epoch trace; all integer, so bit-exact)."""
import numpy as np
import pytest

import inputs
from tests.gpu_util import SCHEDS, Job, assert_matches_oracle, register_all

pytestmark = pytest.mark.gpu

ARENA = 256 << 20


def make_ctx(sched, trace=True, **kw):
    import paper_1608_00571_amd as T
    return T.Context(ARENA, sched=sched, trace=trace, timeout_s=20.0, **kw)


def run_alone(sched, jobs, trace=True, **kw):
    with make_ctx(sched, trace=trace, **kw) as ctx:
        register_all(ctx, jobs)
        for j in jobs:
            j.submit(ctx)
        ctx.run()
        for j in jobs:
            j.collect(ctx, trace=trace)
    return jobs


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("kind", ["fib32", "fib64"])
def test_fib(sched, kind):
    for n in [0, 1, 2, 3, 5, 10, 17, 22]:
        (j,) = run_alone(sched, [Job(kind, n)])
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", SCHEDS)
def test_nqueens(sched):
    for n in range(1, 10):
        (j,) = run_alone(sched, [Job("nqueens", n)])
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
@pytest.mark.parametrize("wg", [256, 512, 1024])
def test_nqueens_wide_boards(sched, wg):
    """Boards of 12 to 14 columns: up to 14 children per task, so a
    wavefront step's children span many 64-entry rows of its block (the
    single-tree step writes them with consecutive lanes on consecutive
    entries); a fib tree beside them keeps the other program in the kernel."""
    import paper_1608_00571_amd as T
    jobs = [Job("nqueens", n) for n in (12, 13, 14)] + [Job("fib64", 20)]
    arena = (sum(T.tv_bound(T.NQUEENS, [n]) for n in (12, 13, 14)) + T.tv_bound(T.FIB_I64, [20]) + 4096) \
        * T.BYTES_PER_ENTRY
    with T.Context(arena, sched=sched, wg=wg, timeout_s=20.0) as ctx:
        register_all(ctx, jobs)
        for j in jobs:
            j.submit(ctx)
        ctx.run()
        for j in jobs:
            j.collect(ctx)
    for j in jobs:
        assert_matches_oracle(j, check_trace=False)


MSORT_SIZES = [0, 1, 2, 63, 64, 65, 129, 1000, 4096, (1 << 16) + 3]


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("nomap", [False, True])
def test_msort(sched, nomap):
    """Merges as data-parallel map jobs (default) and serially in their lane
    (the naive form): same output, same task statistics."""
    for n in MSORT_SIZES:
        keys = inputs.keys_u32(n, 1000 + n)
        (j,) = run_alone(sched, [Job("msort", keys=keys)], nomap=nomap)
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", SCHEDS)
def test_msort_large_map(sched):
    """2^20 + 5 keys (ragged halves): map jobs span many tiles at the top and
    many jobs share a tile at the bottom; also heavy duplicates, and keys equal
    to the largest key (which the merge pads halves with)."""
    for n, mod in [((1 << 20) + 5, None), (300000, 7), (200003, "top")]:
        keys = inputs.keys_u32(n, 77 + n)
        if mod == "top":   # keys in the top eight values: many equal the largest key
            keys = keys | np.uint32(0xFFFFFFF8)
        elif mod:
            keys = keys % np.uint32(mod)
        (j,) = run_alone(sched, [Job("msort", keys=keys)], trace=False)
        assert_matches_oracle(j)


def tiny_graphs():
    from tests.test_oracle_bfs import tiny_graphs as tg
    out = []
    for name, (V, arcs, s) in tg().items():
        out.append((name, inputs.csr_from_arcs(V, arcs, s)))
    for scale, seed in [(8, 1), (10, 2), (12, 3)]:
        out.append((f"rmat{scale}", inputs.rmat(scale, seed)))
    return out


@pytest.mark.parametrize("sched", SCHEDS)
def test_bfs(sched):
    for name, g in tiny_graphs():
        (j,) = run_alone(sched, [Job("bfs", graph=g)])
        assert_matches_oracle(j)


def sssp_jobs(lo=1, hi=100, seed=900):
    """Each tiny graph and R-MAT graph with seeded arc weights on [lo, hi]
    (in the graph's CSR order)."""
    return [Job("sssp", graph=g, weights=inputs.arc_weights(g.E, seed + i, lo, hi))
            for i, (name, g) in enumerate(tiny_graphs())]


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("lo,hi", [(1, 100), (0, 3), (7, 7)])
def test_sssp(sched, lo, hi):
    """Shortest distances equal Dijkstra's: weights 1..100, weights 0..3
    (zero-weight arcs and many equal-length paths) and one weight for every
    arc (distances are 7 x BFS depth)."""
    for j in sssp_jobs(lo, hi):
        run_alone(sched, [j])
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("delta", [1, 16, 1 << 20])
def test_sssp_buckets(sched, delta):
    """With a bucket width, visits that are not due wait (fork themselves
    unchanged): the distances are still Dijkstra's, every epoch is at its
    depth, and the run spans at least max distance // delta + 1 epochs."""
    for j in sssp_jobs(1, 100, seed=950):
        j.delta = delta
        j.cap = 256 * j.graph.V + 4096
        run_alone(sched, [j])
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", SCHEDS)
def test_sssp_batch(sched):
    """16 weighted R-MAT graphs of scale 10..16 in one run."""
    jobs = []
    for g in range(16):
        gr, w = inputs.sssp_graph(10 + g % 7, 700 + g)
        jobs.append(Job("sssp", graph=gr, weights=w))
    run_alone(sched, jobs, trace=False)
    for j in jobs:
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", SCHEDS)
def test_sssp_arena_overflow(sched):
    """A tree whose visits outgrow its arena fails with OVERFLOW, and a tree
    of another program in the same run is unaffected."""
    import paper_1608_00571_amd as T
    g, w = inputs.sssp_graph(10, 32)   # the source reaches 814 vertices in 2223 visits
    bad = Job("sssp", graph=g, weights=w, cap=64)
    ok = Job("fib64", 16)
    with make_ctx(sched) as ctx:
        register_all(ctx, [bad, ok])
        bad.submit(ctx)
        ok.submit(ctx)
        ctx.run()
        with pytest.raises(T.TreesError) as e:
            ctx.results(bad.tree)
        assert e.value.status == T.E_OVERFLOW
        ok.collect(ctx, trace=True)
    assert_matches_oracle(ok)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
def test_sssp_full_scale_graph(sched):
    """One weighted graph of 2^20 vertices and 2^24 arcs."""
    g, w = inputs.sssp_graph(20, 5)
    (j,) = run_alone(sched, [Job("sssp", graph=g, weights=w)], trace=False)
    assert_matches_oracle(j, check_trace=False)


def bintree(left, right, root):
    return (np.asarray(left, dtype=np.int32), np.asarray(right, dtype=np.int32), root)


@pytest.mark.parametrize("sched", SCHEDS)
def test_postorder_fig3(sched, golden_dir):
    """Figure 2's postorder program on the paper's worked example: the
    per-epoch trace is Figure 3's (CEN 0,1,2,3,2,1,0; 4 lanes launched and 3
    valid when CEN first falls back to 2)."""
    from tests.test_oracle_tvm import read_fig3
    left, right, want = read_fig3(golden_dir)
    (j,) = run_alone(sched, [Job("postorder", bintree=bintree(left, right, 0))])
    assert_matches_oracle(j)
    got = [(int(r["epoch"]), int(r["cen"]), int(r["b"]), int(r["e"]) - 1, int(r["launched"]), int(r["valid"]))
           for r in j.trace]
    assert got == want
    assert j.stats.peak_entries == 13


@pytest.mark.parametrize("sched", SCHEDS)
def test_postorder_random_trees(sched):
    """Random binary trees up to 20,000 nodes (up to 40,001 tasks an epoch
    apart in the widest epochs), a one-node tree and the empty tree."""
    jobs = [Job("postorder", bintree=bintree(*inputs.binary_tree(n, seed), 0))
            for n, seed in [(1, 0), (2, 5), (300, 3), (20000, 7)]]
    jobs.append(Job("postorder", bintree=bintree([-1], [-1], -1)))
    for j in jobs:
        (j,) = run_alone(sched, [j])
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", SCHEDS)
def test_preorder_trees(sched, golden_dir):
    """Figure 2's preorder program: Figure 3's tree, random binary trees up
    to 20,000 nodes, a subtree root, a one-node tree and the empty tree; the
    per-epoch trace equals the oracle's (epoch k runs depth k)."""
    from tests.test_oracle_tvm import read_fig3
    left, right, _ = read_fig3(golden_dir)
    jobs = [Job("preorder", bintree=bintree(left, right, 0))]
    jobs += [Job("preorder", bintree=bintree(*inputs.binary_tree(n, seed), root))
             for n, seed, root in [(1, 0, 0), (2, 5, 0), (300, 3, 0), (300, 3, 17), (20000, 7, 0)]]
    jobs.append(Job("preorder", bintree=bintree([-1], [-1], -1)))
    for j in jobs:
        (j,) = run_alone(sched, [j])
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
def test_mixed_batch_equals_alone(sched):
    """Independent trees of every program share epochs; each tree's result,
    statistics and trace equal its own oracle run; the batch takes as many
    global epochs as its longest tree."""
    jobs = []
    for k, n in [("fib64", 15), ("nqueens", 7), ("fib32", 9), ("nqueens", 5), ("fib64", 1)]:
        jobs.append(Job(k, n))
    jobs.append(Job("msort", keys=inputs.keys_u32(3000, 5)))
    jobs.append(Job("msort", keys=inputs.keys_u32(64, 6)))
    jobs.append(Job("bfs", graph=inputs.rmat(9, 4)))
    jobs.append(Job("bfs", graph=inputs.csr_from_arcs(5, [(0, 1), (1, 2), (2, 3), (3, 4)], 0)))
    jobs.append(Job("postorder", bintree=bintree(*inputs.binary_tree(500, 11), 0)))
    jobs.append(Job("preorder", bintree=bintree(*inputs.binary_tree(700, 13), 0)))
    jobs.append(Job("fft", signal=inputs.complex_signal(1 << 12, 14)))
    gs, ws = inputs.sssp_graph(9, 12)
    jobs.append(Job("sssp", graph=gs, weights=ws))
    with make_ctx(sched) as ctx:
        register_all(ctx, jobs)
        for j in jobs:
            j.submit(ctx)
        rs = ctx.run()
        for j in jobs:
            j.collect(ctx, trace=True)
    for j in jobs:
        assert_matches_oracle(j)
        assert j.stats.start_epoch == 0
        assert j.stats.done_epoch == j.stats.epochs - 1
    assert rs.global_epochs == max(j.stats.epochs for j in jobs)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
def test_many_small_trees(sched):
    """Hundreds of small trees: work-groups straddle many trees, so the
    segmented fork allocation and per-tree finishing are exercised."""
    mix = inputs.batch_mix(600, fib_range=(0, 12), nq_range=(1, 7))
    jobs = [Job("fib64" if k == "fib" else "nqueens", n) for k, n in mix]
    with make_ctx(sched) as ctx:
        register_all(ctx, jobs)
        for j in jobs:
            j.submit(ctx)
        ctx.run()
        for j in jobs:
            j.collect(ctx, trace=True)
    for j in jobs:
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", SCHEDS)
def test_bfs_batch(sched):
    """16 R-MAT graphs of scale 10..16 in one run: hubs with thousands of
    arcs, many trees per chunk, claim queues flushed several times."""
    scales = [10 + (g % 7) for g in range(16)]
    jobs = [Job("bfs", graph=inputs.rmat(sc, 500 + g)) for g, sc in enumerate(scales)]
    run_alone(sched, jobs, trace=True)
    for j in jobs:
        assert_matches_oracle(j)


def hub_graph():
    """Vertex 0 has 50,000 out-arcs (its chunk publishes an arc job); each
    leaf points into a second layer of 10,000 vertices whose chunks hold 8
    arcs per vertex (jobs whose tiles span many items)."""
    V = 60001
    arcs = [(0, i) for i in range(1, 50001)]
    arcs += [(i, 50001 + i % 10000) for i in range(1, 50001)]
    arcs += [(50001 + i, 50001 + (i + d) % 10000) for i in range(10000) for d in range(1, 9)]
    return inputs.csr_from_arcs(V, arcs, 0)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
@pytest.mark.parametrize("wg", [256, 512, 1024])
def test_bfs_arc_phase(sched, wg):
    """Chunks with many arcs hand them to the arc phase; the hub tree and a
    small tree in the same epochs both match the oracle."""
    jobs = [Job("bfs", graph=hub_graph()), Job("bfs", graph=inputs.rmat(9, 4))]
    run_alone(sched, jobs, wg=wg)
    for j in jobs:
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
@pytest.mark.parametrize("wg", [256, 512, 1024])
def test_sssp_arc_phase(sched, wg):
    """Relaxations in the arc phase: the hub graph with weights on [0, 9]
    (many improvements of one vertex inside an epoch, so many stale visits),
    beside a BFS tree of the same hub graph whose arcs share the phase."""
    g = hub_graph()
    jobs = [Job("sssp", graph=g, weights=inputs.arc_weights(g.E, 41, 0, 9)), Job("bfs", graph=g),
            Job("sssp", graph=inputs.rmat(9, 4), weights=inputs.arc_weights(inputs.rmat(9, 4).E, 42))]
    run_alone(sched, jobs, wg=wg)
    for j in jobs:
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
def test_bfs_full_scale_graph(sched):
    """One graph at the batch's largest scale (2^22 vertices, 2^26 arcs)."""
    g = inputs.bfs_batch_graph(0, 22)
    (j,) = run_alone(sched, [Job("bfs", graph=g)], trace=False)
    assert_matches_oracle(j, check_trace=False)


@pytest.mark.parametrize("sched", SCHEDS)
def test_arena_reuse_across_runs(sched):
    """Three rounds on one context whose arena fits about one round: every
    program's trees reuse the task-vector entries earlier trees left behind
    (stale codes and arguments), and each result still equals its oracle's."""
    import paper_1608_00571_amd as T

    def round_jobs(r):
        g, w = inputs.sssp_graph(9, 60 + r)
        return [Job("fib64", 17 + r), Job("nqueens", 6 + r), Job("msort", keys=inputs.keys_u32(5000 + r, 70 + r)),
                Job("bfs", graph=inputs.rmat(9, 80 + r)), Job("sssp", graph=g, weights=w),
                Job("postorder", bintree=bintree(*inputs.binary_tree(900, 90 + r), 0)),
                Job("preorder", bintree=bintree(*inputs.binary_tree(700, 95 + r), 0)),
                Job("fft", signal=inputs.complex_signal(1 << (10 + r), 99 + r))]

    rounds = [round_jobs(r) for r in range(3)]
    with make_ctx(sched, trace=True) as ctx:
        register_all(ctx, [j for jobs in rounds for j in jobs])
        for jobs in rounds:
            for j in jobs:
                j.submit(ctx)
            ctx.run()
            for j in jobs:
                j.collect(ctx, trace=True)
            for j in jobs:
                assert_matches_oracle(j)
        assert ctx.num_trees == 0
