"""GPU parity at the benchmark's full sizes, in the launch configurations
bench.py times: the default line (fib(32) with 64-bit sums and a merge sort
of 2^24 keys under the plain scheduler, 1024 lanes) and the batch of 4096
fib / N-queens trees (graph and persistent forms, 512 lanes).  Every tree's
result and statistics equal the oracle's emulation; the sort's output is the
oracle's, key for key."""
import concurrent.futures
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


def test_graph_batches_full_size():
    """The 64 R-MAT graphs of the BFS and SSSP configurations (scale 16..22,
    E = 16 V; SSSP weights 1..100), in shared epochs under the graph form at
    512 lanes: every depth equals the queue BFS's, every distance Dijkstra's,
    and each BFS tree visits each reached vertex once in max depth + 1 epochs."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import oracle
    import paper_1608_00571_amd as T
    scales = inputs.bfs_batch_scales(64)
    gs = [inputs.sssp_batch_graph(g, sc) for g, sc in enumerate(scales)]
    with ThreadPoolExecutor(8) as ex:
        want_d = list(ex.map(lambda gw: oracle.bfs_queue(gw[0].V, gw[0].row_ptr, gw[0].col_idx, gw[0].source), gs))
        want_s = list(ex.map(lambda gw: oracle.dijkstra(gw[0].V, gw[0].row_ptr, gw[0].col_idx, gw[1],
                                                        gw[0].source), gs))
    V = sum(G.V for G, _ in gs)
    dev = [(torch.from_numpy(G.row_ptr).cuda(), torch.from_numpy(G.col_idx).cuda(), torch.from_numpy(w).cuda())
           for G, w in gs]
    for kind in (T.BFS_CSR, T.SSSP_CSR):
        cap = sum(T.tv_bound(kind, [G.V, G.source]) + 64 for G, _ in gs)
        outs = [torch.empty(G.V, dtype=torch.int32, device="cuda") for G, _ in gs]
        with make_ctx("graph", (cap + 4096) * T.BYTES_PER_ENTRY, wg=512, max_trees=64) as ctx:
            p = ctx.register(kind)
            ids = []
            for (G, _), (rp, ci, wt), o in zip(gs, dev, outs):
                bufs = [rp, ci, o] if kind == T.BFS_CSR else [rp, ci, wt, o]
                ids.append(ctx.submit(p, [G.V, G.source], bufs))
            ctx.run()
            stats = [ctx.results(t)[1] for t in ids]
        for o, wd, ws, st in zip(outs, want_d, want_s, stats):
            got = o.cpu().numpy()
            if kind == T.BFS_CSR:
                assert np.array_equal(got, wd)
                assert st.tasks == int((wd >= 0).sum()) and st.epochs == int(wd.max()) + 1
            else:
                assert np.array_equal(got, ws)
                assert st.tasks >= int((ws != oracle.UNREACHED).sum())
        del outs
    assert V > 7 * 10**7


@functools.lru_cache(maxsize=1)
def _fft_oracle_batch(m: int, n: int):
    """The oracle's fp64 transforms of the batch's n signals (computed once
    for both schedulers; the oracle's C code runs outside the interpreter
    lock, so the transforms go through a few threads)."""
    import oracle
    xs = [inputs.complex_signal(1 << m, 900 + g).astype(np.complex128) for g in range(n)]
    with concurrent.futures.ThreadPoolExecutor(8) as ex:
        return list(ex.map(lambda x: oracle.fft(x)[0], xs))


@pytest.mark.parametrize("sched", ["graph", "persistent"])
def test_fft_batch_full_size(sched):
    """The FFT configuration's batch, 64 transforms of 2^18 complex fp32
    points in shared epochs at 1024 lanes: every tree's statistics equal the
    oracle's, and every transform is compared with the oracle's fp64 run
    within the radix-2 error bound."""
    import torch

    import oracle
    import paper_1608_00571_amd as T
    from tests.gpu_util import fft_tolerance
    m, n = 18, 64
    xs = [inputs.complex_signal(1 << m, 900 + g) for g in range(n)]
    xt = [torch.from_numpy(x.view(np.float32).copy()).cuda() for x in xs]
    ys = [torch.empty_like(t) for t in xt]
    arena = (n * (T.tv_bound(T.FFT, [m]) + 64) + 4096) * T.BYTES_PER_ENTRY
    with make_ctx(sched, arena, wg=1024, max_trees=n) as ctx:
        p = ctx.register(T.FFT)
        ids = [ctx.submit(p, [m], [a, b]) for a, b in zip(xt, ys)]
        ctx.run()
        stats = [ctx.results(t)[1] for t in ids]
    _, r = oracle.fft(np.zeros(1 << m, dtype=np.complex128))
    tol = fft_tolerance(1 << m)
    for g, (x, y, st) in enumerate(zip(xs, ys, stats)):
        assert (st.tasks, st.epochs, st.peak_entries, st.launched) == (r.tasks, r.epochs, r.peak, r.launched)
        got = y.cpu().numpy().view(np.complex64).astype(np.complex128)
        want = _fft_oracle_batch(m, n)[g]
        assert np.linalg.norm(got - want) / np.linalg.norm(want) <= tol, g
