"""Native worklist BFS and SSSP (Section 6.3's hand-managed comparison)
through the C ABI: depths and distances equal the oracle's element by
element.  BFS's iteration and push counts follow from the depths (one
iteration per level, the deepest one pushing nothing; every reached vertex
but the source pushed once); SSSP's depend on the order of relaxations, so
they are checked against what every schedule satisfies."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


def run_wl(ctx, g, weights=None):
    import torch

    import paper_1608_00571_amd as T
    sssp = weights is not None
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int32)).cuda()
    ci = torch.from_numpy(np.ascontiguousarray(g.col_idx, dtype=np.int32)).cuda()
    if ci.numel() == 0:
        ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.full((g.V,), -7, dtype=torch.int32, device="cuda")
    ws = torch.empty(T.wl_workspace_bytes(g.V, sssp), dtype=torch.uint8, device="cuda")
    if sssp:
        w = torch.from_numpy(np.ascontiguousarray(weights, dtype=np.int32)).cuda()
        if w.numel() == 0:
            w = torch.zeros(1, dtype=torch.int32, device="cuda")
        st = ctx.wl_sssp(g.V, g.source, rp, ci, w, out, ws)
    else:
        st = ctx.wl_bfs(g.V, g.source, rp, ci, out, ws)
    return out.cpu().numpy(), st


def graphs():
    from tests.test_gpu_parity import hub_graph, tiny_graphs
    return tiny_graphs() + [("hub", hub_graph())]


def check_bfs(g, d, st):
    want = oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source)
    bad = np.flatnonzero(d != want)
    assert bad.size == 0, f"{bad.size} depths differ, first at {bad[:5]}"
    assert st.iterations == int(want.max()) + 1
    assert st.pushed == int(np.count_nonzero(want >= 0)) - 1


def check_sssp(g, w, d, st):
    want = oracle.dijkstra(g.V, g.row_ptr, g.col_idx, w, g.source)
    bad = np.flatnonzero(d != want)
    assert bad.size == 0, f"{bad.size} distances differ, first at {bad[:5]}"
    hops = oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source)
    reached = int(np.count_nonzero(want != oracle.UNREACHED))
    # every reached vertex but the source is pushed at least once, and a
    # vertex h arcs away is reached no earlier than iteration h
    assert st.pushed >= reached - 1
    assert st.iterations >= int(hops.max()) + 1


@pytest.mark.parametrize("wg", [256, 512, 1024])
def test_wl_bfs(wg):
    import paper_1608_00571_amd as T
    with T.Context(1 << 20, sched="plain", wg=wg) as ctx:
        for name, g in graphs():
            d, st = run_wl(ctx, g)
            check_bfs(g, d, st)


@pytest.mark.parametrize("wg", [256, 512])
@pytest.mark.parametrize("lo,hi", [(1, 100), (0, 3), (7, 7)])
def test_wl_sssp(wg, lo, hi):
    import paper_1608_00571_amd as T
    with T.Context(1 << 20, sched="plain", wg=wg) as ctx:
        for i, (name, g) in enumerate(graphs()):
            w = inputs.arc_weights(g.E, 300 + i, lo, hi)
            d, st = run_wl(ctx, g, w)
            check_sssp(g, w, d, st)


def test_wl_batch_graphs_full_scale():
    """Graphs of the 64-graph batch at scales 16, 19 and 22 (2^22 vertices,
    2^26 arcs), BFS and weighted SSSP, in the work-group size the bench
    times, reusing one workspace."""
    import torch

    import paper_1608_00571_amd as T
    with T.Context(1 << 20, sched="plain", wg=512) as ctx:
        for gi, sc in [(5, 16), (9, 19), (0, 22)]:
            g, w = inputs.sssp_batch_graph(gi, sc)
            d, st = run_wl(ctx, g)
            check_bfs(g, d, st)
            d, st = run_wl(ctx, g, w)
            check_sssp(g, w, d, st)
            torch.cuda.empty_cache()


def test_wl_argument_errors():
    import torch

    import paper_1608_00571_amd as T
    g = inputs.rmat(8, 1)
    rp = torch.from_numpy(g.row_ptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(g.col_idx.astype(np.int32)).cuda()
    d = torch.empty(g.V, dtype=torch.int32, device="cuda")
    need = T.wl_workspace_bytes(g.V)
    with T.Context(1 << 20, sched="plain") as ctx:
        small = torch.empty(need - 4, dtype=torch.uint8, device="cuda")
        with pytest.raises(T.TreesError) as e:
            ctx.wl_bfs(g.V, g.source, rp, ci, d, small)
        assert e.value.status == T.E_INVALID
        with pytest.raises(T.TreesError) as e:
            ctx.wl_bfs(g.V, g.V, rp, ci, d, torch.empty(need, dtype=torch.uint8, device="cuda"))
        assert e.value.status == T.E_INVALID
        big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
        with pytest.raises(T.TreesError) as e:   # not 256-byte aligned
            ctx.wl_bfs(g.V, g.source, rp, ci, d, big[4:])
        assert e.value.status == T.E_INVALID
        with pytest.raises(T.TreesError) as e:   # the output inside the workspace
            ctx.wl_bfs(g.V, g.source, rp, ci, big[256:256 + 4 * g.V].view(torch.int32), big)
        assert e.value.status == T.E_INVALID
        # the same context still runs a valid call afterwards
        st = ctx.wl_bfs(g.V, g.source, rp, ci, d, big)
        check_bfs(g, d.cpu().numpy(), st)
