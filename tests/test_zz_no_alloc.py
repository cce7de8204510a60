"""The allocation-free worklist BFS (trees_wl_bfs_noalloc, workspace in the
library's fixed device array) against trees_wl_bfs with a caller's
workspace: identical depths, iteration and push counts on consecutive calls,
a large graph then smaller ones (the array keeps the previous call's
contents, so each call must initialise what it reads), and the oracle's
depths; a graph beyond the array's limit is refused."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    return t if t.numel() else torch.zeros(1, dtype=torch.int32, device="cuda")


def test_noalloc_equals_workspace_form():
    import torch

    import paper_1608_00571_amd as T
    from tests.test_gpu_parity import tiny_graphs
    graphs = [inputs.rmat(20, 31), inputs.rmat(12, 32)] + [g for _, g in tiny_graphs()[:4]]
    with T.Context(1 << 20, sched="plain", wg=512) as ctx:
        for g in graphs:
            rp, ci = to_dev(g.row_ptr), to_dev(g.col_idx)
            ws = torch.empty(T.wl_workspace_bytes(g.V), dtype=torch.uint8, device="cuda")
            d_ref = torch.full((g.V,), -7, dtype=torch.int32, device="cuda")
            st_ref = ctx.wl_bfs(g.V, g.source, rp, ci, d_ref, ws)
            d = torch.full((g.V,), -9, dtype=torch.int32, device="cuda")
            st = ctx.wl_bfs_noalloc(g.V, g.source, rp, ci, d)
            got, ref = d.cpu().numpy(), d_ref.cpu().numpy()
            assert np.array_equal(got, ref), f"V={g.V}: depths differ"
            assert (st.iterations, st.pushed) == (st_ref.iterations, st_ref.pushed)
            want = oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source)
            assert np.array_equal(got, want)
    # a second context on the same GPU uses the same array
    g = inputs.rmat(10, 33)
    with T.Context(1 << 20, sched="plain", wg=256) as ctx:
        d = torch.empty(g.V, dtype=torch.int32, device="cuda")
        st = ctx.wl_bfs_noalloc(g.V, g.source, to_dev(g.row_ptr), to_dev(g.col_idx), d)
        want = oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source)
        assert np.array_equal(d.cpu().numpy(), want)
        assert st.iterations == int(want.max()) + 1


def test_noalloc_refuses_graphs_beyond_its_array():
    import torch

    import paper_1608_00571_amd as T
    dummy = torch.zeros(4, dtype=torch.int32, device="cuda")
    with T.Context(1 << 20, sched="plain") as ctx:
        with pytest.raises(T.TreesError) as e:
            ctx.wl_bfs_noalloc((1 << 22) + 1, 0, dummy, dummy, dummy)
        assert e.value.status == T.E_INVALID
