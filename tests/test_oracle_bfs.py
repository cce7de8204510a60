"""Pins of the oracle's breadth-first search (Section 6.3's task-per-vertex
bfs) and of the emulated VISIT task program.

Expected values: brute-force hop distances on tiny graphs (Bellman-Ford style
relaxation over the arc list), scipy's unweighted shortest paths (a library
routine), and the defining invariants of BFS depths."""
import numpy as np
import pytest

import inputs
import oracle


def brute_depths(V, arcs, src):
    INF = 1 << 30
    d = [INF] * V
    d[src] = 0
    for _ in range(V):
        for u, v in arcs:
            if d[u] + 1 < d[v]:
                d[v] = d[u] + 1
    return np.array([x if x < INF else -1 for x in d], dtype=np.int32)


def tiny_graphs():
    g = {}
    g["path"] = (6, [(i, i + 1) for i in range(5)], 0)
    g["star"] = (7, [(0, i) for i in range(1, 7)], 0)
    g["star_leaf_src"] = (7, [(0, i) for i in range(1, 7)], 3)
    g["cycle"] = (5, [(i, (i + 1) % 5) for i in range(5)], 2)
    g["complete"] = (5, [(i, j) for i in range(5) for j in range(5) if i != j], 1)
    g["two_components"] = (6, [(0, 1), (1, 2), (3, 4), (4, 5)], 0)
    g["self_loops_multi"] = (4, [(0, 0), (0, 1), (0, 1), (1, 1), (1, 2), (2, 0), (1, 2)], 0)
    g["isolated_source"] = (4, [(1, 2), (2, 3)], 0)
    g["single"] = (1, [], 0)
    g["diamond_back"] = (5, [(0, 1), (0, 2), (1, 3), (2, 3), (3, 4), (4, 0)], 0)
    return g


def check_invariants(g, depth):
    V, rp, ci, s = g.V, g.row_ptr, g.col_idx, g.source
    assert depth[s] == 0
    src = np.repeat(np.arange(V, dtype=np.int64), np.diff(rp))
    du = depth[src]
    dv = depth[ci]
    reached = du >= 0
    # an arc out of a reached vertex reaches a vertex at most one level deeper
    assert np.all(dv[reached] >= 0) and np.all(dv[reached] <= du[reached] + 1)
    # every reached vertex other than the source has an in-arc from the level above
    has_parent = np.zeros(V, dtype=bool)
    m = reached & (dv == du + 1)
    has_parent[ci[m]] = True
    need = (depth > 0)
    assert np.all(has_parent[need])


@pytest.mark.parametrize("name", list(tiny_graphs()))
def test_tiny_graphs_brute_force(name):
    V, arcs, s = tiny_graphs()[name]
    g = inputs.csr_from_arcs(V, arcs, s)
    want = brute_depths(V, arcs, s)
    assert np.array_equal(oracle.bfs_queue(V, g.row_ptr, g.col_idx, s), want)
    d, r = oracle.bfs(V, g.row_ptr, g.col_idx, s)
    assert np.array_equal(d, want)
    assert r.tasks == int((want >= 0).sum())
    assert r.epochs == int(want.max()) + 1


@pytest.mark.parametrize("scale,seed", [(8, 1), (10, 2), (12, 3)])
def test_rmat_vs_scipy(scale, seed):
    sp = pytest.importorskip("scipy.sparse")
    csg = pytest.importorskip("scipy.sparse.csgraph")
    g = inputs.rmat(scale, seed)
    A = sp.csr_matrix((np.ones(g.E), g.col_idx, g.row_ptr), shape=(g.V, g.V))
    dist = csg.shortest_path(A, directed=True, unweighted=True, indices=g.source)
    want = np.where(np.isinf(dist), -1, dist).astype(np.int32)
    d, r = oracle.bfs(g.V, g.row_ptr, g.col_idx, g.source, records=True)
    assert np.array_equal(d, want)
    assert np.array_equal(oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source), want)
    check_invariants(g, d)
    assert r.tasks == int((want >= 0).sum())
    assert r.epochs == int(want.max()) + 1
    # one epoch per BFS level; its valid tasks are that level's vertices
    counts = np.bincount(want[want >= 0])
    assert list(r.records["valid"]) == list(counts)
    assert r.peak == r.tasks  # nothing joins, so no entry is reclaimed


def test_invariant_check_catches_a_wrong_depth():
    g = inputs.rmat(9, 5)
    d, _ = oracle.bfs(g.V, g.row_ptr, g.col_idx, g.source)
    bad = d.copy()
    v = int(np.flatnonzero(d == 2)[0])
    bad[v] = 3
    with pytest.raises(AssertionError):
        check_invariants(g, bad)
