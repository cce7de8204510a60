"""Pins of the SSSP oracle: Dijkstra against an independent library routine
(scipy), brute force on tiny graphs, BFS under unit weights and the
optimality conditions; the emulator's relaxation program against Dijkstra
(task counts are one schedule's and not compared)."""
import numpy as np
import pytest

import inputs
import oracle

INF = oracle.UNREACHED


def scipy_dist(g, w):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra
    src = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    # duplicate arcs: keep the lightest (csr_matrix would add them up)
    best = {}
    for s, d, x in zip(src.tolist(), g.col_idx.tolist(), w.tolist()):
        if (s, d) not in best or x < best[(s, d)]:
            best[(s, d)] = x
    if not best:
        out = np.full(g.V, INF, dtype=np.int64)
        out[g.source] = 0
        return out
    ks = np.array(list(best.keys()))
    vs = np.array(list(best.values()), dtype=np.float64)
    # zero weights would vanish from a sparse matrix: shift every weight by a
    # tiny epsilon (paths here have < 10^4 arcs, so ordering is kept)
    m = csr_matrix((vs + 1e-9, (ks[:, 0], ks[:, 1])), shape=(g.V, g.V))
    d = sp_dijkstra(m, indices=g.source)
    out = np.where(np.isinf(d), INF, np.floor(d + 1e-6)).astype(np.int64)
    return out


@pytest.mark.parametrize("scale,seed,lo,hi", [(6, 1, 1, 100), (9, 2, 1, 100), (10, 3, 0, 3), (11, 4, 1, 1)])
def test_dijkstra_matches_scipy(scale, seed, lo, hi):
    g, w = inputs.sssp_graph(scale, seed, lo, hi)
    d = oracle.dijkstra(g.V, g.row_ptr, g.col_idx, w, g.source)
    assert np.array_equal(d.astype(np.int64), scipy_dist(g, w))


def floyd_warshall(V, arcs):
    D = np.full((V, V), np.iinfo(np.int64).max // 4, dtype=np.int64)
    np.fill_diagonal(D, 0)
    for u, v, x in arcs:
        D[u, v] = min(D[u, v], x)
    for k in range(V):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def test_dijkstra_brute_force_tiny():
    for seed in range(30):
        V = 1 + seed % 7
        arcs = []
        for i in range(3 * V):
            u = inputs.uniform(seed, 3 * i, 0, V - 1)
            v = inputs.uniform(seed, 3 * i + 1, 0, V - 1)
            arcs.append((u, v, inputs.uniform(seed, 3 * i + 2, 0, 9)))
        g = inputs.csr_from_arcs(V, [(u, v) for u, v, _ in arcs], 0)
        # csr_from_arcs keeps arcs in a stable order per source: weights follow
        order = sorted(range(len(arcs)), key=lambda i: arcs[i][0])
        w = np.array([arcs[i][2] for i in order], dtype=np.int32)
        d = oracle.dijkstra(g.V, g.row_ptr, g.col_idx, w, g.source)
        D = floyd_warshall(V, arcs)[g.source]
        want = np.where(D >= np.iinfo(np.int64).max // 8, INF, D)
        assert np.array_equal(d.astype(np.int64), want), seed


def test_unit_weights_give_bfs_depths():
    for scale, seed in [(8, 1), (12, 5)]:
        g = inputs.rmat(scale, seed)
        w = np.ones(g.col_idx.shape[0], dtype=np.int32)
        d = oracle.dijkstra(g.V, g.row_ptr, g.col_idx, w, g.source)
        b = oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source)
        assert np.array_equal(d, np.where(b < 0, INF, b))


def check_optimal(g, w, d):
    """d[source] = 0; no arc can shorten a distance; every reached vertex
    other than the source is reached by an arc that attains its distance."""
    assert d[g.source] == 0
    src = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    reach = d[src] != INF
    nd = d[src].astype(np.int64) + w
    assert np.all(d[g.col_idx[reach]].astype(np.int64) <= nd[reach])
    tight = np.zeros(g.V, dtype=bool)
    tight[g.col_idx[reach & (d[g.col_idx].astype(np.int64) == nd)]] = True
    others = (d != INF) & (np.arange(g.V) != g.source)
    assert np.all(tight[others])


@pytest.mark.parametrize("scale,seed,lo,hi", [(8, 1, 1, 100), (12, 2, 1, 100), (12, 3, 0, 3)])
def test_relaxation_program_reaches_dijkstra(scale, seed, lo, hi):
    g, w = inputs.sssp_graph(scale, seed, lo, hi)
    want = oracle.dijkstra(g.V, g.row_ptr, g.col_idx, w, g.source)
    check_optimal(g, w, want)
    d, r = oracle.sssp(g.V, g.row_ptr, g.col_idx, w, g.source, records=True)
    assert np.array_equal(d, want)
    reached = int(np.sum(want != INF))
    assert r.tasks >= reached          # every reached vertex is visited at least once
    assert r.epochs >= 1


def test_sssp_source_only():
    g = inputs.csr_from_arcs(3, [], 0)
    d, r = oracle.sssp(g.V, g.row_ptr, g.col_idx, np.zeros(0, np.int32), g.source)
    assert d.tolist() == [0, INF, INF] and r.tasks == 1 and r.epochs == 1


@pytest.mark.parametrize("delta", [1, 3, 16, 100])
@pytest.mark.parametrize("scale,seed,lo,hi", [(8, 5, 1, 100), (10, 6, 0, 9)])
def test_bucketed_program_reaches_dijkstra(delta, scale, seed, lo, hi):
    """With a bucket width, a visit waits (re-forks itself unchanged) until
    (CEN + 1) * delta exceeds its distance: the distances are still
    Dijkstra's, and a vertex at distance d is relaxed no earlier than epoch
    floor(d / delta), so the run has at least floor(max d / delta) + 1 epochs."""
    g, w = inputs.sssp_graph(scale, seed, lo, hi)
    want = oracle.dijkstra(g.V, g.row_ptr, g.col_idx, w, g.source)
    d, r = oracle.sssp(g.V, g.row_ptr, g.col_idx, w, g.source, delta=delta)
    assert np.array_equal(d, want)
    reached = want[want != INF]
    assert r.epochs >= int(reached.max()) // delta + 1
    assert r.tasks >= reached.size


def test_bucket_wider_than_every_distance_changes_nothing():
    """A bucket wider than any distance never delays a visit: the run is the
    plain program's, epoch for epoch."""
    g, w = inputs.sssp_graph(9, 7)
    d0, r0 = oracle.sssp(g.V, g.row_ptr, g.col_idx, w, g.source, records=True)
    d1, r1 = oracle.sssp(g.V, g.row_ptr, g.col_idx, w, g.source, records=True, delta=1 << 30)
    assert np.array_equal(d0, d1)
    assert (r0.tasks, r0.epochs, r0.peak) == (r1.tasks, r1.epochs, r1.peak)
    assert np.array_equal(r0.records, r1.records)

