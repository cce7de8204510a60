"""The seeded input generators: SplitMix64 against its published test vector,
C and Python draws agreeing, and the structural properties of the R-MAT
graphs, sort keys, tree batch and request trace."""
import os

import numpy as np

import inputs


def test_splitmix64_reference_vector(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64_seed1234567.txt")) as f:
        want = [int(x) for x in f if x.strip() and not x.startswith("#")]
    assert [inputs.draw(1234567, i) for i in range(5)] == want
    L = inputs.lib()
    assert [int(L.tin_draw(1234567, i)) for i in range(5)] == want


def test_c_and_python_agree():
    L = inputs.lib()
    for i in range(50):
        s = inputs.item_seed(3, i)
        assert int(L.tin_uniform(s, i, 6, 11)) == inputs.uniform(s, i, 6, 11)
    k = inputs.keys_u32(100, 42)
    assert [int(x) for x in k] == [inputs.draw(42, i) >> 32 for i in range(100)]


def test_keys_deterministic_and_spread():
    a = inputs.keys_u32(1 << 16, 9)
    b = inputs.keys_u32(1 << 16, 9)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, inputs.keys_u32(1 << 16, 10))
    # roughly uniform over [0, 2^32): each of 16 bins holds 1/16 +- 5%
    h = np.bincount(a >> np.uint32(28), minlength=16)
    assert np.all(np.abs(h / a.size - 1 / 16) < 0.05 / 16 * 16)


def test_permutation_is_a_permutation():
    p = inputs.permutation(7, 1000)
    assert sorted(p.tolist()) == list(range(1000))


def test_rmat_structure():
    g = inputs.rmat(12, 3)
    assert g.V == 4096 and g.E == 16 * 4096
    assert g.row_ptr[0] == 0 and g.row_ptr[-1] == g.E
    assert np.all(np.diff(g.row_ptr) >= 0)
    assert g.col_idx.min() >= 0 and g.col_idx.max() < g.V
    assert g.row_ptr[g.source + 1] > g.row_ptr[g.source]
    g2 = inputs.rmat(12, 3)
    assert np.array_equal(g.col_idx, g2.col_idx) and g.source == g2.source


def test_rmat_quadrant_frequencies():
    # before relabelling, the top bit of (src, dst) follows (a, b, c, d)
    V, E = 1 << 10, 1 << 16
    src = np.empty(E, np.int32)
    dst = np.empty(E, np.int32)
    thr = np.array(inputs.RMAT_THRESHOLDS, dtype=np.uint32)
    inputs.lib().tin_rmat_edges(10, E, 5, thr.ctypes.data, src.ctypes.data, dst.ctypes.data)
    q = 2 * (src >= V // 2) + (dst >= V // 2)
    freq = np.bincount(q, minlength=4) / E
    assert np.allclose(freq, inputs.RMAT_PROBS, atol=0.01)


def test_batch_mix():
    m = inputs.batch_mix(4096)
    assert len(m) == 4096
    fibs = [n for k, n in m if k == "fib"]
    nqs = [n for k, n in m if k == "nqueens"]
    assert len(fibs) == len(nqs) == 2048
    assert min(fibs) >= 10 and max(fibs) <= 28 and min(nqs) >= 6 and max(nqs) <= 11
    assert m == inputs.batch_mix(4096)


def test_serving_trace():
    tr = inputs.serving_trace(2000, 100.0)
    t = np.array([r.t_arrive for r in tr])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.01) < 0.001            # rate 100/s
    kinds = [r.kind for r in tr]
    for k, p in (("fib", 0.4), ("msort", 0.4), ("bfs", 0.2)):
        assert abs(kinds.count(k) / len(kinds) - p) < 0.04
    ms = [r.size for r in tr if r.kind == "msort"]
    assert min(ms) >= 1 << 10 and max(ms) <= 1 << 22


def test_binary_tree_matches_scalar_draws():
    """The C tree generator takes the same draws as the scalar definition
    (the oracle's postorder tests build their trees that way)."""
    from tests.test_oracle_tvm import random_tree
    for n, seed in [(1, 0), (7, 1), (40, 2), (300, 3), (2000, 9)]:
        left, right = random_tree(n, seed)
        L, R = inputs.binary_tree(n, seed)
        assert L.tolist() == left and R.tolist() == right


def test_binary_tree_is_a_tree():
    L, R = inputs.binary_tree(5000, 4)
    ch = np.concatenate([L[L >= 0], R[R >= 0]])
    assert len(ch) == 4999 and len(np.unique(ch)) == 4999 and 0 not in ch
    # every child comes after its parent
    for arr in (L, R):
        has = arr >= 0
        assert np.all(arr[has] > np.nonzero(has)[0])
