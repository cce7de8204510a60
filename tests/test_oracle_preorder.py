"""Pins of the oracle's preorder program (Figure 2): preorder(node) visits
node, then forks preorder of both children; nothing joins.  Every value
below is computed from the tree alone (depths by an explicit walk), not by
the emulator."""
import numpy as np
import pytest

import oracle
from tests.test_oracle_tvm import random_tree, read_fig3


def depths(left, right, root):
    """Depth of every node reachable from root (-1 elsewhere), by a walk."""
    d = [-1] * len(left)
    stack = [(root, 0)] if root >= 0 else []
    while stack:
        v, k = stack.pop()
        d[v] = k
        for c in (left[v], right[v]):
            if c >= 0:
                stack.append((c, k + 1))
    return d


def expected_trace(left, right, root):
    """Epoch k runs the preorder tasks at depth k (nodes and empty children);
    the tasks of epoch k + 1 are the two children of each node at depth k,
    allocated right after epoch k's range."""
    d = depths(left, right, root)
    nodes = np.bincount([x for x in d if x >= 0]) if root >= 0 else np.zeros(0, dtype=np.int64)
    recs, b, e = [], 0, 1
    for k in range(len(nodes) + 1):
        nk = int(nodes[k]) if k < len(nodes) else 0
        recs.append((k, k, b, e, e - b, e - b, 2 * nk, 0, e + 2 * nk))
        b, e = e, e + 2 * nk
    return recs


def test_fig3_tree_preorder(golden_dir):
    left, right, _ = read_fig3(golden_dir)
    order, ep, r = oracle.preorder(left, right, 0)
    got = [tuple(int(x[f]) for f in ("epoch", "cen", "b", "e", "launched", "valid", "forks", "joins", "nfc"))
           for x in r.records]
    assert got == expected_trace(left, right, 0)
    assert list(ep) == depths(left, right, 0)
    assert r.tasks == 2 * 6 + 1 and r.peak == 2 * 6 + 1


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (50, 2), (1000, 3), (5000, 4)])
def test_preorder_random_trees(n, seed):
    left, right = random_tree(n, seed)
    order, ep, r = oracle.preorder(left, right, 0)
    d = depths(left, right, 0)
    assert sorted(order.tolist()) == list(range(n))
    assert list(ep) == d                                  # a node is visited in the epoch of its depth
    assert all(d[a] <= d[b] for a, b in zip(order[:-1], order[1:]))   # so the log goes level by level
    assert r.tasks == 2 * n + 1 and r.peak == 2 * n + 1 and r.epochs == max(d) + 2
    assert [tuple(int(x[f]) for f in ("epoch", "cen", "b", "e", "launched", "valid", "forks", "joins", "nfc"))
            for x in r.records] == expected_trace(left, right, 0)


def test_preorder_subtree_and_empty():
    left, right = random_tree(300, 9)
    root = 17                                             # a subtree: only its nodes are visited
    order, ep, r = oracle.preorder(left, right, root)
    d = depths(left, right, root)
    assert sorted(order.tolist()) == [v for v in range(300) if d[v] >= 0]
    order, ep, r = oracle.preorder([-1], [-1], -1)
    assert len(order) == 0 and r.tasks == 1 and r.epochs == 1
