"""Pins of the epoch emulator's machine-level behaviour: the worked example of
Section 5.3 (Figures 2-4), stack and space properties of Sections 4.3.3 and
4.4, independent trees in shared epochs, checkpoint/resume and overflow."""
import os

import numpy as np
import pytest

import inputs
import oracle


def read_fig3(golden_dir):
    tree, epochs = {}, []
    with open(os.path.join(golden_dir, "fig3_postorder.txt")) as f:
        for line in f:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "tree":
                tree[int(p[1])] = (int(p[2]), int(p[3]))
            elif p[0] == "epoch":
                epochs.append(tuple(int(x) for x in p[1:]))
    n = len(tree)
    left = [tree[i][0] for i in range(n)]
    right = [tree[i][1] for i in range(n)]
    return left, right, epochs


def test_fig3_worked_example(golden_dir):
    left, right, want = read_fig3(golden_dir)
    order, ep, r = oracle.postorder(left, right, 0)
    got = [(int(x["epoch"]), int(x["cen"]), int(x["b"]), int(x["e"]) - 1, int(x["launched"]),
            int(x["valid"])) for x in r.records]
    assert got == want
    # CEN decreases for the first time after epoch 3 (Section 5.3)
    cens = [g[1] for g in got]
    assert cens == [0, 1, 2, 3, 2, 1, 0]
    assert r.peak == 13          # entries 0..12
    assert r.epochs == 7


def test_postorder_visits_children_first(golden_dir):
    left, right, _ = read_fig3(golden_dir)
    order, ep, r = oracle.postorder(left, right, 0)
    pos = {int(v): i for i, v in enumerate(order)}
    assert sorted(pos) == list(range(6))
    for v in range(6):
        for c in (left[v], right[v]):
            if c >= 0:
                assert pos[c] < pos[v]
                assert ep[c] < ep[v]


def random_tree(n, seed):
    left = [-1] * n
    right = [-1] * n
    for v in range(1, n):
        k = 0
        while True:
            p = inputs.uniform(seed, v * 64 + k, 0, v - 1)
            side = inputs.uniform(seed, v * 64 + k + 32, 0, 1)
            arr = left if side == 0 else right
            if arr[p] == -1:
                arr[p] = v
                break
            k += 1
    return left, right


@pytest.mark.parametrize("n,seed", [(1, 0), (7, 1), (40, 2), (300, 3)])
def test_postorder_random_trees(n, seed):
    left, right = random_tree(n, seed)
    order, ep, r = oracle.postorder(left, right, 0)
    assert sorted(order.tolist()) == list(range(n))
    pos = {int(v): i for i, v in enumerate(order)}
    for v in range(n):
        for c in (left[v], right[v]):
            if c >= 0:
                assert pos[c] < pos[v]
    # every node and every NULL child is one postorder task; nodes also join
    assert r.tasks_by_type == (2 * n + 1, n)


def test_empty_postorder():
    order, ep, r = oracle.postorder([-1], [-1], -1)
    assert len(order) == 0 and r.tasks == 1 and r.epochs == 1


@pytest.mark.parametrize("prog", ["fib", "nqueens", "msort", "bfs"])
def test_space_bounds(prog):
    # Section 4.4.2: T1/Tinf <= space <= T1 (tasks as work, epochs as span)
    if prog == "fib":
        r = oracle.fib(17)
    elif prog == "nqueens":
        r = oracle.nqueens(8)
    elif prog == "msort":
        _, r = oracle.msort(inputs.keys_u32(3000, 1))
    else:
        g = inputs.rmat(10, 4)
        _, r = oracle.bfs(g.V, g.row_ptr, g.col_idx, g.source)
    assert r.tasks / r.epochs <= r.peak <= r.tasks


def make(spec):
    kind, n = spec
    if kind == "fib":
        return oracle.Emulator(oracle.FIB64, n, records=True), None
    if kind == "nqueens":
        return oracle.Emulator(oracle.NQUEENS, n, records=True), None
    if kind == "msort":
        a = inputs.keys_u32(n, 5 + n)
        t = np.zeros_like(a)
        return oracle.Emulator(oracle.MSORT, n, ptrs=(a, t, None, None), records=True), a
    g = inputs.rmat(n, 9 + n)
    d = np.empty(g.V, dtype=np.int32)
    return oracle.Emulator(oracle.BFS, g.V, g.source, ptrs=(g.row_ptr, g.col_idx, d, None),
                           records=True), d


def test_batch_equals_alone():
    specs = [("fib", 12), ("nqueens", 7), ("fib", 3), ("msort", 900), ("bfs", 8), ("fib", 0),
             ("nqueens", 5), ("fib", 19)]
    together = [make(s) for s in specs]
    g = oracle.run_batch([e for e, _ in together])
    alone = []
    for s in specs:
        e, p = make(s)
        e.run()
        alone.append((e, p))
    for (e1, p1), (e2, p2) in zip(together, alone):
        a, b = e1.stats(), e2.stats()
        assert (a.result, a.epochs, a.tasks, a.launched, a.peak, a.tasks_by_type) == \
               (b.result, b.epochs, b.tasks, b.launched, b.peak, b.tasks_by_type)
        assert np.array_equal(a.records, b.records)
        if p1 is not None:
            assert np.array_equal(p1, p2)
    # all trees start at global epoch 0, so the batch takes the longest tree's epochs
    assert g == max(e.stats().epochs for e, _ in alone)


@pytest.mark.parametrize("spec", [("fib", 16), ("nqueens", 7), ("msort", 5000), ("bfs", 10)])
@pytest.mark.parametrize("k", [0, 1, 5, 9])
def test_resume_from_snapshot(spec, k):
    straight, p_straight = make(spec)
    straight.run()
    want = straight.stats()

    first, p = make(spec)
    first.run(k)
    snap = first.snapshot()
    kind = first.kind
    if spec[0] == "msort":
        keys = p.copy()
        tmp = np.frombuffer(bytes(first._keep[1]), dtype=np.uint32).copy()
        resumed = oracle.Emulator.restore(kind, snap, (keys, tmp, None, None), records=True)
        payload = keys
    elif spec[0] == "bfs":
        depth = p.copy()
        rp, ci = first._keep[0], first._keep[1]
        resumed = oracle.Emulator.restore(kind, snap, (rp, ci, depth, None), records=True)
        payload = depth
    else:
        resumed = oracle.Emulator.restore(kind, snap, records=True)
        payload = None
    del first
    resumed.run()
    got = resumed.stats()
    assert (got.result, got.epochs, got.tasks, got.launched, got.peak, got.tasks_by_type) == \
           (want.result, want.epochs, want.tasks, want.launched, want.peak, want.tasks_by_type)
    if payload is not None:
        assert np.array_equal(payload, p_straight)


def test_overflow_is_reported():
    em = oracle.Emulator(oracle.FIB64, 12, cap=50)
    rc = em.run()
    assert rc == oracle.E_OVERFLOW
    assert em.stats().status == oracle.E_OVERFLOW


def test_exact_capacity_suffices():
    r = oracle.fib(14)
    em = oracle.Emulator(oracle.FIB64, 14, cap=r.peak)
    assert em.run() == 0
    assert em.stats().result == r.result
