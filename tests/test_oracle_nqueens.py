"""Pins of the oracle's N-queens evaluators (Section 6.5's nqueens program).

Expected values: the textbook table of solution counts (golden fixture),
brute force over permutations, and an explicit enumeration of partial
placements written with lists of columns (no bitmasks), which fixes the task
counts of the one-task-per-partial-placement program."""
import itertools
import os

import pytest

import oracle


def golden_counts(golden_dir):
    out = {}
    with open(os.path.join(golden_dir, "nqueens_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, c = line.split()
                out[int(n)] = int(c)
    return out


def brute_force_solutions(n: int) -> int:
    return sum(1 for p in itertools.permutations(range(n))
               if all(abs(p[i] - p[j]) != j - i for i in range(n) for j in range(i + 1, n)))


def partial_placements(n: int):
    """All non-attacking placements of queens in rows 0..r-1, r = 0..n, as
    tuples of columns; and for each, its number of legal extensions."""
    def ok(cols, c):
        r = len(cols)
        return all(c != q and abs(c - q) != r - i for i, q in enumerate(cols))

    nodes = []
    frontier = [()]
    while frontier:
        nxt = []
        for cols in frontier:
            ext = [cols + (c,) for c in range(n) if len(cols) < n and ok(cols, c)]
            nodes.append((cols, len(ext)))
            nxt.extend(ext)
        frontier = nxt
    return nodes


def test_recursive_counts_match_textbook(golden_dir):
    g = golden_counts(golden_dir)
    for n in range(1, 13):
        assert oracle.nqueens_rec(n) == g[n], n


@pytest.mark.parametrize("n", range(1, 8))
def test_recursive_counts_brute_force(n):
    assert oracle.nqueens_rec(n) == brute_force_solutions(n)


@pytest.mark.parametrize("n", range(1, 10))
def test_emulator_stats_match_enumeration(n):
    nodes = partial_placements(n)
    q_tasks = len(nodes)
    qsum_tasks = sum(1 for cols, k in nodes if len(cols) < n and k > 0)
    depth = max(len(c) for c, _ in nodes)
    r = oracle.nqueens(n, records=True)
    assert r.status == 0
    assert r.result == sum(1 for c, _ in nodes if len(c) == n)
    assert r.tasks_by_type == (q_tasks, qsum_tasks)
    assert r.tasks == q_tasks + qsum_tasks
    # the deepest level expands one epoch per row, then joins come back up
    levels_with_joins = len({len(c) for c, k in nodes if len(c) < n and k > 0})
    assert r.epochs == depth + 1 + levels_with_joins
    # nothing is reclaimed before the deepest level has run: peak = all Q tasks
    assert r.peak == q_tasks


def test_emulator_counts_match_textbook(golden_dir):
    g = golden_counts(golden_dir)
    for n in range(1, 12):
        r = oracle.nqueens(n)
        assert r.result == g[n], n


def test_emulator_config_range_stats():
    # n = 6..11 (the batch mix): epochs 2n + 1 since every such n has solutions
    for n in range(6, 12):
        r = oracle.nqueens(n)
        assert r.epochs == 2 * n + 1
        assert r.peak == r.tasks_by_type[0]
