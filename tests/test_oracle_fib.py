"""Pins of the oracle's Fibonacci evaluators and of the epoch emulator on the
fib program (Section 6.2's workload; fork/join/emit of Section 4.3.2).

The expected values come from mathematics, not from the oracle: Binet's
closed form, the doubling identities, and the shape of the naive call tree
(counted here by a small dynamic programme over (n, depth))."""
from decimal import Decimal, getcontext
from functools import lru_cache

import numpy as np
import pytest

import oracle


def binet(n: int) -> int:
    getcontext().prec = 80
    s5 = Decimal(5).sqrt()
    phi = (1 + s5) / 2
    psi = (1 - s5) / 2
    return int(((phi ** n - psi ** n) / s5).to_integral_value())


def fib_doubling(n: int) -> int:
    # F(2k) = F(k) (2F(k+1) - F(k)),  F(2k+1) = F(k)^2 + F(k+1)^2
    def fd(k):
        if k == 0:
            return (0, 1)
        a, b = fd(k // 2)
        c = a * (2 * b - a)
        d = a * a + b * b
        return (d, c + d) if k % 2 else (c, d)
    return fd(n)[0]


@pytest.mark.parametrize("n", list(range(0, 60)) + [90])
def test_fib_iter_closed_form(n):
    assert oracle.fib_iter(n) == binet(n) == fib_doubling(n)


def test_fib_known_values():
    assert oracle.fib_iter(20) == 6765
    assert oracle.fib_iter(32) == 2178309


@pytest.mark.parametrize("n", [0, 1, 2, 5, 10, 20, 25])
def test_fib_rec_calls(n):
    v, calls = oracle.fib_rec(n)
    assert v == binet(n)
    # the naive call tree has 2F(n+1) - 1 nodes
    assert calls == 2 * binet(n + 1) - 1


@lru_cache(maxsize=None)
def level_counts(n: int, d: int) -> tuple[int, int]:
    """(nodes, internal nodes) at depth d of the naive call tree of fib(n)."""
    if d == 0:
        return (1, 1 if n >= 2 else 0)
    if n < 2:
        return (0, 0)
    a = level_counts(n - 1, d - 1)
    b = level_counts(n - 2, d - 1)
    return (a[0] + b[0], a[1] + b[1])


def expected_fib_records(n: int):
    """Per-epoch (CEN, launched, valid, forks, joins): the tree expands one
    level per epoch (forks run next epoch), then the joins of each level run
    at that level's epoch number on the way back (Section 4.3.3)."""
    levels = []
    d = 0
    while level_counts(n, d)[0]:
        levels.append(level_counts(n, d))
        d += 1
    recs = []
    for c, (nodes, internal) in enumerate(levels):
        recs.append((c, nodes, nodes, 2 * internal, internal))
    for c in range(len(levels) - 1, -1, -1):
        nodes, internal = levels[c]
        if internal:
            recs.append((c, nodes, internal, 0, 0))
    return recs


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n", list(range(0, 26)))
def test_emulator_fib_result_and_stats(n, width):
    r = oracle.fib(n, width=width, records=True)
    assert r.status == 0
    assert r.result == binet(n)
    if n < 2:
        assert (r.tasks, r.epochs, r.launched, r.peak) == (1, 1, 1, 1)
        return
    C = 2 * binet(n + 1) - 1
    assert r.tasks_by_type == (C, binet(n + 1) - 1)
    assert r.tasks == C + binet(n + 1) - 1
    assert r.epochs == 2 * n - 1
    assert r.peak == C
    assert r.launched == 2 * C - 2
    got = [(int(x["cen"]), int(x["launched"]), int(x["valid"]), int(x["forks"]), int(x["joins"]))
           for x in r.records]
    assert got == expected_fib_records(n)


def test_emulator_fib32_workload():
    r = oracle.fib(32, width=64, records=True)
    assert r.result == 2178309
    assert r.tasks == 10573732 and r.epochs == 63 and r.peak == 7049155
    assert int(r.records["valid"].max()) == 1391720


def test_emulator_fib20_int32_workload():
    r = oracle.fib(20, width=32, records=True)
    assert r.result == 6765 and r.tasks == 32836 and r.epochs == 39
    assert int(r.records["launched"].max()) == 5020


def test_records_sum_to_totals():
    r = oracle.fib(18, records=True)
    assert int(r.records["valid"].sum()) == r.tasks
    assert int(r.records["launched"].sum()) == r.launched
    assert int(r.records["nfc"].max()) == r.peak
    # ranges are contiguous task-vector index intervals (Section 5.1.2)
    assert np.all(r.records["e"] - r.records["b"] == r.records["launched"])


def test_int32_and_int64_agree_below_overflow():
    for n in (2, 11, 24):
        a = oracle.fib(n, width=32)
        b = oracle.fib(n, width=64)
        assert (a.result, a.tasks, a.epochs, a.peak) == (b.result, b.tasks, b.epochs, b.peak)
