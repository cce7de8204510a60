"""Pins of the oracle's sorting evaluators and of the emulated merge-sort task
tree (Section 6.4's naive mergesort: split in halves, fork both, join a
merge; runs of at most 64 keys are insertion sorted).

Expected values: numpy's sort (a library routine), multiset equality, and the
task-tree shape counted by recursion on the range length alone."""
from functools import lru_cache

import numpy as np
import pytest

import inputs
import oracle


@lru_cache(maxsize=None)
def shape(n: int):
    """(MS tasks, leaves, MERGE tasks, height) of the split tree of a range of n keys."""
    if n <= 64:
        return (1, 1, 0, 0)
    a = shape(n // 2)
    b = shape(n - n // 2)
    return (1 + a[0] + b[0], a[1] + b[1], 1 + a[2] + b[2], 1 + max(a[3], b[3]))


def merge_levels(n: int, d: int = 0, acc=None):
    """Depths at which merges happen (each depth is one join epoch)."""
    acc = set() if acc is None else acc
    if n > 64:
        acc.add(d)
        merge_levels(n // 2, d + 1, acc)
        merge_levels(n - n // 2, d + 1, acc)
    return acc


SIZES = [0, 1, 2, 63, 64, 65, 127, 128, 129, 1000, 4096, (1 << 16) + 3]


@pytest.mark.parametrize("n", SIZES)
def test_sort_u32_matches_numpy(n):
    k = inputs.keys_u32(n, 11 + n)
    assert np.array_equal(oracle.sort_u32(k), np.sort(k))
    assert np.array_equal(oracle.msort_rec(k), np.sort(k))


@pytest.mark.parametrize("n", SIZES)
def test_emulated_msort(n):
    k = inputs.keys_u32(n, 1000 + n)
    out, r = oracle.msort(k, records=True)
    assert r.status == 0
    assert np.array_equal(out, np.sort(k))
    ms, leaves, merges, h = shape(n)
    assert r.tasks_by_type == (ms, merges)
    assert r.peak == ms
    assert r.epochs == h + 1 + len(merge_levels(n))


def test_duplicates_and_extremes():
    k = np.array([5, 0, 0xFFFFFFFF, 5, 5, 1, 0, 0xFFFFFFFF] * 40, dtype=np.uint32)
    out, _ = oracle.msort(k)
    assert np.array_equal(out, np.sort(k))


def test_workload_shapes():
    # 2^24 keys: 262144 leaves of 64, 37 epochs; 2^22: 33 epochs; 2^10: 9 epochs
    ms, leaves, merges, h = shape(1 << 24)
    assert (ms, leaves, merges, ms + merges, h) == (524287, 262144, 262143, 786430, 18)
    assert shape(1 << 22)[0] + shape(1 << 22)[2] == 196606
    k = inputs.keys_u32(1 << 10, 3)
    out, r = oracle.msort(k)
    assert (r.tasks, r.epochs) == (46, 9)


def test_permutation_property():
    k = inputs.keys_u32(5000, 77) % np.uint32(50)   # many ties
    out, _ = oracle.msort(k)
    assert np.all(out[1:] >= out[:-1])
    assert np.array_equal(np.bincount(out, minlength=50), np.bincount(k, minlength=50))
