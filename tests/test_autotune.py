"""Autotuner logic on the CPU: search, selection of the fastest shape, and
the JSON cache keyed by device and workload class."""
from paper_1608_00571_amd import autotune as A


def test_candidates_respect_residency():
    shapes = A.candidates()
    assert all(s.blocks_per_cu * s.wg <= 2048 for s in shapes)
    assert {s.sched for s in shapes} == {"persistent", "graph"}
    assert {s.wg for s in shapes} == {256, 512, 1024}


def test_tune_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "cache.json")
    cost = {s: 1.0 + 0.01 * i for i, s in enumerate(A.candidates())}
    fastest = A.Shape("graph", 512, 2, 8)
    cost[fastest] = 0.5
    calls = []

    def measure(s):
        calls.append(s)
        return cost[s]

    best, table = A.tune(measure, list(cost), "devX", "batch", cache_path=path)
    assert best == fastest and table[0][1] == 0.5
    n = len(calls)
    # a second call is served from the cache without measuring
    best2, _ = A.tune(measure, list(cost), "devX", "batch", cache_path=path)
    assert best2 == fastest and len(calls) == n
    # another workload class is tuned separately
    A.tune(measure, list(cost)[:3], "devX", "other", cache_path=path)
    assert len(calls) == n + 3
