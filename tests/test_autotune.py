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


def test_tuned_file_round_trip(tmp_path):
    """The tuner's tuned file is what the library's AUTO scheduler reads: a
    shape written for (device, workload class) comes back through the C ABI,
    the last line for a pair wins, other pairs and malformed lines do not
    interfere."""
    import paper_1608_00571_amd as T
    path = str(tmp_path / "tuned.txt")
    A.write_tuned("AMD Instinct MI355X", "2+4", A.Shape("graph", 512, 2, 16), path)
    A.write_tuned("AMD Instinct MI355X", "5", A.Shape("persistent", 1024, 1, 8), path)
    with open(path, "a") as f:
        f.write("garbage line\nAMD Instinct MI355X\t2+4\tnot numbers\n")
    assert T.tuned_shape("AMD Instinct MI355X", "2+4", path) == (T.GRAPH, 512, 2, 16)
    assert T.tuned_shape("AMD Instinct MI355X", "5", path) == (T.PERSISTENT, 1024, 1, 8)
    assert T.tuned_shape("AMD Instinct MI355X", "3", path) is None
    assert T.tuned_shape("other device", "2+4", path) is None
    # a later choice for the same pair replaces the earlier one
    A.write_tuned("AMD Instinct MI355X", "2+4", A.Shape("persistent", 256, 0, 8), path)
    assert T.tuned_shape("AMD Instinct MI355X", "2+4", path) == (T.PERSISTENT, 256, 0, 8)
    with open(path) as f:
        assert sum(1 for ln in f if ln.startswith("AMD Instinct MI355X\t2+4\t")) == 1
    # a line with an invalid work-group size is skipped
    with open(path, "a") as f:
        f.write("AMD Instinct MI355X\t5\t1 384 0 8\n")
    assert T.tuned_shape("AMD Instinct MI355X", "5", path) == (T.PERSISTENT, 1024, 1, 8)
    assert T.tuned_shape("nobody", "x", str(tmp_path / "missing.txt")) is None
