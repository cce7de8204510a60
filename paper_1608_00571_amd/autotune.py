"""Launch-shape autotuner for the batched schedulers.

Picks, for a workload class, the scheduler (persistent kernel vs. captured
graph chains), the work-group size, the work-groups per CU (wave occupancy)
and the graph chunk length, by timing real runs of a representative batch.
The winner is cached as JSON keyed by device name and workload class, and
recorded in the library's tuned file (one line per device and workload
class: device TAB class TAB "sched wg blocks_per_cu graph_chunk"), which a
context created with the AUTO scheduler follows.
"""
from __future__ import annotations

import itertools
import json
import os
import time
from dataclasses import asdict, dataclass

CACHE = os.environ.get("TREES_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "trees", "autotune.json"))
SCHED_ID = {"plain": 0, "graph": 1, "persistent": 2}


def tuned_file() -> str:
    """Where the library looks for tuned shapes (TREES_TUNE_FILE, else the default)."""
    return os.environ.get("TREES_TUNE_FILE") or os.path.join(os.path.expanduser("~"), ".cache", "trees",
                                                             "tuned.txt")


def write_tuned(device: str, wclass: str, shape, path: str | None = None) -> str:
    """Record `shape` for (device, workload class) in the tuned file, replacing
    an earlier line for the same pair."""
    path = path or tuned_file()
    if "\t" in device or "\t" in wclass or "\n" in device or "\n" in wclass:
        raise ValueError("device and workload class must not hold tabs or newlines")
    keep = []
    try:
        with open(path) as f:
            for ln in f:
                parts = ln.rstrip("\n").split("\t")
                if len(parts) >= 2 and parts[0] == device and parts[1] == wclass:
                    continue
                keep.append(ln if ln.endswith("\n") else ln + "\n")
    except OSError:
        pass
    keep.append(f"{device}\t{wclass}\t{SCHED_ID[shape.sched]} {shape.wg} {shape.blocks_per_cu} "
                f"{shape.graph_chunk}\n")
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.writelines(keep)
    os.replace(tmp, path)
    return path


@dataclass(frozen=True)
class Shape:
    sched: str
    wg: int
    blocks_per_cu: int   # 0 = the library's automatic choice
    graph_chunk: int

    def apply(self, ctx):
        ctx.set_schedule(self.sched, self.wg, self.blocks_per_cu, self.graph_chunk)


def candidates(wgs=(256, 512, 1024), bpcs=(0, 1, 2, 3, 4, 6, 8), chunks=(4, 8, 16)):
    """The search space; shapes that cannot run (too many work-groups per
    CU for the kernel) are clamped by the library, so duplicates are cheap."""
    out = []
    for wg, bpc in itertools.product(wgs, bpcs):
        if bpc * wg > 2048:   # more than 32 wavefronts per CU cannot be resident
            continue
        out.append(Shape("persistent", wg, bpc, 8))
        for ch in chunks:
            out.append(Shape("graph", wg, bpc, ch))
    return out


def _key(device: str, workload: str) -> str:
    return f"{device}|{workload}"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = CACHE):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(measure, shapes, device: str, workload: str, reps: int = 1, cache_path: str | None = CACHE,
         use_cache: bool = True, tuned_path: str | None = None, wclass: str | None = None):
    """measure(shape) -> seconds for one run of the workload under `shape`
    (it must check its results).  Returns (best shape, table of
    (shape, seconds)).  The best is the minimum over `reps` runs each.  With
    `wclass` (a context's workload_class) the winner is also written to the
    tuned file that the library's AUTO scheduler reads."""
    cache = load_cache(cache_path) if cache_path else {}
    k = _key(device, workload)
    if use_cache and k in cache:
        best = Shape(**cache[k]["shape"])
        if wclass is not None:
            write_tuned(device, wclass, best, tuned_path)
        return best, cache[k].get("table", [])
    table = []
    for sh in shapes:
        best = min(measure(sh) for _ in range(reps))
        table.append((sh, best))
    table.sort(key=lambda x: x[1])
    winner = table[0][0]
    if cache_path:
        cache[k] = {"shape": asdict(winner), "seconds": table[0][1], "tuned_at": time.time(),
                    "table": [[asdict(s), t] for s, t in table[:10]]}
        save_cache(cache, cache_path)
    if wclass is not None:
        write_tuned(device, wclass, winner, tuned_path)
    return winner, table
