#!/usr/bin/env python3
"""Benchmark of the TREES epoch path on one MI355X.

Default workload (one "step"): the two programs of the plain-scheduler
configuration, run back to back through the C ABI --
  * naive fib(32) with 64-bit sums: 10,573,732 tasks in 63 epochs;
  * merge sort of 2^24 uint32 keys drawn uniformly from a seed (split in
    halves, runs of <= 64 keys insertion sorted, merge continuation):
    786,430 tasks in 37 epochs;
under the plain scheduler (one launch per epoch, Phases 1 and 3 on the host).
Inputs are resident in HBM before the timed region; every step sorts its own
fresh copy of the keys.

Prints one JSON line: tasks/s over the whole step (the metric, timed without
per-launch events), epochs/s, the roofline of the dominant kernel and of the
epoch kernel (algorithmic bytes / HIP-event kernel time, against 8 TB/s HBM),
the CPU oracle timed on this host, and the rest of the metric measured in
the same run, each checked against the oracle: the 4096-tree batch (graph
and persistent forms vs one tree at a time under the plain scheduler, with
the batched epoch kernel's task-vector roofline), the 64-graph R-MAT BFS
batch beside the native worklist BFS, and serving latency (p50/p99 at 50%
and 80% of saturation).

    python bench.py [--steps K] [--warmup W] [--config 2|1|3|4|5|6|7|8] [--sched plain|graph|persistent]
                    [--no-blocks] [--no-cpu] [--no-compare]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str):
    """A progress line on stderr (the JSON line is stdout's only output)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)

# HBM bytes per launch of a kernel as rocprofv3 counted them (FETCH_SIZE and
# WRITE_SIZE, each in its own run, scaled by what the same counters read for
# `bench.py --calib-copy`), for the kernel sources with the given digest.  A
# source change makes the figure stale, and it is then reported as null.
MEASURED_TRAFFIC = {   # profiles/plain_fib32_msort2e24.md
    "k_map_merge<1024,8192>": {"src": "a3c1221125ea595c", "fetch_bytes": 68794794, "write_bytes": 67108864},
    "k_plain<FIB>": {"src": "1e02a739f0990e68", "fetch_bytes": 2812957, "write_bytes": 3510431},
    "k_plain<MS>": {"src": "1e02a739f0990e68", "fetch_bytes": 2243668, "write_bytes": 2355210},
    # one persistent run of the 4096-tree batch (profiles/batched_4096trees_fib_nqueens.md)
    "k_epochs<FIB|NQ>": {"src": "1e02a739f0990e68", "wg": 512, "fetch_bytes": 10741529088,
                         "write_bytes": 12627534720},
    # one graph-form run of the 64-graph BFS batch, k_epochs and k_arcs together
    # (profiles/batched_64rmat_bfs.md)
    "k_epochs<GRAPH> bfs": {"src": "1e02a739f0990e68", "wg": 512, "fetch_bytes": 20028926720 + 81312432256,
                            "write_bytes": 464622720 + 2482833728},
    # one persistent run of the FFT batch (64 x 2^18), one k_epochs dispatch
    # (profiles/fft_64x2e18_and_2e20.md)
    "k_epochs<FFT> batch": {"src": "1e02a739f0990e68", "wg": 1024, "fetch_bytes": 1903887872,
                            "write_bytes": 1764621824},
    # one graph-form run of the 64-graph SSSP batch, k_epochs and k_arcs together
    # (profiles/sssp_64rmat_weighted.md)
    "k_epochs<GRAPH> sssp": {"src": "1e02a739f0990e68", "wg": 512, "fetch_bytes": 174533754368 + 140109007232,
                             "write_bytes": 3394525792 + 4234848480},
}


KERNEL_SOURCES = {   # the files a kernel's code comes from
    "k_map": ("map.hip", "map.h", "bodies.h", "prims.h", "trees_dev.h"),
    "k_plain": ("epoch.hip", "map.h", "bodies.h", "prims.h", "trees_dev.h"),
    "k_epochs": ("epoch.hip", "map.h", "bodies.h", "prims.h", "trees_dev.h"),
}


def src_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1608_00571_amd", "csrc")
    fam = next(k for k in KERNEL_SOURCES if kernel.startswith(k))
    for f in KERNEL_SOURCES[fam]:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, alg_bytes_per_launch: int):
    m = MEASURED_TRAFFIC.get(kernel)
    if not m or m["src"] != src_digest(kernel):
        return None
    return m["fetch_bytes"] + m["write_bytes"]


# ---------------------------------------------------------------------------
# Algorithmic bytes (task-vector fields each task type must touch, reads +
# writes, plus payload bytes), per program.
# ---------------------------------------------------------------------------
def fib_counts(n: int):
    F = [0, 1]
    for _ in range(n + 2):
        F.append(F[-1] + F[-2])
    if n < 2:
        return dict(leaves=1, internal=0, sums=0)
    return dict(leaves=F[n + 1], internal=F[n + 1] - 1, sums=F[n + 1] - 1)


def fib_bytes(n: int, launched: int, tasks: int, rbytes: int = 8) -> dict:
    c = fib_counts(n)
    idle = launched - tasks
    # FIB leaf: read code, a0; write r, code.  FIB internal: read code, a0;
    # write 2 children (code, a0) and own (code, a0).  SUM: read code, a0,
    # two child r; write r, code.  Idle lane: read code.
    tv = c["leaves"] * (8 + rbytes + 4) + c["internal"] * 32 + c["sums"] * (8 + 2 * rbytes + rbytes + 4) \
        + idle * 4
    return dict(tv=tv, payload=0)


def msort_counts(N: int):
    """(MS internal, leaves, merged keys over all merges, leaf keys)."""
    memo = {}

    def rec(n):
        if n in memo:
            return memo[n]
        if n <= 64:
            r = (0, 1, 0)
        else:
            a, b = rec(n // 2), rec(n - n // 2)
            r = (1 + a[0] + b[0], a[1] + b[1], n + a[2] + b[2])
        memo[n] = r
        return r

    internal, leaves, merged = rec(N)
    return internal, leaves, merged


def msort_bytes(N: int, launched: int, tasks: int) -> dict:
    internal, leaves, merged = msort_counts(N)
    merges = internal
    idle = launched - tasks
    # MS internal: read code, a0..a2; write 2 children (code, a0..a2), own code.
    # MS leaf / MERGE: read code, a0..a2; write code.  Idle: read code.
    tv = internal * 52 + leaves * 20 + merges * 20 + idle * 4
    payload = 8 * N + 8 * merged   # every key read + written once per leaf sort and per merge level
    return dict(tv=tv, payload=payload)


def nqueens_shape(n: int):
    """(Q tasks, QSUM tasks, task-vector bytes excluding idle lanes) of the
    one-task-per-partial-placement N-queens tree, by enumeration."""
    full = (1 << n) - 1
    q = qs = tv = 0
    stack = [(0, 0, 0, 0)]
    while stack:
        row, cols, ld, rd = stack.pop()
        q += 1
        if row == n:
            tv += 32
            continue
        avail = ~(cols | ld | rd) & full
        k = bin(avail).count("1")
        if k == 0:
            tv += 32
            continue
        # Q internal: read code, a0..a3; write k children (code, a0..a3) and own code, a0, a1
        # QSUM: read code, a0, a1, k child r; write r, code
        tv += 32 + 20 * k + 24 + 8 * k
        qs += 1
        while avail:
            bit = avail & -avail
            avail ^= bit
            stack.append((row + 1, cols | bit, ((ld | bit) << 1) & full, (rd | bit) >> 1))
    return q, qs, tv


# ---------------------------------------------------------------------------
def host_cpu() -> str:
    """The host's CPU model and logical core count (from /proc/cpuinfo)."""
    try:
        names = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")]
        return f"{names[0]} ({len(names)} logical cores)" if names else "unknown"
    except OSError:
        return "unknown"


def cpu_baseline_cfg2(sample_keys_log2: int = 24, min_seconds: float = 10.0):
    """The oracle's epoch emulator on this host's cores: fib(32) and a merge
    sort of 2^k keys (single-threaded C), whole steps repeated until at least
    min_seconds of CPU work (key generation excluded)."""
    import inputs
    import oracle
    keys = inputs.keys_u32(1 << sample_keys_log2, inputs.item_seed(2, 0))
    tasks, dt, steps = 0, 0.0, 0
    while dt < min_seconds:
        t0 = time.perf_counter()
        r = oracle.fib(32)
        _, m = oracle.msort(keys)
        dt += time.perf_counter() - t0
        tasks += r.tasks + m.tasks
        steps += 1
    # the sequential recursive evaluators (the T1 baseline): the same work
    # (fib(32)'s calls, the sort's tasks) without the epoch machinery
    t0 = time.perf_counter()
    _, calls = oracle.fib_rec(32)
    oracle.msort_rec(keys)
    dr = time.perf_counter() - t0
    return {"value": tasks / dt, "unit": "tasks/s", "cores": 1, "kind": "oracle",
            "sample": f"epoch emulator: {steps} whole steps of fib(32) + msort 2^{sample_keys_log2} "
                      f"({dt:.1f} s)",
            "host_cpu": host_cpu(),
            "recursive": {"tasks_per_s": (tasks / steps) / dr, "seconds_per_step": round(dr, 3),
                          "kind": "sequential recursive evaluators (fib by naive recursion, "
                                  "recursive merge sort), one core"}}


def run_cfg2(args, sched, steps, warmup, nomap=False, key_bufs=None, keys_np=None, timed_kinds=()):
    """Time `steps` steps of fib(32) + msort under one scheduler.  Launches
    of the kernel_times() kinds in `timed_kinds` carry HIP events (None:
    every launch)."""
    import numpy as np
    import torch

    import paper_1608_00571_amd as T

    N = 1 << args.log2n
    tmp = torch.empty_like(key_bufs[0])
    arena = (T.tv_bound(T.FIB_I64, [32]) + T.tv_bound(T.MSORT_U32, [N]) + 1024) * T.BYTES_PER_ENTRY
    ctx = T.Context(arena, sched=sched, wg=args.wg, profile=True, nomap=nomap, max_trees=8)
    if timed_kinds is not None:
        ctx.profile_mask(timed_kinds)
    pf = ctx.register(T.FIB_I64)
    pm = ctx.register(T.MSORT_U32)
    base = key_bufs[-1]

    def step(k):
        tf = ctx.submit(pf, [32])
        tm = ctx.submit(pm, [N], [key_bufs[k], tmp])
        rs = ctx.run()
        vf, sf = ctx.results(tf)
        _, sm = ctx.results(tm)
        return vf, sf, sm, rs

    for k in range(warmup):
        key_bufs[k].copy_(base)
        step(k)
    for k in range(steps):
        key_bufs[k].copy_(base)
    kt0 = ctx.kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [step(k) for k in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt1 = ctx.kernel_times()
    ref = np.sort(keys_np)
    for k, (vf, sf, sm, rs) in enumerate(outs):
        assert vf == 2178309 and sf.tasks == 10573732 and sf.epochs == 63, (vf, sf)
        got = key_bufs[k].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref), "sorted keys differ from np.sort"
    ctx.close()
    kt = {k: (kt1[k][0] - kt0[k][0], kt1[k][1] - kt0[k][1]) for k in kt1}
    return dict(dt=dt, outs=outs, kt=kt)


def bench_cfg2(args):
    import numpy as np
    import torch

    import inputs
    import paper_1608_00571_amd as T

    N = 1 << args.log2n
    keys_np = inputs.msort_keys(N)
    nbuf = max(args.steps, args.warmup, 1)
    base = torch.from_numpy(keys_np.view(np.int32)).to("cuda")
    key_bufs = [base.clone() for _ in range(nbuf)] + [base]
    torch.cuda.synchronize()

    # Breakdown: one step with every launch timed (HIP events cost host time
    # per launch, so this step is not the throughput measurement).
    bd = run_cfg2(args, args.sched, 1, args.warmup, key_bufs=key_bufs, keys_np=keys_np, timed_kinds=None)
    kt = bd["kt"]
    _, sf, sm, _ = bd["outs"][-1]
    bf = fib_bytes(32, sf.launched, sf.tasks)
    bm = msort_bytes(N, sm.launched, sm.tasks)
    internal, leaves, merged = msort_counts(N)
    kinds = {"k_plain<FIB>": T.FIB_I64, "k_plain<MS>": T.MSORT_U32,
             "k_map_part<1024,8192>": 6, "k_map_merge<1024,8192>": 7}
    per_step_bytes = {
        "k_plain<FIB>": (bf["tv"], bf["tv"]),
        # the msort epoch kernel: task-vector traffic + leaf sorts (8 B per key)
        "k_plain<MS>": (bm["tv"] + 8 * N, bm["tv"]),
        # the partition pass reads O(log) keys per tile boundary (not counted)
        "k_map_part<1024,8192>": (0, 0),
        # the merge pass reads and writes each key once per merge level
        "k_map_merge<1024,8192>": (8 * merged, 0),
    }
    per = {k: dict(ms=kt[kinds[k]][0], launches=kt[kinds[k]][1], bytes=per_step_bytes[k][0],
                   tv=per_step_bytes[k][1]) for k in kinds}
    # the dominant kernel: the largest share of device time in the breakdown
    # step (every launch timed)
    dom = max(per, key=lambda k: per[k]["ms"])
    epk = "k_plain<FIB>"   # the epoch kernel of the step's largest tree

    # The throughput: steps with no per-launch events (an event pair costs
    # host time per launch, and the plain scheduler's loop is host-driven).
    r = run_cfg2(args, args.sched, args.steps, args.warmup, key_bufs=key_bufs, keys_np=keys_np,
                 timed_kinds=[])
    dt, outs = r["dt"], r["outs"]
    vf, sf, sm, rs = outs[-1]
    tasks = sf.tasks + sm.tasks
    epochs = sf.epochs + sm.epochs
    ms_step = dt * 1e3 / args.steps
    # The roofline: the same steps again, events on the dominant kernel's and
    # the epoch kernel's launches only (HIP events on the launching stream)
    rr = run_cfg2(args, args.sched, args.steps, 0, key_bufs=key_bufs, keys_np=keys_np,
                  timed_kinds=sorted({kinds[dom], kinds[epk]}))
    ktl = rr["kt"]

    def roof_of(k, what):
        d = dict(ms=ktl[kinds[k]][0], launches=ktl[kinds[k]][1], bytes=per[k]["bytes" if what == "all" else "tv"]
                 * args.steps)
        a = d["bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
        return {"bound": "hbm", "achieved": round(a, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(a / HBM_PEAK_GBS, 6),
                "traffic": traffic_for(k, d["launches"] and d["bytes"] // d["launches"]),
                "kernel": k, "launches": d["launches"],
                "avg_launch_us": round(d["ms"] * 1e3 / max(1, d["launches"]), 3),
                "algorithmic_bytes_per_launch": int(d["bytes"] / max(1, d["launches"])),
                "timed_steps": args.steps}
    roof = roof_of(dom, "all")
    roof["dominant_from"] = "largest summed HIP-event kernel time per step over all launches of the step"
    roof["traffic_from"] = "rocprofv3 FETCH_SIZE + WRITE_SIZE per launch (profiles/plain_fib32_msort2e24.md)"
    sp = stream_peak(4 * N)
    roof["achievable"] = {**sp, "frac": round(roof["achieved"] / sp["GBps"], 4)}
    roof_ep = roof_of(epk, "tv")
    roof_ep["what"] = "task-vector bytes of fib(32)'s tasks (D3) over its epoch launches' kernel time"
    kernels = {k: {"ms_per_step": round(v["ms"], 3),
                   "launches_per_step": v["launches"],
                   "GBps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 2) if v["ms"] else None,
                   "tv_GBps": round(v["tv"] / (v["ms"] * 1e-3) / 1e9, 2) if v["ms"] else None}
               for k, v in per.items()}
    line = {
        "metric": "tasks/s", "value": tasks / (dt / args.steps), "unit": "tasks/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64+u32",
        "data": "synthetic",
        "config": {"workload": f"fib(32) int64 + msort 2^{args.log2n} uint32, {args.sched} scheduler",
                   "sched": args.sched, "wg": args.wg, "tasks_per_step": tasks, "epochs_per_step": epochs},
        "epochs_per_s": epochs / (dt / args.steps),
        "kernels": kernels,
        "roofline": roof,
        "roofline_epoch_kernel": roof_ep,
    }
    if args.compare:
        alt = {}
        for sched in ("graph", "persistent"):
            if sched == args.sched:
                continue
            # timed like the line's own steps: no per-launch events
            na = max(1, min(5, len(key_bufs) - 1))
            rr = run_cfg2(args, sched, na, 1, key_bufs=key_bufs, keys_np=keys_np, timed_kinds=[])
            alt[sched] = {"tasks_per_s": tasks / (rr["dt"] / na), "ms_per_step": round(rr["dt"] * 1e3 / na, 3),
                          "steps": na}
        rr = run_cfg2(args, "plain", 1, 0, nomap=True, key_bufs=key_bufs, keys_np=keys_np)
        alt["plain_naive_merge"] = {"tasks_per_s": tasks / rr["dt"], "ms_per_step": round(rr["dt"] * 1e3, 3),
                                    "note": "merges serial in one lane (no map)"}
        line["same_workload"] = alt
    return line


def batch_block(ntrees: int = 4096, wg: int = 512, reps: int = 3, plain_subset: int = 512, tune: bool = False):
    """The batched configuration: `ntrees` independent trees (half fib(10..28),
    half N-queens(6..11), seeded random order) in shared epochs, under the
    graph and persistent forms; the first `plain_subset` of them also one at
    a time under the plain scheduler and batched, for the batched-vs-plain
    factor on the same trees.  Every tree checked against its oracle run.
    The roofline is the batched epoch kernel's: algorithmic task-vector
    bytes of the whole batch over its summed kernel time (HIP events around
    each graph replay or the persistent launch)."""
    import numpy as np
    import torch

    import inputs
    import oracle
    import paper_1608_00571_amd as T

    mix = inputs.batch_mix(ntrees)
    kinds = [(T.FIB_I64 if k == "fib" else T.NQUEENS, n) for k, n in mix]
    expect = {}
    for kind, n in set(kinds):
        r = oracle.fib(n) if kind == T.FIB_I64 else oracle.nqueens(n)
        expect[(kind, n)] = (r.result, r.tasks, r.epochs, r.peak, r.launched)
    nq = {n: nqueens_shape(n) for kind, n in set(kinds) if kind == T.NQUEENS}

    def tv_of(ks):
        tv = 0
        for kind, n in ks:
            res, tasks, epochs, peak, launched = expect[(kind, n)]
            tv += fib_bytes(n, launched, tasks)["tv"] if kind == T.FIB_I64 else nq[n][2] + 4 * (launched - tasks)
        return tv
    tv_bytes = tv_of(kinds)
    total_tasks = sum(expect[k][1] for k in kinds)
    arena = (sum(T.tv_bound(k, [n]) + 64 for k, n in kinds) + 4096) * T.BYTES_PER_ENTRY

    def run_in(ctx, sched, ks, steps, warmup):
        pf, pq = ctx.register(T.FIB_I64), ctx.register(T.NQUEENS)
        times = []
        for it in range(warmup + steps):
            ids = [ctx.submit(pf if k == T.FIB_I64 else pq, [n]) for k, n in ks]
            torch.cuda.synchronize()
            kt0 = ctx.kernel_times()
            t0 = time.perf_counter()
            rs = ctx.run()
            dt = time.perf_counter() - t0
            kt1 = ctx.kernel_times()
            for (k, n), t in zip(ks, ids):
                v, st = ctx.results(t)
                e = expect[(k, n)]
                assert (v, st.tasks, st.epochs, st.peak_entries, st.launched) == e, (k, n, v, st, e)
            if it >= warmup:
                kms = sum(kt1[x][0] - kt0[x][0] for x in kt1)
                et = ctx.epoch_times() if sched != "plain" else None
                times.append((dt, kms, rs, et))
        b = min(times, key=lambda t: t[0])
        return dict(dt=b[0], kernel_ms=min(t[1] for t in times), rs=b[2], et=b[3])

    def run(sched, wg_, bpc=0, chunk=8, steps=1, warmup=1, subset=None, timed=True):
        ks = kinds if subset is None else kinds[:subset]
        ctx = T.Context(arena, sched=sched, wg=wg_, blocks_per_cu=bpc, graph_chunk=chunk, profile=True,
                        max_trees=len(ks))
        if not timed:
            ctx.profile_mask([])
        try:
            return run_in(ctx, sched, ks, steps, warmup)
        finally:
            ctx.close()

    out = {"workload": f"{len(kinds)} trees: fib(10..28) int64 + nqueens(6..11), shared epochs",
           "tasks": total_tasks, "tv_bytes": tv_bytes, "wg": wg}
    tuned = None
    if tune:
        from paper_1608_00571_amd import autotune
        tctx = T.Context(arena, sched="graph", profile=True, max_trees=len(kinds))
        tctx.register(T.FIB_I64)
        tctx.register(T.NQUEENS)

        def measure(shape):
            shape.apply(tctx)
            return run_in(tctx, shape.sched, kinds, 1, 0)["dt"]
        tuned, table = autotune.tune(measure, autotune.candidates(bpcs=(0, 2, 3, 4, 6, 8), chunks=(8, 16)),
                                     torch.cuda.get_device_name(0), f"batch{len(kinds)}", use_cache=False,
                                     wclass=tctx.workload_class)
        tctx.close()
        out["autotune_top5"] = [{**s.__dict__, "ms": round(t * 1e3, 3)} for s, t in table[:5]]
    shapes = [("graph", wg, 0, 8), ("persistent", wg, 0, 8)]
    if tuned is not None:
        shapes.insert(0, (tuned.sched, tuned.wg, tuned.blocks_per_cu, tuned.graph_chunk))
    forms = {}
    for i, (sched, wg_, bpc, ch) in enumerate(shapes):
        # wall time without per-launch events, kernel time from an identical timed run with them
        rw = run(sched, wg_, bpc, ch, steps=reps, warmup=1, timed=False)
        rk = run(sched, wg_, bpc, ch, steps=reps, warmup=0, timed=True)
        name = f"tuned:{sched}/wg{wg_}/bpc{bpc}/chunk{ch}" if (i == 0 and tuned is not None) else sched
        f = {"tasks_per_s": total_tasks / rw["dt"], "ms": round(rw["dt"] * 1e3, 3),
             "kernel_ms": round(rk["kernel_ms"], 3), "global_epochs": rw["rs"].global_epochs,
             "epochs_per_s": rw["rs"].global_epochs / rw["dt"], "grid": rw["rs"].grid,
             "tv_GBps_kernel": round(tv_bytes / (rk["kernel_ms"] * 1e-3) / 1e9, 1)}
        et = rk["et"]
        if et is not None and len(et):
            f["epoch_us"] = {"min": round(float(np.min(et)), 2), "median": round(float(np.median(et)), 2),
                             "max": round(float(np.max(et)), 2),
                             "narrow_epochs_median": round(float(np.median(np.sort(et)[:10])), 2)}
        forms[name] = f
    out["forms"] = forms
    best = max(forms, key=lambda k: forms[k]["tasks_per_s"])
    out["best"] = best
    # the same first `plain_subset` trees: one at a time (plain) and batched
    sub = min(plain_subset, len(kinds))
    sub_tasks = sum(expect[k][1] for k in kinds[:sub])
    rp = run("plain", 1024, steps=1, warmup=0, subset=sub, timed=False)
    bsched = forms[best]
    rb = run(best.split(":")[-1].split("/")[0], wg, steps=reps, warmup=1, subset=sub, timed=False)
    out["same_trees"] = {"trees": sub, "tasks": sub_tasks,
                         "plain_one_at_a_time": {"tasks_per_s": sub_tasks / rp["dt"], "ms": round(rp["dt"] * 1e3, 2),
                                                 "wg": 1024},
                         "batched": {"tasks_per_s": sub_tasks / rb["dt"], "ms": round(rb["dt"] * 1e3, 3)}}
    out["batched_vs_plain_factor"] = round(rp["dt"] / rb["dt"], 2)
    ach = tv_bytes / (bsched["kernel_ms"] * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": f"k_epochs<FIB|NQ> ({best}, wg {wg})",
                       "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_run": tv_bytes,
                       "traffic": traffic_for("k_epochs<FIB|NQ>", tv_bytes),
                       "what": "task-vector bytes each task must move (D3) over the summed kernel time"}
    out["checked"] = "every tree's result, tasks, epochs, peak and lanes against its oracle run"
    return out


def bench_cfg3(args):
    """The batched configuration as its own line (see batch_block)."""
    blk = batch_block(args.trees, args.wg if args.wg != 256 else 512, max(1, args.steps), args.plain_subset,
                      args.tune)
    b = blk["forms"][blk["best"]]
    return {"metric": "tasks/s", "value": b["tasks_per_s"], "unit": "tasks/s", "n_gpus": 1,
            "steps": max(1, args.steps), "warmup": 1, "ms_per_step": b["ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64+int32",
            "data": "synthetic",
            "config": {"workload": blk["workload"], "sched": blk["best"], "wg": blk["wg"]},
            "epochs_per_s": b["epochs_per_s"], "batch": blk, "roofline": blk["roofline"]}


def bench_cfg1(args):
    """fib(20) with 32-bit sums under the plain scheduler: 32,836 tasks in 39
    epochs, so the per-epoch launch + readback overhead dominates."""
    import torch

    import paper_1608_00571_amd as T

    ctx = T.Context(T.tv_bound(T.FIB_I32, [20]) * T.BYTES_PER_ENTRY + 4096, sched="plain", wg=args.wg,
                    profile=True, max_trees=4)
    p = ctx.register(T.FIB_I32)
    for _ in range(args.warmup):
        t = ctx.submit(p, [20]); ctx.run(); ctx.results(t)
    # timed steps carry no per-launch events (they cost host time per launch)
    ctx.profile_mask([])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t = ctx.submit(p, [20]); ctx.run(); v, st = ctx.results(t)
        assert v == 6765 and st.tasks == 32836 and st.epochs == 39
    dt = (time.perf_counter() - t0) / args.steps
    # then the same steps with every epoch launch timed, for the kernel share
    ctx.profile_mask([T.FIB_I32])
    kt0 = ctx.kernel_times()
    for _ in range(args.steps):
        t = ctx.submit(p, [20]); ctx.run(); ctx.results(t)
    kt1 = ctx.kernel_times()
    kms = (kt1[T.FIB_I32][0] - kt0[T.FIB_I32][0]) / args.steps
    ctx.close()
    return {"metric": "tasks/s", "value": 32836 / dt, "unit": "tasks/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": "fib(20) int32, plain scheduler", "sched": "plain", "wg": args.wg},
            "epochs_per_s": 39 / dt, "us_per_epoch": round(dt * 1e6 / 39, 2),
            "kernel_us_per_epoch": round(kms * 1e3 / 39, 2),
            "launch_readback_us_per_epoch": round(dt * 1e6 / 39 - kms * 1e3 / 39, 2)}


def bfs_graphs(ngraphs: int = 64, workers: int = 16):
    """The BFS batch's R-MAT graphs (scale 16..22, E = 16 V) on the host and
    the device, and the oracle's queue-BFS depths of each (both generated in
    parallel threads: the C routines release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import inputs
    import oracle
    scales = inputs.bfs_batch_scales(ngraphs)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:
        gs = list(ex.map(lambda a: inputs.bfs_batch_graph(*a), list(enumerate(scales))))
    gen_s = time.perf_counter() - t0
    dev = [(torch.from_numpy(G.row_ptr).to("cuda"), torch.from_numpy(G.col_idx).to("cuda"),
            torch.empty(G.V, dtype=torch.int32, device="cuda")) for G in gs]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:
        want = list(ex.map(lambda G: oracle.bfs_queue(G.V, G.row_ptr, G.col_idx, G.source), gs))
    orc_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    return gs, dev, want, {"generate": round(gen_s, 1), "oracle_bfs": round(orc_s, 1)}


def bfs_block(ngraphs: int = 64, wg: int = 512, reps: int = 3, scheds=("graph", "persistent", "plain"),
              worklist: bool = True, graphs=None):
    """The batched graph configuration: 64 BFS trees (one per R-MAT graph,
    scale 16..22) in shared epochs, and, as the paper's comparison (Section
    6.3), the native worklist BFS on each graph one after another, beside
    TREES' plain scheduler on each graph one after another.  Depths checked
    against the oracle's queue BFS in every run."""
    import numpy as np
    import torch

    import paper_1608_00571_amd as T

    gs, dev, want, setup = graphs if graphs is not None else bfs_graphs(ngraphs)
    V = sum(G.V for G in gs)
    E = sum(G.E for G in gs)
    scanned = sum(int(np.diff(G.row_ptr)[w >= 0].sum()) for G, w in zip(gs, want))
    reached = sum(int((w >= 0).sum()) for w in want)
    # algorithmic bytes of the batch: per reached vertex its VISIT entry (code,
    # a0 read; code written) and the child entry that created it; its row_ptr
    # pair; per arc of a reached vertex the head and its depth probe; per claim
    # the depth written
    tv = 12 * reached + 8 * reached
    payload = 8 * reached + 8 * scanned + 4 * reached
    arena = (V + 64 * len(gs) + 4096) * T.BYTES_PER_ENTRY

    def check(stats):
        for (G, b, w, st) in zip(gs, dev, want, stats):
            assert np.array_equal(b[2].cpu().numpy(), w), "BFS depths differ from the queue BFS"
            assert st.tasks == int((w >= 0).sum()) and st.epochs == int(w.max()) + 1

    out = {"workload": f"{len(gs)} R-MAT BFS trees, scale 16..22, E=16V (0.57,0.19,0.19,0.05)",
           "V": V, "E": E, "reached": reached, "arcs_scanned": scanned, "wg": wg, "setup_s": setup}
    forms = {}
    for sched in scheds:
        ctx = T.Context(arena, sched=sched, wg=wg if sched != "plain" else wg, profile=True, max_trees=len(gs))
        ctx.profile_mask([])
        p = ctx.register(T.BFS_CSR)
        best = None
        per_graph = None
        n_it = 1 + (reps if sched != "plain" else 1)
        for it in range(n_it):
            if sched == "plain":   # one graph at a time: a run per graph
                times = []
                stats = []
                for G, b in zip(gs, dev):
                    t = ctx.submit(p, [G.V, G.source], list(b))
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    ctx.run()
                    times.append(time.perf_counter() - t1)
                    stats.append(ctx.results(t)[1])
                dt = sum(times)
                rs = None
            else:
                ids = [ctx.submit(p, [G.V, G.source], list(b)) for G, b in zip(gs, dev)]
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                rs = ctx.run()
                dt = time.perf_counter() - t1
                stats = [ctx.results(t)[1] for t in ids]
                times = None
            check(stats)
            if it >= 1 or sched == "plain":
                if best is None or dt < best[0]:
                    best = (dt, rs, ctx.epoch_times() if sched != "plain" else None)
                    per_graph = times
        ctx.close()
        dt, rs, et = best
        forms[sched] = {"vertices_per_s": reached / dt, "edges_per_s": scanned / dt, "ms": round(dt * 1e3, 3)}
        if rs is not None:
            forms[sched]["global_epochs"] = rs.global_epochs
            forms[sched]["epochs_per_s"] = rs.global_epochs / dt
        if et is not None and len(et):
            forms[sched]["epoch_us"] = [round(float(x), 1) for x in et]
        if per_graph is not None:
            forms[sched]["per_graph_ms"] = [round(x * 1e3, 3) for x in per_graph]
    out["forms"] = forms
    best = max((k for k in forms if k != "plain"), key=lambda k: forms[k]["vertices_per_s"])
    out["best"] = best
    if worklist:   # the native worklist BFS, one graph after another
        ctx = T.Context(1 << 20, sched="plain", wg=wg)
        ws = torch.empty(T.wl_workspace_bytes(max(G.V for G in gs)), dtype=torch.uint8, device="cuda")
        wl_best = None
        for it in range(2):
            times, iters = [], 0
            for G, b, w in zip(gs, dev, want):
                st = ctx.wl_bfs(G.V, G.source, b[0], b[1], b[2], ws)
                assert np.array_equal(b[2].cpu().numpy(), w), "worklist BFS depths differ from the queue BFS"
                assert st.iterations == int(w.max()) + 1
                times.append(st.seconds)
                iters += st.iterations
            if wl_best is None or sum(times) < sum(wl_best[0]):
                wl_best = (times, iters)
        ctx.close()
        wt = sum(wl_best[0])
        out["worklist"] = {"ms": round(wt * 1e3, 3), "vertices_per_s": reached / wt, "iterations": wl_best[1],
                           "per_graph_ms": [round(x * 1e3, 3) for x in wl_best[0]],
                           "trees_plain_over_worklist": round(forms["plain"]["ms"] / (wt * 1e3), 4)
                           if "plain" in forms else None,
                           "trees_batched_over_worklist": round(forms[best]["ms"] / (wt * 1e3), 4),
                           "note": "times are host wall per graph (launches, per-iteration count readback); "
                                   "the paper reports TREES within 6% of LonestarGPU's bfs on its APU"}
    b = forms[best]
    ach = (tv + payload) / (b["ms"] * 1e-3) / 1e9
    lines = (tv + payload + 60 * scanned) / (b["ms"] * 1e-3) / 1e9   # a depth probe moves a 64-B sector
    m = MEASURED_TRAFFIC["k_epochs<GRAPH> bfs"]
    traffic = traffic_for("k_epochs<GRAPH> bfs", 0) if (best == "graph" and wg == m["wg"]) else None
    out["roofline"] = {"bound": "hbm", "kernel": f"k_epochs<GRAPH> + k_arcs ({best}, wg {wg})",
                       "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "tv_bytes": tv, "payload_bytes": payload,
                       "traffic": traffic,
                       "traffic_from": "rocprofv3 FETCH_SIZE + WRITE_SIZE of k_epochs and k_arcs per graph-form "
                                       "run, work-groups of 512 (profiles/batched_64rmat_bfs.md)",
                       "what": "algorithmic bytes (task-vector + graph payload) over the run's wall time",
                       "waste": {"note": "random 4-B depth probes move whole 64-B sectors",
                                 "line_traffic_GBps": round(lines, 1),
                                 "traffic_over_algorithmic": round(traffic / (tv + payload), 2) if traffic else None}}
    out["checked"] = "every depth against the oracle's queue BFS; tasks = reached, epochs = max depth + 1"
    return out


def bench_cfg4(args):
    """The batched graph configuration as its own line (see bfs_block)."""
    blk = bfs_block(args.graphs, args.wg, max(1, args.steps), tuple(args.scheds.split(",")))
    b = blk["forms"][blk["best"]]
    return {"metric": "tasks/s", "value": b["vertices_per_s"], "unit": "tasks/s (vertices visited)",
            "n_gpus": 1, "steps": max(1, args.steps), "warmup": 1, "ms_per_step": b["ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic", "config": {"workload": blk["workload"], "sched": blk["best"], "wg": blk["wg"]},
            "edges_per_s": b["edges_per_s"], "epochs_per_s": b.get("epochs_per_s"), "bfs": blk,
            "roofline": blk["roofline"]}


def bench_cfg7(args):
    """Single-source shortest paths (the relaxation program) on the BFS
    batch's 64 R-MAT graphs with arc weights uniform on [1, 100], one tree
    each, in shared epochs; distances checked against Dijkstra."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import inputs
    import oracle
    import paper_1608_00571_amd as T

    scales = inputs.bfs_batch_scales(args.graphs)
    t0 = time.perf_counter()
    gs, dev = [], []
    for g, sc in enumerate(scales):
        G, w = inputs.sssp_batch_graph(g, sc)
        rp = torch.from_numpy(G.row_ptr).to("cuda")
        ci = torch.from_numpy(G.col_idx).to("cuda")
        wt = torch.from_numpy(w).to("cuda")
        d = torch.empty(G.V, dtype=torch.int32, device="cuda")
        gs.append((G, w))
        dev.append((rp, ci, wt, d))
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(8) as ex:   # (the oracle's C call releases the GIL)
        want = list(ex.map(lambda gw: oracle.dijkstra(gw[0].V, gw[0].row_ptr, gw[0].col_idx, gw[1],
                                                      gw[0].source), gs))
    orc_s = time.perf_counter() - t0
    V = sum(G.V for G, _ in gs)
    E = sum(G.E for G, _ in gs)
    reached = sum(int((w != oracle.UNREACHED).sum()) for w in want)
    # a work-efficient schedule visits each reached vertex once: its arcs are
    # read (head, weight, head's distance) once; the bytes per visit are the
    # entry read, the entry that created it, the row_ptr pair and the distance
    scanned = sum(int(np.diff(G.row_ptr)[w != oracle.UNREACHED].sum()) for (G, _), w in zip(gs, want))
    cap = sum(T.tv_bound(T.SSSP_CSR, [G.V, G.source]) + 64 for G, _ in gs)
    arena = (cap + 4096) * T.BYTES_PER_ENTRY
    out = {}
    runs = [(sched, 0) for sched in args.scheds.split(",")]
    runs += [("graph", dl) for dl in args.sssp_deltas]   # bucket widths, beside the plain program
    for sched, delta in runs:
        ctx = T.Context(arena if not delta else 2 * arena, sched=sched, wg=args.wg, profile=True,
                        max_trees=len(gs))
        p = ctx.register(T.SSSP_CSR)
        best = None
        for it in range(args.warmup + args.steps):
            sargs = lambda G: [G.V, G.source] + ([16 * G.V, delta] if delta else [])
            ids = [ctx.submit(p, sargs(G), list(b)) for (G, _), b in zip(gs, dev)]
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rs = ctx.run()
            dt = time.perf_counter() - t1
            stats = [ctx.results(t)[1] for t in ids]
            for b, w in zip(dev, want):
                assert np.array_equal(b[3].cpu().numpy(), w), "SSSP distances differ from Dijkstra"
            tasks = sum(st.tasks for st in stats)
            if it >= args.warmup and (best is None or dt < best[0]):
                best = (dt, rs, tasks, ctx.epoch_times() if sched != "plain" else None)
        ctx.close()
        dt, rs, tasks, et = best
        tv = 20 * tasks
        payload = 12 * tasks + 12 * scanned + 4 * tasks
        out[sched if not delta else f"graph_delta{delta}"] = {
                      "tasks_per_s": tasks / dt, "reached_per_s": reached / dt, "ms": round(dt * 1e3, 3),
                      "tasks": tasks, "visits_per_reached": round(tasks / reached, 3),
                      "global_epochs": rs.global_epochs, "alg_bytes": tv + payload}
        if et is not None and len(et):
            out[sched if not delta else f"graph_delta{delta}"]["epoch_us"] = [round(float(x), 1) for x in et]
    # the line's value: the plain relaxation program (the paper's); the
    # bucketed runs are reported beside it
    best = min((k for k in out if "delta" not in k), key=lambda k: out[k]["ms"])
    bucketed = min((k for k in out if "delta" in k), key=lambda k: out[k]["ms"], default=None)
    b = out[best]
    ach = b["alg_bytes"] / (b["ms"] * 1e-3) / 1e9
    # random probes of a head's distance move a 64-B sector, not 4 B
    amp = (b["alg_bytes"] + 60 * scanned) / (b["ms"] * 1e-3) / 1e9
    m = MEASURED_TRAFFIC["k_epochs<GRAPH> sssp"]
    traffic = traffic_for("k_epochs<GRAPH> sssp", 0) if (best == "graph" and args.wg == m["wg"]) else None
    return {"metric": "tasks/s", "value": b["tasks_per_s"], "unit": "tasks/s (vertex visits)",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic",
            "config": {"workload": f"{len(gs)} weighted R-MAT SSSP trees, scale 16..22, E=16V, w in [1,100]",
                       "sched": best, "V": V, "E": E, "reached": reached, "arcs_of_reached": scanned},
            "reached_vertices_per_s": b["reached_per_s"],
            "schedulers": out,
            "bucketed": None if bucketed is None else {
                "best": bucketed, "ms": out[bucketed]["ms"],
                "speedup_vs_plain_program": round(b["ms"] / out[bucketed]["ms"], 2)},
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                         "note": "bytes of the visits made, with each reached vertex's arcs read once",
                         "sector_amplified": {"achieved": round(amp, 1), "frac": round(amp / HBM_PEAK_GBS, 4)},
                         "traffic_GBps": round(traffic / (b["ms"] * 1e-3) / 1e9, 1) if traffic else None,
                         "traffic_from": "rocprofv3 FETCH_SIZE + WRITE_SIZE of k_epochs and k_arcs per "
                                         "graph-form run, work-groups of 512 (profiles/sssp_64rmat_weighted.md)"},
            "setup_s": {"generate": round(gen_s, 1), "oracle_dijkstra": round(orc_s, 1)}}


def fft_bytes(m: int) -> int:
    """Algorithmic payload bytes of one FFT of 2^m complex fp32 points: the
    leaves read x and write y (8 + 8 B a point), and every combine level reads
    and writes y once more (16 B a point)."""
    n = 1 << m
    return 16 * n * (1 + max(0, m - 6))


def bench_cfg8(args):
    """The FFT program (a widening beyond the five configurations): one
    transform of 2^20 complex fp32 points under every scheduler, and a batch
    of 64 transforms of 2^18 points in shared epochs (plain: one after
    another).  Every output is checked against numpy's fp64 FFT within the
    fp32 error bound of a radix-2 FFT."""
    import numpy as np
    import torch

    import inputs
    import paper_1608_00571_amd as T

    def tol(m):
        u = 2.0 ** -24
        eta = 4 * u + (4 * u / (1 - 4 * u)) * (np.sqrt(2) + 4 * u)
        t = max(1, m) * eta
        return t / (1 - t)

    def make(m, count, seed):
        xs, ys, want = [], [], []
        for g in range(count):
            x = inputs.complex_signal(1 << m, seed + g)
            xs.append(torch.from_numpy(x.view(np.float32).copy()).to("cuda"))
            ys.append(torch.empty_like(xs[-1]))
            want.append(np.fft.fft(x.astype(np.complex128)) if g < 4 else None)
        return xs, ys, want

    def run(sched, m, xs, ys, want, wg):
        arena = (len(xs) * (T.tv_bound(T.FFT, [m]) + 64) + 4096) * T.BYTES_PER_ENTRY
        ctx = T.Context(arena, sched=sched, wg=wg, max_trees=len(xs))
        p = ctx.register(T.FFT)
        best, st = None, None
        for it in range(args.warmup + args.steps):
            ids = [ctx.submit(p, [m], [x, y]) for x, y in zip(xs, ys)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rs = ctx.run()
            dt = time.perf_counter() - t0
            st = [ctx.results(t)[1] for t in ids]
            for y, w in zip(ys, want):
                if w is not None:
                    got = y.cpu().numpy().view(np.complex64).astype(np.complex128)
                    err = np.linalg.norm(got - w) / np.linalg.norm(w)
                    assert err <= tol(m), f"fft {sched}: relative error {err:.2e}"
            if it >= args.warmup and (best is None or dt < best[0]):
                best = (dt, rs, ctx.epoch_times() if sched != "plain" else None)
        ctx.close()
        dt, rs, et = best
        tasks = sum(s.tasks for s in st)
        pts = len(xs) << m
        out = {"ms": round(dt * 1e3, 3), "tasks_per_s": tasks / dt, "tasks": tasks,
               "gflops": 5.0 * pts * m / dt / 1e9, "GBps": len(xs) * fft_bytes(m) / dt / 1e9,
               "global_epochs": rs.global_epochs}
        if et is not None and len(et):
            out["epoch_us"] = [round(float(x), 1) for x in et]
        return out

    one = make(20, 1, 800)
    single = {s: run(s, 20, *one, 1024 if s == "plain" else args.wg) for s in ("plain", "graph", "persistent")}
    bm, bn = 18, 64
    batch_in = make(bm, bn, 900)
    batch = {s: run(s, bm, *batch_in, args.wg) for s in ("graph", "persistent")}
    batch["plain_one_at_a_time"] = run("plain", bm, batch_in[0][:16], batch_in[1][:16], batch_in[2][:16], 1024)
    bbest = max(("graph", "persistent"), key=lambda k: batch[k]["tasks_per_s"])
    sbest = min(single, key=lambda k: single[k]["ms"])
    b = batch[bbest]
    ach = bn * fft_bytes(bm) / (b["ms"] * 1e-3) / 1e9
    m = MEASURED_TRAFFIC["k_epochs<FFT> batch"]
    traffic = traffic_for("k_epochs<FFT> batch", 0) if (bbest == "persistent" and args.wg == m["wg"]) else None
    return {
        "metric": "tasks/s", "value": b["tasks_per_s"], "unit": "tasks/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64 (fp32)",
        "data": "synthetic",
        "config": {"workload": f"{bn} FFTs of 2^{bm} complex fp32 points in shared epochs; "
                               "one FFT of 2^20 points beside it",
                   "sched": bbest, "wg": args.wg, "tasks": b["tasks"]},
        "gflops": b["gflops"],
        "batch": batch,
        "batched_vs_plain_factor": round(b["tasks_per_s"] / batch["plain_one_at_a_time"]["tasks_per_s"], 2),
        "single_2e20": {"best": sbest, **{k: v for k, v in single.items()}},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_from": "rocprofv3 FETCH_SIZE + WRITE_SIZE of the persistent batch's k_epochs "
                                     "dispatch, work-groups of 1024 (profiles/fft_64x2e18_and_2e20.md)",
                     "algorithmic_bytes_per_run": bn * fft_bytes(bm)},
    }


def serving_setup(n_warm: int, n: int, seed: int = 0, workers: int = 16):
    """The serving configuration's requests (one Poisson trace of n_warm + n
    requests, arrival times at rate 1, rescaled per run) with their payloads
    on the device: msort keys (a pristine copy, re-copied into the working
    buffer before every run, since the sort is in place) and, for every BFS
    request, its own seeded R-MAT graph.  Host payloads are generated in
    parallel (the C generators release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import inputs
    reqs = inputs.serving_trace(n_warm + n, 1.0, seed)
    with ThreadPoolExecutor(workers) as ex:
        host = list(ex.map(inputs.request_payload, reqs))
    dev = []
    for r, p in zip(reqs, host):
        if r.kind == "msort":
            k = torch.from_numpy(np.ascontiguousarray(p).view(np.int32)).to("cuda")
            dev.append((k, torch.empty_like(k), torch.empty_like(k)))   # pristine, working, merge buffer
        elif r.kind == "bfs":
            ci = torch.from_numpy(p.col_idx).to("cuda")
            if ci.numel() == 0:
                ci = torch.zeros(1, dtype=torch.int32, device="cuda")
            dev.append((torch.from_numpy(p.row_ptr).to("cuda"), ci,
                        torch.empty(p.V, dtype=torch.int32, device="cuda")))
        else:
            dev.append(())
    torch.cuda.synchronize()
    return reqs, host, dev


def serving_jobs(reqs, host, dev, lo: int, hi: int, rate: float | None):
    """Jobs for requests [lo, hi) of the trace; arrivals at `rate` per second
    (None: all at once), measured from the first of them."""
    from paper_1608_00571_amd.serving import Job
    t0 = reqs[lo].t_arrive
    jobs = []
    for r, p, d in zip(reqs[lo:hi], host[lo:hi], dev[lo:hi]):
        t = 0.0 if rate is None else (r.t_arrive - t0) / rate
        if r.kind == "fib":
            jobs.append(Job(r.rid, t, "fib", [r.size]))
        elif r.kind == "msort":
            d[1].copy_(d[0])
            jobs.append(Job(r.rid, t, "msort", [r.size], p, dev=(d[1], d[2]), bytes_payload=8 * r.size))
        else:
            jobs.append(Job(r.rid, t, "bfs", [p.V, p.source], p, dev=d,
                            bytes_payload=4 * (p.V + 1) + 4 * p.E + 4 * p.V))
    return jobs


class ServingCheck:
    """Every served result against the oracle's run of that request alone:
    fib value and statistics, msort output, BFS depths (each request's own
    graph; the queue BFS of a graph is computed once)."""

    def __init__(self):
        self.fib, self.bfs = {}, {}

    def __call__(self, jobs):
        import numpy as np

        import oracle
        tasks = 0
        for j in jobs:
            if j.kind == "fib":
                n = j.args[0]
                if n not in self.fib:
                    self.fib[n] = oracle.fib(n)
                r = self.fib[n]
                assert (j.value, j.stats.tasks, j.stats.epochs, j.stats.peak_entries) == \
                    (r.result, r.tasks, r.epochs, r.peak), f"fib request {j.rid}"
            elif j.kind == "msort":
                assert np.array_equal(j.out, np.sort(j.host_payload)), f"msort request {j.rid}"
            else:
                g = j.host_payload
                if j.rid not in self.bfs:
                    self.bfs[j.rid] = oracle.bfs_queue(g.V, g.row_ptr, g.col_idx, g.source)
                assert np.array_equal(j.out, self.bfs[j.rid]), f"bfs request {j.rid}"
            tasks += j.stats.tasks
        return tasks


def serving_block(n: int = 600, n_warm: int = 60, arena_gib: int = 16, wg: int = 1024, loads=(0.5, 0.8),
                  modes=("async", "bursts"), burst: int = 4):
    """The serving configuration: Poisson arrivals of the 40/40/20 fib /
    msort / BFS mix (fib(12..30), msort of 2^10..2^22 keys, R-MAT BFS of
    scale 12..20, each BFS request on its own graph).  Saturation from a
    closed batch, then p50/p99 latency at 50% and 80% of it, in the
    asynchronous mode (submissions into the running persistent kernel) and,
    for comparison, the burst mode; every result checked against the
    oracle."""
    from paper_1608_00571_amd.serving import Server
    t0 = time.perf_counter()
    reqs, host, dev = serving_setup(n_warm, n)
    setup_s = time.perf_counter() - t0
    check = ServingCheck()
    out = {"requests": n, "warmup_requests": n_warm,
           "mix": "40% fib(12..30) int64, 40% msort 2^10..2^22 uint32 (log-uniform), 20% R-MAT BFS "
                  "scale 12..20 (one graph per request)",
           "budget_gib": {"arena": arena_gib, "payload": arena_gib}}
    for mode in modes:
        srv = Server(arena_gib << 30, mode=mode, sched="graph", burst=burst, wg=wg,
                     payload_budget=arena_gib << 30)
        try:
            srv.serve(serving_jobs(reqs, host, dev, 0, n_warm, None), realtime=False)
            sat = srv.serve(serving_jobs(reqs, host, dev, n_warm, n_warm + n, None), realtime=False)
            sat_tasks = check(sat.jobs)
            sat_rate = n / sat.seconds
            m = {"saturation": {"requests_per_s": round(sat_rate, 1), "tasks_per_s": sat_tasks / sat.seconds,
                                "seconds": round(sat.seconds, 4), "max_inflight": sat.max_inflight,
                                "epochs": sat.epochs}}
            for load in loads:
                r = srv.serve(serving_jobs(reqs, host, dev, n_warm, n_warm + n, load * sat_rate), realtime=True)
                tasks = check(r.jobs)
                m[f"load_{int(load * 100)}"] = {
                    "offered_rps": round(load * sat_rate, 1), "requests_per_s": round(n / r.seconds, 1),
                    "tasks_per_s": tasks / r.seconds, "p50_ms": round(r.pct(50) * 1e3, 3),
                    "p99_ms": round(r.pct(99) * 1e3, 3), "max_inflight": r.max_inflight, "epochs": r.epochs}
        finally:
            srv.close()
        out[mode] = m
    out["checked"] = "every result against the oracle's run of the request alone"
    out["setup_s"] = round(setup_s, 1)
    return out


def bench_cfg5(args):
    """Serving, as its own line: the serving block, value = tasks/s at 80%
    of saturation in the asynchronous mode."""
    blk = serving_block(args.requests, args.serve_warmup, args.serve_arena_gib, args.wg, burst=args.burst)
    l80 = blk["async"]["load_80"]
    return {"metric": "tasks/s", "value": l80["tasks_per_s"], "unit": "tasks/s", "n_gpus": 1,
            "steps": 1, "warmup": args.serve_warmup, "ms_per_step": round(args.requests / l80["requests_per_s"] * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64+u32+int32",
            "data": "synthetic",
            "config": {"workload": f"serving {args.requests} requests: 40% fib(12..30), 40% msort 2^10..2^22, "
                                   "20% R-MAT BFS 12..20 (own graph each), asynchronous persistent run",
                       "arena_gib": args.serve_arena_gib},
            "p50_ms": l80["p50_ms"], "p99_ms": l80["p99_ms"], "serving": blk}


def run_traversal(args, prog_kind, n, left, right, lt, rt, log):
    """One traversal program over the bench tree under every scheduler; each
    run's visit log is checked (every node once; postorder: after its
    children; preorder: after its parent)."""
    import numpy as np
    import torch

    import paper_1608_00571_amd as T

    arena = (T.tv_bound(prog_kind, [n, 0]) + 64) * T.BYTES_PER_ENTRY
    pos = np.empty(n, dtype=np.int64)
    out = {}
    st = None
    for sched in ("graph", "persistent", "plain"):
        ctx = T.Context(arena, sched=sched, wg=args.wg, max_trees=2)
        prog = ctx.register(prog_kind)
        times = []
        for it in range(args.warmup + args.steps):
            t = ctx.submit(prog, [n, 0], [lt, rt, log])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.run()
            dt = time.perf_counter() - t0
            _, st = ctx.results(t)
            if it >= args.warmup:
                times.append(dt)
        ctx.close()
        lg = log.cpu().numpy()
        assert lg[n] == n, f"traversal {sched}: {lg[n]} visits of {n} nodes"
        pos[lg[:n]] = np.arange(n)
        for arr in (left, right):
            has = arr >= 0
            if prog_kind == T.POSTORDER:
                assert np.all(pos[arr[has]] < pos[has]), f"postorder {sched}: a node visited before its child"
            else:
                assert np.all(pos[arr[has]] > pos[has]), f"preorder {sched}: a node visited before its parent"
        dt = sum(times) / len(times)
        out[sched] = {"tasks_per_s": st.tasks / dt, "ms": round(dt * 1e3, 3), "epochs_per_s": st.epochs / dt}
    best = max(("graph", "persistent"), key=lambda k: out[k]["tasks_per_s"])
    return out, best, st


def bench_cfg6(args):
    """Figure 2's postorder program over a random binary tree of 2^log2tree
    nodes (a widening beyond the five configurations), with the same tree's
    preorder program beside it: every scheduler; each run's visit log is
    checked against the tree."""
    import torch

    import inputs
    import paper_1608_00571_amd as T

    n = 1 << args.log2tree
    left, right = inputs.postorder_tree(n)
    lt, rt = torch.from_numpy(left).to("cuda"), torch.from_numpy(right).to("cuda")
    log = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    out, best, st = run_traversal(args, T.POSTORDER, n, left, right, lt, rt, log)
    pre, pbest, pst = run_traversal(args, T.PREORDER, n, left, right, lt, rt, log)
    return {
        "metric": "tasks/s", "value": out[best]["tasks_per_s"], "unit": "tasks/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": out[best]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"postorder (Figure 2) of a random binary tree with 2^{args.log2tree} nodes",
                   "sched": best, "wg": args.wg, "tasks": st.tasks, "epochs": st.epochs},
        "epochs_per_s": out[best]["epochs_per_s"],
        "schedulers": out,
        "batched_vs_plain_factor": round(out[best]["tasks_per_s"] / out["plain"]["tasks_per_s"], 2),
        "preorder": {"tasks": pst.tasks, "epochs": pst.epochs, "sched": pbest, "schedulers": pre},
    }


def stream_peak(bytes_each_way: int) -> dict:
    """Achievable streaming bandwidth on this GPU: an int32 elementwise kernel
    that reads and writes `bytes_each_way` bytes per launch (capped at 1 GiB),
    timed with events over 20 launches.  The roofline reports its kernel's
    rate against this beside the data-sheet peak."""
    import torch
    n = max(1, min(bytes_each_way, 1 << 30) // 4)
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.bitwise_not(src, out=dst)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(20):
        torch.bitwise_not(src, out=dst)
    ev[1].record()
    torch.cuda.synchronize()
    us = ev[0].elapsed_time(ev[1]) * 1e3 / 20
    del src, dst
    return {"GBps": round(8 * n / us / 1e3, 1), "bytes_per_launch": 8 * n,
            "kernel": "int32 elementwise read + write (torch bitwise_not)"}


def calib_copy(args):
    """Counter calibration: a streaming elementwise kernel over int32 buffers
    (reads and writes each byte once, like a copy) of --calib-mib MiB, run
    --steps times.  A profiler's FETCH_SIZE / WRITE_SIZE per dispatch of it,
    against the bytes printed here, gives the counters' scale factor."""
    import torch
    n = (args.calib_mib << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    assert int(dst[12345].item()) == ~12345
    return {"calibration": "int32 bitwise_not", "read_bytes_per_dispatch": 4 * n,
            "write_bytes_per_dispatch": 4 * n, "dispatches": args.steps + 1,
            "GBps": round(8 * n / dt / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--sched", default="plain")
    ap.add_argument("--wg", type=int, default=0,
                    help="epoch-kernel work-group size (default: 1024 for the plain scheduler, the FFT "
                         "configuration and serving, 512 for BFS, SSSP and the traversals, 256 otherwise)")
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--log2tree", type=int, default=22, help="config 6: postorder tree of 2^k nodes")
    ap.add_argument("--sssp-deltas", type=lambda t: [int(x) for x in t.split(",") if x], default=[],
                    help="config 7: bucket widths to run beside the plain program (comma-separated)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--trees", type=int, default=4096)
    ap.add_argument("--graphs", type=int, default=64)
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--serve-warmup", type=int, default=60)
    ap.add_argument("--serve-arena-gib", type=int, default=16)
    ap.add_argument("--burst", type=int, default=4)
    ap.add_argument("--no-tune", dest="tune", action="store_false")
    ap.add_argument("--scheds", default="persistent,graph,plain")
    ap.add_argument("--plain-subset", type=int, default=512)
    ap.add_argument("--no-blocks", dest="blocks", action="store_false",
                    help="default line only: skip the batch, BFS and serving blocks")
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip the graph / persistent / naive-merge runs of the same workload")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only the counter-calibration copy kernel")
    ap.add_argument("--calib-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.wg == 0:
        args.wg = (1024 if (args.config in (1, 2, 8) and (args.sched == "plain" or args.config == 8))
                   or args.config == 5
                   else 512 if args.config in (4, 6, 7) else 256)
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent trees would shard by tree, one context per GPU)", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        line = calib_copy(args)
    elif args.config == 1:
        line = bench_cfg1(args)
    elif args.config == 3:
        line = bench_cfg3(args)
    elif args.config == 4:
        line = bench_cfg4(args)
    elif args.config == 5:
        line = bench_cfg5(args)
    elif args.config == 6:
        line = bench_cfg6(args)
    elif args.config == 7:
        line = bench_cfg7(args)
    elif args.config == 8:
        line = bench_cfg8(args)
    elif args.config == 2:
        line = bench_cfg2(args)
        log(f"default step: {line['value']:.4g} tasks/s")
        if not args.no_cpu:
            line["cpu_baseline"] = cpu_baseline_cfg2()
            log("cpu baseline done")
        if args.blocks:
            # the rest of the metric, measured in the same run and checked
            # against the oracle: batched vs per-epoch launch (the tree batch),
            # BFS (with the worklist comparison) and serving latency
            line["batch"] = batch_block(wg=512)
            log("batch block done")
            line["bfs"] = bfs_block(wg=512)
            log("bfs block done")
            line["serving"] = serving_block(wg=1024)
            log("serving block done")
    else:
        print(f"bench.py: --config {args.config} is not wired", file=sys.stderr)
        sys.exit(2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
