"""GPU parity of the FFT program (radix-2 decimation in time, complex fp32):
every scheduler, through the C ABI, against the oracle's fp64 run of the same
task tree.  Task statistics and the per-epoch trace are integers and compared
exactly; the transform is compared within the fp32 error bound of a radix-2
FFT (tests/gpu_util.fft_tolerance)."""
import functools

import numpy as np
import pytest

import inputs
from tests.gpu_util import SCHEDS, Job, assert_matches_oracle, register_all

pytestmark = pytest.mark.gpu


def make_ctx(sched, trace=True, **kw):
    import paper_1608_00571_amd as T
    return T.Context(1 << 30, sched=sched, trace=trace, timeout_s=20.0, **kw)


def run_alone(sched, jobs, trace=True, **kw):
    with make_ctx(sched, trace=trace, **kw) as ctx:
        register_all(ctx, jobs)
        for j in jobs:
            j.submit(ctx)
        ctx.run()
        for j in jobs:
            j.collect(ctx, trace=trace)
    return jobs


@functools.lru_cache(maxsize=None)
def signal(m, seed=0):
    return inputs.complex_signal(1 << m, 500 + 37 * m + seed)


@pytest.mark.parametrize("sched", SCHEDS)
def test_fft_sizes(sched):
    """1 to 2^20 points: a lone leaf (and leaves of 1..32 points), one
    combine level, and up to 14 combine levels above 64-point leaves."""
    for m in [0, 1, 2, 5, 6, 7, 8, 10, 13, 16, 20]:
        (j,) = run_alone(sched, [Job("fft", signal=signal(m))], trace=m <= 16)
        assert_matches_oracle(j, check_trace=m <= 16)


@pytest.mark.parametrize("sched", SCHEDS)
def test_fft_closed_forms(sched):
    """An impulse transforms to all ones; a pure tone to N at its bin."""
    n = 1 << 12
    imp = np.zeros(n, dtype=np.complex64)
    imp[0] = 1
    k = np.arange(n)
    tone = np.exp(2j * np.pi * 1234 * k / n).astype(np.complex64)
    a, b = run_alone(sched, [Job("fft", signal=imp), Job("fft", signal=tone)])
    assert np.allclose(a.out, 1.0, atol=1e-6)
    want = np.zeros(n)
    want[1234] = n
    assert np.abs(b.out - want).max() < 1e-3 * n ** 0.5
    assert_matches_oracle(a)
    assert_matches_oracle(b)


@pytest.mark.parametrize("sched", SCHEDS)
def test_fft_batch(sched):
    """24 transforms of 1 to 2^14 points in one run (batched forms share
    epochs; the plain form runs them one after another)."""
    jobs = [Job("fft", signal=signal(m % 15, seed=g)) for g, m in enumerate(range(0, 48, 2))]
    run_alone(sched, jobs, trace=True)
    for j in jobs:
        assert_matches_oracle(j)


@pytest.mark.parametrize("sched", ["graph", "persistent"])
@pytest.mark.parametrize("wg", [256, 512, 1024])
def test_fft_arc_phase(sched, wg):
    """Combines of more than 16,384 butterflies go to the arc phase, beside
    a BFS tree whose hub arcs go there too."""
    g = inputs.rmat(12, 3)
    jobs = [Job("fft", signal=signal(18)), Job("bfs", graph=g)]
    run_alone(sched, jobs, wg=wg)
    for j in jobs:
        assert_matches_oracle(j)


def test_fft_bad_arguments():
    import torch

    import paper_1608_00571_amd as T
    with make_ctx("plain") as ctx:
        p = ctx.register(T.FFT)
        x = torch.zeros(2 << 10, dtype=torch.float32, device="cuda")
        y = torch.zeros_like(x)
        for args, bufs in [([21], [x, y]), ([-1], [x, y]), ([10], [x, x]), ([11], [x, y]), ([10], [x]),
                           ([9], [x[:1024], x[512:]])]:   # (the last two overlap by half)
            with pytest.raises(T.TreesError) as e:
                ctx.submit(p, args, bufs)
            assert e.value.status == T.E_INVALID
