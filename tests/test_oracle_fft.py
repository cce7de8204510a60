"""Pins of the oracle's FFT: the DFT by its defining sum against numpy's FFT;
the FFT program (epoch emulator, fp64) against numpy's FFT, the defining sum
and closed forms; its task and epoch counts against their closed forms."""
import numpy as np
import pytest

import inputs
import oracle


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 64, 100, 257])
def test_dft_is_numpy_fft(n):
    x = inputs.complex_signal(n, 10 + n).astype(np.complex128)
    assert rel_err(oracle.dft(x), np.fft.fft(x)) < 1e-12


@pytest.mark.parametrize("m", [0, 1, 5, 6, 7, 10, 16])
def test_fft_program_is_numpy_fft(m):
    n = 1 << m
    x = inputs.complex_signal(n, 100 + m).astype(np.complex128)
    y, r = oracle.fft(x)
    assert rel_err(y, np.fft.fft(x)) < 1e-12
    if m <= 10:
        assert rel_err(y, oracle.dft(x)) < 1e-12


@pytest.mark.parametrize("m", [0, 6, 7, 12])
def test_fft_closed_forms(m):
    n = 1 << m
    k = np.arange(n)
    y, _ = oracle.fft(np.eye(1, n, 0)[0].astype(np.complex128))       # impulse at 0: all ones
    assert np.allclose(y, 1.0, atol=1e-12)
    t = (5 * n) // 7
    y, _ = oracle.fft(np.eye(1, n, t)[0].astype(np.complex128))       # impulse at t: exp(-2 pi i k t / n)
    assert np.allclose(y, np.exp(-2j * np.pi * k * t / n), atol=1e-12)
    f = (3 * n) // 5
    y, _ = oracle.fft(np.exp(2j * np.pi * f * k / n))                 # a pure tone: n at bin f
    want = np.zeros(n, dtype=np.complex128)
    want[f] = n
    assert np.allclose(y, want, atol=1e-9 * n)


def test_fft_parseval_and_linearity():
    n = 1 << 11
    x = inputs.complex_signal(n, 7).astype(np.complex128)
    z = inputs.complex_signal(n, 8).astype(np.complex128)
    yx, _ = oracle.fft(x)
    yz, _ = oracle.fft(z)
    assert abs(np.vdot(yx, yx).real - n * np.vdot(x, x).real) < 1e-9 * n * np.vdot(x, x).real
    y, _ = oracle.fft(2.0 * x - 3j * z)
    assert rel_err(y, 2.0 * yx - 3j * yz) < 1e-12


@pytest.mark.parametrize("m", [0, 3, 6, 7, 8, 13])
def test_fft_task_counts(m):
    """A tree of FFT tasks down to 64-point leaves: 2L - 1 FFT tasks and
    L - 1 combines for L = max(1, n/64) leaves; the leaves run in epoch
    m - 6, and every combine level adds one epoch on the way back up."""
    n = 1 << m
    _, r = oracle.fft(inputs.complex_signal(n, 3).astype(np.complex128), records=True)
    leaves = max(1, n // oracle.FFT_LEAF)
    depth = max(0, m - 6)
    assert r.tasks_by_type == (2 * leaves - 1, leaves - 1)
    assert r.tasks == 3 * leaves - 2
    assert r.epochs == 2 * depth + 1
    assert [int(c) for c in r.records["cen"]] == list(range(depth + 1)) + list(range(depth - 1, -1, -1))
