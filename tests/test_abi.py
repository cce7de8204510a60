"""The C-ABI library loads on the CPU and exports every entry point that
include/trees.h declares (no compute calls: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "trees.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trees_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("trees_create", "trees_register_program", "trees_submit", "trees_run", "trees_results"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1608_00571_amd as T
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtrees.so not built")
    L = ctypes.CDLL(T.LIB_PATH)
    for n in declared():
        assert hasattr(L, n), n
    assert sorted(T.EXPORTED) == declared()


def test_tv_bound_on_host():
    import oracle
    import paper_1608_00571_amd as T
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtrees.so not built")
    # the admission size equals the emulator's peak (the tree's space)
    for n in (0, 1, 2, 10, 20):
        assert T.tv_bound(T.FIB_I64, [n]) == oracle.fib(n).peak
    for n in range(1, 10):
        assert T.tv_bound(T.NQUEENS, [n]) == oracle.nqueens(n).peak
    import inputs
    for N in (0, 1, 64, 65, 1000, 4099):
        _, r = oracle.msort(inputs.keys_u32(N, 1))
        assert T.tv_bound(T.MSORT_U32, [N]) == r.peak
    with pytest.raises(T.TreesError):
        T.tv_bound(T.FIB_I64, [44])
    with pytest.raises(T.TreesError):
        T.tv_bound(T.NQUEENS, [15])


def test_tv_bound_of_the_widened_programs():
    """Arena sizes of BFS, SSSP, the traversals and the FFT against the
    emulator's peaks (traversals, FFT) or their stated rules (BFS: V; SSSP:
    8 V unless the caller sets it), and their argument checks."""
    import numpy as np

    import inputs
    import oracle
    import paper_1608_00571_amd as T
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtrees.so not built")
    for n, seed in [(1, 0), (6, 1), (300, 2), (5000, 3)]:
        left, right = inputs.binary_tree(n, seed)
        _, _, rp = oracle.postorder(left, right, 0, records=False)
        _, _, rq = oracle.preorder(left, right, 0, records=False)
        assert T.tv_bound(T.POSTORDER, [n, 0]) >= rp.peak
        assert T.tv_bound(T.PREORDER, [n, 0]) == rq.peak == 2 * n + 1
    for m in (0, 3, 6, 7, 12, 20):
        if m <= 12:
            _, r = oracle.fft(np.zeros(1 << m, dtype=np.complex128))
            assert T.tv_bound(T.FFT, [m]) == r.peak
        assert T.tv_bound(T.FFT, [m]) == 2 * max(1, (1 << m) // 64) - 1
    assert T.tv_bound(T.BFS_CSR, [1000, 3]) == 1000
    assert T.tv_bound(T.SSSP_CSR, [1000, 3]) == 8000
    assert T.tv_bound(T.SSSP_CSR, [1000, 3, 123]) == 123
    assert T.tv_bound(T.SSSP_CSR, [1000, 3, 0, 16]) == 8000      # 0: the default, with a bucket width
    for kind, args in [(T.FFT, [21]), (T.FFT, [-1]), (T.PREORDER, [5, 5]), (T.PREORDER, [0, -1]),
                       (T.SSSP_CSR, [10, 10]), (T.SSSP_CSR, [10, 0, -1]), (T.SSSP_CSR, [10, 0, 0, 1 << 24])]:
        with pytest.raises(T.TreesError):
            T.tv_bound(kind, args)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1608_00571_amd as T
    monkeypatch.setattr(T, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(T, "_lib", None)
    with pytest.raises(ImportError):
        T.lib()


def test_worklist_workspace_bytes():
    """The worklist comparator's workspace: 256 B of counters and two lists of
    V int32 (plus V push stamps for SSSP), each section 256-byte aligned."""
    import paper_1608_00571_amd as T
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtrees.so not built")
    up = lambda x: (x + 255) // 256 * 256
    for V in (1, 63, 64, 1000, 1 << 22):
        assert T.wl_workspace_bytes(V) == 256 + 2 * up(4 * V)
        assert T.wl_workspace_bytes(V, sssp=True) == 256 + 3 * up(4 * V)
    with pytest.raises(T.TreesError):
        T.wl_workspace_bytes(0)
