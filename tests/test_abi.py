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


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1608_00571_amd as T
    monkeypatch.setattr(T, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(T, "_lib", None)
    with pytest.raises(ImportError):
        T.lib()
