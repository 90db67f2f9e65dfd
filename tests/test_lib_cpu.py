"""CPU checks of the C-ABI library: it loads, exports every function the
public header declares, and its host-only entry points behave (no GPU work)."""
import ctypes as C
import os

import pytest

import paper_2506_18408_amd._lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfgmres.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2506_18408_amd import build
        build.build()
    return L.load()


def test_exports_every_declared_symbol(lib):
    names = L.header_symbols(HEADER)
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.SIGNATURES)


def test_nm_lists_symbols_as_global_text(lib):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in L.header_symbols(HEADER):
        assert name in exported, name


def test_default_options(lib):
    o = L.Options()
    assert lib.sfgmres_default_options(C.byref(o)) == 0
    # cond_threshold 0 selects the precision's default (1e15 in FP64)
    assert o.precision == L.FP64 and o.max_outer == 100 and o.cond_threshold == 0.0
    assert lib.sfgmres_default_options(None) == L.ERR_INVALID


def test_workspace_bytes(lib):
    out = C.c_size_t()
    assert lib.sfgmres_workspace_bytes(4096, 20224, 30, 2, 60, 8, None, 0, C.byref(out)) == 0
    small = out.value
    assert small > 8 * 4096 * (30 + 1 + 2 * 100 + 1)
    o = L.Options()
    lib.sfgmres_default_options(C.byref(o))
    o.precision = L.MIXED
    assert lib.sfgmres_workspace_bytes(4096, 20224, 30, 2, 60, 8, C.byref(o), 0, C.byref(out)) == 0
    mixed = out.value
    assert mixed < small + 4 * 20224 + 4 * 4096 + 4096
    assert lib.sfgmres_workspace_bytes(4096, 20224, 30, 2, 60, 8, None, 1, C.byref(out)) == 0
    assert out.value > small + 16 * 20224
    # invalid sizes
    assert lib.sfgmres_workspace_bytes(4096, 20224, 60, 2, 60, 8, None, 0, C.byref(out)) == L.ERR_INVALID
    assert lib.sfgmres_workspace_bytes(0, 0, 30, 2, 60, 8, None, 0, C.byref(out)) == L.ERR_INVALID
    assert lib.sfgmres_workspace_bytes(10, 10, 30, 2, 60, 8, None, 0, None) == L.ERR_INVALID


def test_small_workspace_queries(lib):
    out = C.c_size_t()
    # (at least the packed sketch: 12 bytes per column at zeta = 8)
    assert lib.sfgmres_sketch_workspace_bytes(10**6, 400, 8, C.byref(out)) == 0 and out.value >= 12 * 10**6
    assert lib.sfgmres_sketch_workspace_bytes(10**6, 5000, 8, C.byref(out)) == L.ERR_INVALID
    assert lib.sfgmres_transpose_workspace_bytes(100, 500, C.byref(out)) == 0
    assert lib.sfgmres_spmv_workspace_bytes(100, 500, 60, 8, C.byref(out)) == 0


def test_null_handle_is_rejected(lib):
    assert lib.sfgmres_solve(None, None, None, None, None, 30, 2, 60, 8, 1e-8, 0, None, None,
                             None, 0, None) == L.ERR_INVALID
    assert lib.sfgmres_last_error(None) == b"null handle"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_LIB", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L.load()
