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
    assert o.sketch_source == L.SKETCH_AUTO
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


def test_ctypes_structures_match_the_header(tmp_path):
    """sizeof and offsetof of the option and info structs, from a C program
    compiled against include/sfgmres.h, equal the ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = {"sfgmres_options": L.Options, "sfgmres_info": L.Info, "sfgmres_csr": L.Csr}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln.strip()}
    for cname, cls in fields.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_vector_arguments_are_checked_before_any_launch():
    """The C ABI cannot tell host from device pointers, so the binding
    rejects host, float32, strided and wrongly sized vectors itself."""
    torch = pytest.importorskip("torch")
    import paper_2506_18408_amd.api as api
    cuda0 = torch.device("cuda", 0)
    with pytest.raises(ValueError, match="on cuda:0"):
        api.check_vector("b", torch.zeros(8, dtype=torch.float64), 8, cuda0)
    with pytest.raises(ValueError, match="float64"):
        api.check_vector("g", torch.zeros(8, dtype=torch.float32), 8, cuda0)
    cpu = torch.device("cpu")
    with pytest.raises(ValueError, match="contiguous"):
        api.check_vector("x0", torch.zeros(16, dtype=torch.float64)[::2], 8, cpu)
    with pytest.raises(ValueError, match="8 entries"):
        api.check_vector("out", torch.zeros(9, dtype=torch.float64), 8, cpu)
    api.check_vector("b", torch.zeros(8, dtype=torch.float64), 8, cpu)  # (well formed)
    with pytest.raises(ValueError, match="GPU"):
        api.solve(torch.zeros(9, dtype=torch.int32), torch.zeros(8, dtype=torch.int32),
                  torch.zeros(8, dtype=torch.float64), torch.zeros(8, dtype=torch.float64))
    with pytest.raises(ValueError, match="forced_k"):
        api.check_forced_k([3, 31], 30)
    with pytest.raises(ValueError, match="forced_k"):
        api.check_forced_k([-1], 30)
    api.check_forced_k([0, 30, 5], 30)
