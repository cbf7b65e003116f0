"""The C-ABI library loads and exports every entry point include/spx.h
declares, and its host-only checks behave (no GPU needed, no compute
call is made)."""
import ctypes as C
import os
import re

import pytest

from paper_2006_16767_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "spx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for n in ("spmv_csr", "spmspv_csc", "select_kernel", "run", "run_batch", "spmv_csr_transpose",
              "dvals_pattern", "spx_matrix_create", "spx_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == _declared_functions()


def test_version_and_error_string():
    lib = _lib.load()
    assert b"gfx950" in lib.spx_version()
    assert isinstance(lib.spx_last_error(), bytes)


def test_check_csr_host_only():
    lib = _lib.load()
    good = _lib.Csr(4, 5, 7, _lib.F32, C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000))
    assert lib.spx_check_csr(C.byref(good)) == 0
    bad_shape = _lib.Csr(-1, 5, 7, _lib.F32, C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000))
    assert lib.spx_check_csr(C.byref(bad_shape)) == -2
    no_vals = _lib.Csr(4, 5, 7, _lib.F32, C.c_void_p(0x1000), C.c_void_p(0x2000), None)
    assert lib.spx_check_csr(C.byref(no_vals)) == -1
    assert b"vals" in lib.spx_last_error()
    bool_no_vals = _lib.Csr(4, 5, 7, _lib.BOOL, C.c_void_p(0x1000), C.c_void_p(0x2000), None)
    assert lib.spx_check_csr(C.byref(bool_no_vals)) == 0
    bad_dt = _lib.Csr(4, 5, 7, 9, C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000))
    assert lib.spx_check_csr(C.byref(bad_dt)) == -4
    assert lib.spx_check_csr(None) == -1


@pytest.mark.parametrize("plan,ok", [
    ((0, 0, 0, 0, 0, 0), True),
    ((0, 1, 0, 0, 0, 0), True),
    ((1, 0, 0, 16, 0, 0), True),
    ((2, 1, 2, 0, 0, 0), True),
    ((2, 0, 4, 0, 0, 4096), True),
    ((2, 0, 0, 0, 0, 0), False),   # column-major needs a write-back
    ((0, 0, 1, 0, 0, 0), False),   # row-major takes none
    ((0, 0, 0, 3, 0, 0), False),   # lanes not a power of two
    ((3, 0, 0, 0, 0, 0), False),   # no such pattern
    ((2, 0, 4, 0, 0, 100), False), # bucket rows not a power of two
])
def test_check_plan(plan, ok):
    lib = _lib.load()
    p = _lib.Plan(*plan)
    rc = lib.spx_check_plan(C.byref(p), _lib.F32)
    assert (rc == 0) == ok


def test_workspace_sizes():
    lib = _lib.load()
    p = _lib.Plan(0, 0, 0, 0, 0, 0)
    assert lib.spx_workspace_size(100, 100, 1000, 100, _lib.F32, C.byref(p)) == 0
    pb = _lib.Plan(0, 1, 0, 0, 0, 0)
    assert lib.spx_workspace_size(100, 100, 1000, 100, _lib.F32, C.byref(pb)) > 0
    ps = _lib.Plan(2, 1, 2, 0, 0, 0)
    small = lib.spx_workspace_size(100, 100, 1000, 10, _lib.F32, C.byref(ps))
    big = lib.spx_workspace_size(100, 100, 100000, 10, _lib.F32, C.byref(ps))
    assert 0 < small < big
    bad = _lib.Plan(2, 0, 0, 0, 0, 0)
    assert lib.spx_workspace_size(100, 100, 1000, 10, _lib.F32, C.byref(bad)) == 0


def test_null_arguments_rejected_without_gpu():
    lib = _lib.load()
    p = _lib.Plan(0, 0, 0, 0, 0, 0)
    assert lib.spmv_csr(None, None, None, C.byref(p), None, 0, None) == -1
    out = C.c_void_p()
    assert lib.spx_matrix_create(None, 0, None, C.byref(out)) == -1
    assert lib.run(None, None, None, None) == -1
    assert lib.select_kernel(None, None, 0, None, None) == -1
    assert lib.spx_matrix_destroy(None) == 0


def test_dynamic_lds_declarations_are_aligned():
    """Every dynamic LDS array in the kernel sources is declared 16-byte
    aligned. Dynamic LDS starts right after a kernel's static LDS with no
    rounding, so an unaligned declaration can put 8-byte accumulators at a
    misaligned address (8-byte LDS operations then fault)."""
    csrc = os.path.join(ROOT, "paper_2006_16767_amd", "csrc")
    found = 0
    for name in sorted(os.listdir(csrc)):
        if not name.endswith((".hip", ".hpp", ".h", ".cpp")):
            continue
        for lineno, line in enumerate(open(os.path.join(csrc, name)), 1):
            code = line.split("//")[0]
            if "extern" in code and "__shared__" in code:
                found += 1
                assert "__align__(16)" in code, f"{name}:{lineno}: dynamic LDS without __align__(16)"
    assert found > 0


def test_noalloc_entry_rejects_oversized_plans_on_the_host():
    """spmspv_csc_noalloc refuses a plan whose workspace exceeds its fixed
    scratch before touching the device (fake pointers, never dereferenced)."""
    lib = _lib.load()
    cap = lib.spmspv_csc_noalloc_capacity()
    assert cap == 64 << 20
    big = _lib.Csc(1 << 20, 1 << 20, 1 << 26, _lib.F32, C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000))
    sort = _lib.Plan(_lib.PAT_CSC_SPMSPV, _lib.DIST_BALANCED, _lib.WB_SORT, 0, 0, 0)
    assert lib.spx_workspace_size(big.m, big.n, big.nnz, 16, _lib.F32, C.byref(sort)) > cap
    rc = lib.spmspv_csc_noalloc(C.byref(big), 16, C.c_void_p(0x4000), C.c_void_p(0x5000), C.c_void_p(0x6000),
                                C.byref(sort), None)
    assert rc == -8 and b"scratch" in lib.spx_last_error()
    rowmajor = _lib.Plan(_lib.PAT_SPMV, _lib.DIST_DIRECT, _lib.WB_NONE, 0, 0, 0)
    assert lib.spmspv_csc_noalloc(C.byref(big), 16, C.c_void_p(0x4000), C.c_void_p(0x5000), C.c_void_p(0x6000),
                                  C.byref(rowmajor), None) == -1
