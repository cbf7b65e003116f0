"""ctypes declarations of the libspx C ABI (include/spx.h).

Argument marshalling only. Loading fails loudly when libspx.so is missing:
there is no CPU fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspx.so")

SPX_OK = 0
ERRORS = {
    -1: "SPX_ERR_ARG", -2: "SPX_ERR_SHAPE", -3: "SPX_ERR_INDEX", -4: "SPX_ERR_DTYPE",
    -5: "SPX_ERR_UNSUPPORTED", -6: "SPX_ERR_ALLOC", -7: "SPX_ERR_HIP", -8: "SPX_ERR_WORKSPACE",
}

F32, F64, BOOL, I32, F32_MINPLUS = 0, 1, 2, 3, 4
PAT_SPMV, PAT_CSR_SPMSPV, PAT_CSC_SPMSPV = 0, 1, 2
DIST_DIRECT, DIST_BALANCED = 0, 1
WB_NONE, WB_ATOMIC, WB_SORT, WB_LDS_ATOMIC, WB_BUCKET, WB_MERGE = 0, 1, 2, 3, 4, 5
VEC_DENSE, VEC_SPARSE = 0, 1
VALIDATE, NO_SYNC, RENUMBER, NO_RENUMBER, FORMAT_CSR, FORMAT_SELL, FORMAT_ELL, FORMAT_CSR5 = 1, 2, 4, 8, 16, 32, 64, 128
FORMAT_DIA = 256
BFS_PUSH_ONLY = 1


class Plan(C.Structure):
    _fields_ = [("pattern", C.c_int32), ("distribution", C.c_int32), ("writeback", C.c_int32),
                ("lanes", C.c_int32), ("tile", C.c_int32), ("bucket_rows", C.c_int32)]

    def as_tuple(self):
        return (self.pattern, self.distribution, self.writeback, self.lanes, self.tile, self.bucket_rows)

    def __repr__(self):
        pat = ["spmv", "csr_spmspv", "csc_spmspv"][self.pattern] if 0 <= self.pattern < 3 else "?"
        dist = ["direct", "balanced"][self.distribution] if 0 <= self.distribution < 2 else "?"
        wb = (["none", "atomic", "sort", "lds_atomic", "bucket", "merge"][self.writeback]
              if 0 <= self.writeback < 6 else "?")
        return f"Plan({pat}, {dist}, {wb}, lanes={self.lanes}, tile={self.tile}, bucket_rows={self.bucket_rows})"


class Csr(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int32), ("dtype", C.c_int32),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("vals", C.c_void_p)]


class Csc(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int32), ("dtype", C.c_int32),
                ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p), ("vals", C.c_void_p)]


class Vec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("nnz_x", C.c_int32), ("idx", C.c_void_p),
                ("val", C.c_void_p)]


# name -> (restype, argtypes); every name here is declared in include/spx.h
P = C.c_void_p
_i32 = C.c_int32
SIGNATURES = {
    "spx_workspace_size": (C.c_size_t, [_i32, _i32, _i32, _i32, _i32, C.POINTER(Plan)]),
    "spmv_csr": (C.c_int, [C.POINTER(Csr), P, P, C.POINTER(Plan), P, C.c_size_t, P]),
    "spmspv_csr": (C.c_int, [C.POINTER(Csr), _i32, P, P, P, C.POINTER(Plan), P, C.c_size_t, P]),
    "spmspv_csc": (C.c_int, [C.POINTER(Csc), _i32, P, P, P, C.POINTER(Plan), P, C.c_size_t, P]),
    "spmspv_csc_noalloc": (C.c_int, [C.POINTER(Csc), _i32, P, P, P, C.POINTER(Plan), P]),
    "spmspv_csc_noalloc_capacity": (C.c_size_t, []),
    "spx_matrix_create": (C.c_int, [C.POINTER(Csr), C.c_uint32, P, C.POINTER(P)]),
    "spx_matrix_destroy": (C.c_int, [P]),
    "spx_matrix_csc": (C.c_int, [P, C.POINTER(Csc)]),
    "spx_matrix_values_updated": (C.c_int, [P, P]),
    "spx_matrix_column_order": (C.c_int, [P, P, C.POINTER(C.c_int32), P]),
    "spx_matrix_features": (C.c_int, [P, C.POINTER(C.c_double)]),
    "spx_matrix_format": (C.c_int, [P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "spx_vector_features": (C.c_int, [P, C.POINTER(Vec), C.POINTER(C.c_double), P]),
    "spx_load_selector": (C.c_int, [P, C.c_char_p]),
    "select_kernel": (C.c_int, [P, C.POINTER(Vec), C.c_uint32, C.POINTER(Plan), P]),
    "run": (C.c_int, [P, C.POINTER(Vec), P, P]),
    "run_plan": (C.c_int, [P, C.POINTER(Vec), P, C.POINTER(Plan), P]),
    "spx_last_plan": (C.c_int, [P, C.POINTER(Plan)]),
    "spx_set_profiling": (C.c_int, [P, _i32]),
    "spx_stage_times": (C.c_int, [P, C.POINTER(C.c_double)]),
    "spx_run_times": (C.c_int, [P, C.POINTER(C.c_double), _i32, C.POINTER(_i32)]),
    "run_batch": (C.c_int, [P, _i32, C.c_int64, P, P, P, P, P]),
    "spx_batch_status": (C.c_int, [P, C.POINTER(_i32), P]),
    "spx_bfs": (C.c_int, [P, _i32, P, _i32, C.POINTER(Plan), C.c_uint32, C.POINTER(C.c_int32), C.POINTER(Plan),
                          _i32, P]),
    "spmspv_sparse": (C.c_int, [P, C.POINTER(Vec), P, C.POINTER(Plan), P, P, C.POINTER(C.c_int32), P]),
    "spx_pagerank": (C.c_int, [P, C.c_double, C.c_double, _i32, C.POINTER(Plan), P, P, C.POINTER(C.c_int32),
                               C.POINTER(Plan), _i32, P]),
    "spmv_csr_batch": (C.c_int, [P, _i32, P, P, P]),
    "spmv_csr_transpose": (C.c_int, [P, _i32, P, P, P]),
    "dvals_pattern": (C.c_int, [P, _i32, P, P, P, P]),
    "spx_backward": (C.c_int, [P, _i32, P, P, P, P, P]),
    "spx_pack_mask": (C.c_int, [_i32, P, P, P]),
    "spx_dense_rows_to_sparse": (C.c_int, [P, _i32, P, P, P, P, P]),
    "spx_stream_copy": (C.c_int, [P, P, C.c_size_t, P]),
    "spx_check_csr": (C.c_int, [C.POINTER(Csr)]),
    "spx_check_plan": (C.c_int, [C.POINTER(Plan), _i32]),
    "spx_last_error": (C.c_char_p, []),
    "spx_version": (C.c_char_p, []),
}

_lib = None


class SpxError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__(f"{fn}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


def load():
    """Loads libspx.so (built by paper_2006_16767_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libspx.so not found at {LIB_PATH}; build it with "
                           "`python paper_2006_16767_amd/build.py` (there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int, fn: str):
    if code != SPX_OK:
        msg = load().spx_last_error().decode(errors="replace")
        raise SpxError(code, fn, msg)


def call(name: str, *args):
    lib = load()
    rc = getattr(lib, name)(*args)
    check(rc, name)
    return rc
