"""CPU oracle for adaptive SpMV / SpMSpV (ctypes wrapper over oracle.c).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
baseline leg of the benchmark import this package. It does not import the
HIP library and the HIP library does not import it.

Matrices are passed as any object with attributes m, n, row_ptr (int32),
col_idx (int32) and vals (or as explicit arrays). Floating-point inputs
are widened to float64 before the call; every sum is Neumaier-compensated
in float64 and returned with S_i = sum |a_ij x_j| over the same terms.
The PageRank driver (pagerank_incremental) is a numpy loop over the
oracle's own product. Every function is pinned by the CPU tests.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    i32 = C.c_int32
    vp = C.c_void_p
    sig = {
        "oracle_spmv": [i32, i32, _i32p, _i32p, _f64p, _f64p, _f64p, vp],
        "oracle_transpose": [i32, i32, _i32p, _i32p, vp, _i32p, _i32p, vp, vp],
        "oracle_spmspv_csc": [i32, i32, _i32p, _i32p, _f64p, i32, _i32p, _f64p, _f64p, vp],
        "oracle_spmspv_csc_rows": [i32, i32, _i32p, _i32p, _f64p, i32, _i32p, _f64p, i32, i32, _f64p, vp],
        "oracle_spmspv_csc_omp": [i32, i32, _i32p, _i32p, _f64p, i32, _i32p, _f64p, _f64p, vp],
        "oracle_omp_threads": [],
        "oracle_bool_spmspv": [i32, i32, _i32p, _i32p, i32, _i32p, _u8p],
        "oracle_minplus_spmv": [i32, i32, _i32p, _i32p, _f32p, _f32p, _f32p],
        "oracle_int_spmv": [i32, i32, _i32p, _i32p, _i32p, _i32p, _i32p],
        "oracle_int_spmspv_csc": [i32, i32, _i32p, _i32p, _i32p, i32, _i32p, _i32p, _i32p],
        "oracle_grad": [i32, i32, _i32p, _i32p, _f64p, i32, _f64p, _f64p, vp, vp, vp],
        "oracle_matrix_features": [i32, i32, _i32p, _f64p],
        "oracle_vector_features": [i32, i32, _i32p, i32, _i32p, _f64p],
        "oracle_bfs_step": [C.c_int64, _i32p, _i32p, i32, _u8p, i32, _u8p],
        "oracle_bfs_levels": [C.c_int64, _i32p, _i32p, i32, i32, _i32p],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"{name} failed with code {rc}")


def spmv(A, x):
    """y = A x over CSR in float64 (compensated); returns (y, S)."""
    lib = _load()
    y = np.empty(A.m, np.float64)
    s = np.empty(A.m, np.float64)
    _check(lib.oracle_spmv(A.m, A.n, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.vals), _f64(x),
                           y, _ptr(s)), "oracle_spmv")
    return y, s


class CSC:
    """The oracle's own column-major copy of a CSR matrix."""

    def __init__(self, m, n, col_ptr, row_idx, perm, vals):
        self.m, self.n = m, n
        self.col_ptr, self.row_idx, self.perm, self.vals = col_ptr, row_idx, perm, vals


def transpose(A, with_values: bool = True, int_values: bool = False) -> CSC:
    """Stable counting-sort CSR -> CSC with the csc-to-csr permutation."""
    lib = _load()
    nnz = int(A.row_ptr[-1])
    col_ptr = np.empty(A.n + 1, np.int32)
    row_idx = np.empty(nnz, np.int32)
    perm = np.empty(nnz, np.int32)
    vals = None
    vals_csc = None
    if with_values and A.vals is not None and not int_values:
        vals = _f64(A.vals)
        vals_csc = np.empty(nnz, np.float64)
    _check(lib.oracle_transpose(A.m, A.n, _i32(A.row_ptr), _i32(A.col_idx), _ptr(vals),
                                col_ptr, row_idx, _ptr(perm), _ptr(vals_csc)), "oracle_transpose")
    if int_values and A.vals is not None:
        # integer values move with the same permutation the oracle produced
        vals_csc = np.ascontiguousarray(np.asarray(A.vals, dtype=np.int32)[perm])
    return CSC(A.m, A.n, col_ptr, row_idx, perm, vals_csc)


def spmspv(csc: CSC, x_idx, x_val):
    """Vector-driven column-major SpMSpV into a dense y; returns (y, S)."""
    lib = _load()
    y = np.empty(csc.m, np.float64)
    s = np.empty(csc.m, np.float64)
    x_idx = _i32(x_idx)
    _check(lib.oracle_spmspv_csc(csc.m, csc.n, csc.col_ptr, csc.row_idx, _f64(csc.vals),
                                 x_idx.size, x_idx, _f64(x_val), y, _ptr(s)),
           "oracle_spmspv_csc")
    return y, s


def spmspv_rows(csc: CSC, x_idx, x_val, r0: int, r1: int):
    """The column scatter restricted to output rows [r0, r1) (equal to
    spmspv's rows bit for bit); returns (y, S) over those rows only."""
    lib = _load()
    y = np.zeros(csc.m, np.float64)
    s = np.zeros(csc.m, np.float64)
    x_idx = _i32(x_idx)
    _check(lib.oracle_spmspv_csc_rows(csc.m, csc.n, csc.col_ptr, csc.row_idx, _f64(csc.vals), x_idx.size,
                                      x_idx, _f64(x_val), int(r0), int(r1), y, _ptr(s)),
           "oracle_spmspv_csc_rows")
    return y[r0:r1], s[r0:r1]


def spmspv_omp(csc: CSC, x_idx, x_val):
    """spmspv with disjoint row ranges on the host's cores (OpenMP); the
    same bits as spmspv. Returns (y, S)."""
    lib = _load()
    y = np.empty(csc.m, np.float64)
    s = np.empty(csc.m, np.float64)
    x_idx = _i32(x_idx)
    _check(lib.oracle_spmspv_csc_omp(csc.m, csc.n, csc.col_ptr, csc.row_idx, _f64(csc.vals), x_idx.size,
                                     x_idx, _f64(x_val), y, _ptr(s)), "oracle_spmspv_csc_omp")
    return y, s


def omp_threads() -> int:
    """Threads the OpenMP leg uses (OMP_NUM_THREADS, else the host's cores)."""
    return int(_load().oracle_omp_threads())


def bool_spmspv(A, x_idx):
    """(OR, AND) product of the pattern of A with the index set x_idx;
    returns uint8 y in {0, 1}."""
    lib = _load()
    y = np.empty(A.m, np.uint8)
    x_idx = _i32(x_idx)
    _check(lib.oracle_bool_spmspv(A.m, A.n, _i32(A.row_ptr), _i32(A.col_idx), x_idx.size, x_idx,
                                  y), "oracle_bool_spmspv")
    return y


def int_spmv(A, x):
    """(+, x) mod 2^32 SpMV with int32 values and dense int32 x."""
    lib = _load()
    y = np.empty(A.m, np.int32)
    _check(lib.oracle_int_spmv(A.m, A.n, _i32(A.row_ptr), _i32(A.col_idx), _i32(A.vals), _i32(x),
                               y), "oracle_int_spmv")
    return y


def int_spmspv(csc: CSC, x_idx, x_val):
    """(+, x) mod 2^32 column-scatter SpMSpV (csc from transpose(...,
    int_values=True))."""
    lib = _load()
    y = np.empty(csc.m, np.int32)
    x_idx = _i32(x_idx)
    _check(lib.oracle_int_spmspv_csc(csc.m, csc.n, csc.col_ptr, csc.row_idx, _i32(csc.vals),
                                     x_idx.size, x_idx, _i32(x_val), y), "oracle_int_spmspv_csc")
    return y


def grad(A, G, X, want_dx=True, want_dvals=True):
    """For L = sum_b <G[b], A X[b]>: returns (dX, S_dX, dvals).
    G is B x m, X is B x n (dense, zero-filled for sparse inputs)."""
    lib = _load()
    G = np.atleast_2d(_f64(G))
    X = np.atleast_2d(_f64(X))
    B = G.shape[0]
    dX = np.empty((B, A.n), np.float64) if want_dx else None
    sdX = np.empty((B, A.n), np.float64) if want_dx else None
    dv = np.empty(int(A.row_ptr[-1]), np.float64) if want_dvals else None
    _check(lib.oracle_grad(A.m, A.n, _i32(A.row_ptr), _i32(A.col_idx), _f64(A.vals), B, G, X,
                           _ptr(dX), _ptr(sdX), _ptr(dv)), "oracle_grad")
    return dX, sdX, dv


MATRIX_FEATURES = ("m", "n", "nnz", "max_row", "min_row", "avg_row", "relative_range",
                   "var_nnz_row", "gini")
VECTOR_FEATURES = ("nnz_x", "x_sparsity", "nnz_s", "m_sparsity")


def matrix_features(A) -> dict:
    lib = _load()
    out = np.empty(9, np.float64)
    _check(lib.oracle_matrix_features(A.m, A.n, _i32(A.row_ptr), out), "oracle_matrix_features")
    return dict(zip(MATRIX_FEATURES, out.tolist()))


def vector_features(csc: CSC, x_idx) -> dict:
    lib = _load()
    out = np.empty(4, np.float64)
    x_idx = _i32(x_idx)
    _check(lib.oracle_vector_features(csc.n, int(csc.col_ptr[-1]), csc.col_ptr, x_idx.size, x_idx,
                                      out), "oracle_vector_features")
    return dict(zip(VECTOR_FEATURES, out.tolist()))


def bfs_levels(src, dst, n, source):
    """Breadth-first levels from source over the directed edges src -> dst
    (-1 where unreachable)."""
    lib = _load()
    src = _i32(src)
    dst = _i32(dst)
    level = np.empty(n, np.int32)
    _check(lib.oracle_bfs_levels(src.size, src, dst, n, source, level), "oracle_bfs_levels")
    return level


def bfs_step(src, dst, n, m, active_idx):
    """Next frontier (uint8 mask over [0, m)) of an edge-list expansion from
    the active vertex set."""
    lib = _load()
    src = _i32(src)
    dst = _i32(dst)
    act = np.zeros(n, np.uint8)
    act[np.asarray(active_idx, dtype=np.int64)] = 1
    nxt = np.empty(m, np.uint8)
    _check(lib.oracle_bfs_step(src.size, src, dst, n, act, m, nxt), "oracle_bfs_step")
    return nxt


def pagerank_incremental(A, damping, eps, max_iters):
    """Incremental (residual-push) PageRank, the second application of the
    paper's evaluation (Section 7), in float64.

    Stored entry (i, j) is an edge j -> i of weight a_ij >= 0; a walk
    leaves j along (i, j) with probability a_ij / W_j, W_j = the sum of
    column j (W_j = 0: j is dangling and its mass leaves the graph). The
    fixed point p solves p = (1 - d)/n * 1 + d * P p, P = A diag(1/W).

    Residual form: r starts at (1 - d)/n everywhere and p at 0. Each
    round, the active vertices (|r_v| > eps) move r_v into p_v; those that
    are not dangling form the sparse input x_v = r_v / W_v of one product
    y = A x; their residual is cleared and r += d * y. The rounds stop
    when no active vertex can propagate or after max_iters products.

    Returns (p, r, products). At any stop, p + (I - d P)^-1 r is the fixed
    point, and when the loop ends by itself every |r_v| <= eps except on
    vertices that are dangling, whose residual was moved (so they are 0)."""
    n = A.n
    assert A.m == n, "PageRank needs a square matrix"
    d = float(damping)
    vals = _f64(A.vals)
    W = np.zeros(n)
    np.add.at(W, _i32(A.col_idx), vals)
    r = np.full(n, (1.0 - d) / n)
    p = np.zeros(n)
    products = 0
    while products < max_iters:
        active = np.abs(r) > eps
        p[active] += r[active]
        prop = active & (W > 0)
        x = np.zeros(n)
        x[prop] = r[prop] / W[prop]
        r[active] = 0.0
        if not prop.any():
            break
        y, _ = spmv(A, x)
        r += d * y
        products += 1
    return p, r, products


def spmspv_sparse(A, x_idx, x_val=None, mask=None, kind="f64"):
    """Sparse-output SpMSpV with a complement mask (the frontier form of
    y = A x that the paper's BFS application chains, Section 7): the rows i
    with at least one stored entry in a column of supp(x) (structural, so a
    row whose products sum to 0 is still listed) and mask[i] false (mask:
    bool[m] or None), ascending, with their values of y = A x.

    kind: "f64" (compensated float64, values and S), "i32" ((+, x) mod 2^32)
    or "bool" ((OR, AND): values all 1). Returns (rows, values, S) with S
    None except for "f64". Built from the oracle's own dense products: the
    pattern product decides which rows are listed, the value product
    supplies their values."""
    touched = bool_spmspv(A, x_idx).astype(bool)
    keep = touched if mask is None else touched & ~np.asarray(mask, bool)
    rows = np.nonzero(keep)[0].astype(np.int32)
    if kind == "bool":
        return rows, np.ones(rows.size, np.uint8), None
    if kind == "i32":
        csc = transpose(A, int_values=True)
        y = int_spmspv(csc, x_idx, x_val)
        return rows, y[rows], None
    csc = transpose(A)
    y, s = spmspv(csc, x_idx, x_val)
    return rows, y[rows], s[rows]


def minplus_spmv(A, x):
    """Min-plus product over float32: y_i = min over stored (i, j) of
    (a_ij + x_j) with x_j = +inf meaning absent; +inf where nothing is
    effective (shortest-path relaxation, the semiring extension of the
    paper's closing section)."""
    lib = _load()
    y = np.empty(A.m, np.float32)
    _check(lib.oracle_minplus_spmv(A.m, A.n, _i32(A.row_ptr), _i32(A.col_idx),
                                   np.ascontiguousarray(A.vals, dtype=np.float32),
                                   np.ascontiguousarray(x, dtype=np.float32), y), "oracle_minplus_spmv")
    return y


def minplus_spmspv(A, x_idx, x_val):
    """The sparse-x form: SpMV with the absent entries at +inf (the semiring
    zero), so SpMSpV equals SpMV with the zero-filled vector, as it does in
    the other semirings."""
    x = np.full(A.n, np.inf, np.float32)
    x[np.asarray(x_idx, np.int64)] = np.asarray(x_val, np.float32)
    return minplus_spmv(A, x)
