"""Adaptive SpMV / SpMSpV on AMD MI355X (gfx950).

A thin Python layer over libspx (include/spx.h). PyTorch supplies device
memory and streams; every step of the computation runs in the library's HIP
kernels. Importing this package does not load the library; the first call
does, and fails loudly if it has not been built.

    A = Matrix.from_csr(row_ptr, col_idx, vals, n)      # torch tensors on cuda
    y = A.run(x)                 # dense x (tensor of length n)
    y = A.run((idx, val))        # sparse x (indices, values)
    y = A.run_plan(x, plan)      # a given candidate kernel
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import (BOOL, DIST_BALANCED, DIST_DIRECT, F32, F32_MINPLUS, F64, I32, NO_SYNC, PAT_CSC_SPMSPV,
                   PAT_CSR_SPMSPV, PAT_SPMV, VALIDATE, RENUMBER, NO_RENUMBER, FORMAT_CSR, FORMAT_SELL, FORMAT_ELL,
                   FORMAT_CSR5, FORMAT_DIA,
                   WB_ATOMIC, WB_BUCKET, WB_LDS_ATOMIC, WB_NONE,
                   WB_MERGE, WB_SORT, Plan, SpxError)

__all__ = ["Matrix", "Plan", "SpxError", "plan", "spmv_csr", "spmspv_csr", "spmspv_csc",
           "F32", "F64", "BOOL", "I32", "all_plans"]

_DEFAULT_SELECTOR = __import__("os").path.join(__import__("os").path.dirname(__file__), "selector_mi355x.json")
# trees that also test nnz_s, for the callers that know it (the graph
# drivers)
_NNZ_S_SELECTOR = __import__("os").path.join(__import__("os").path.dirname(__file__), "selector_mi355x_nnz_s.json")
# trees trained on (OR, AND) timings, loaded into BOOL handles (host
# features, then with nnz_s)
_BOOL_SELECTOR = __import__("os").path.join(__import__("os").path.dirname(__file__), "selector_mi355x_bool.json")
_BOOL_NNZ_S_SELECTOR = __import__("os").path.join(__import__("os").path.dirname(__file__),
                                                  "selector_mi355x_bool_nnz_s.json")
# lazy trees for run(): they may ask for nnz_s (a device count and a round
# trip to the host) at the leaves where the training vectors gained by it.
# Not loaded by default: on the uniform sweep the round trip costs more than
# it saves (Matrix.load_selector(LAZY_SELECTOR) opts in).
LAZY_SELECTOR = __import__("os").path.join(__import__("os").path.dirname(__file__), "selector_mi355x_lazy.json")
_selector_loaded = False


def _ensure_default_selector():
    """Loads the trees trained on MI355X timings (selector_mi355x.json, then
    selector_mi355x_nnz_s.json) once, before the first handle is created;
    spx_load_selector can replace them."""
    global _selector_loaded
    if _selector_loaded:
        return
    import os
    for path in (_DEFAULT_SELECTOR, _NNZ_S_SELECTOR):
        if os.path.exists(path):
            _lib.call("spx_load_selector", None, path.encode())
    _selector_loaded = True


def _torch():
    import torch
    return torch


def dtype_code(t) -> int:
    torch = _torch()
    return {torch.float32: F32, torch.float64: F64, torch.int32: I32, torch.uint8: BOOL,
            torch.bool: BOOL}[t]


def torch_dtype(code: int):
    torch = _torch()
    return {F32: torch.float32, F64: torch.float64, I32: torch.int32, BOOL: torch.uint8,
            F32_MINPLUS: torch.float32}[code]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream.cuda_stream)
    torch = _torch()
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:  # the current stream's handle without building a Stream object
        return C.c_void_p(raw(torch._C._cuda_getDevice()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def plan(pattern="spmv", distribution="direct", writeback="none", lanes=0, tile=0, bucket_rows=0) -> Plan:
    pat = {"spmv": PAT_SPMV, "csr_spmspv": PAT_CSR_SPMSPV, "csc_spmspv": PAT_CSC_SPMSPV}[pattern]
    dist = {"direct": DIST_DIRECT, "balanced": DIST_BALANCED}[distribution]
    wb = {"none": WB_NONE, "atomic": WB_ATOMIC, "sort": WB_SORT, "lds_atomic": WB_LDS_ATOMIC,
          "bucket": WB_BUCKET, "merge": WB_MERGE}[writeback]
    return Plan(pat, dist, wb, lanes, tile, bucket_rows)


def all_plans(include_bucket=True):
    """Every candidate kernel (automatic launch parameters)."""
    out = []
    for d in ("direct", "balanced"):
        out.append(plan("spmv", d))
        out.append(plan("csr_spmspv", d))
        for wb in ("atomic", "lds_atomic", "sort", "merge") + (("bucket",) if include_bucket else ()):
            out.append(plan("csc_spmspv", d, wb))
    return out


def _vec(x, n):
    """x: dense tensor (length n) or (idx, val) pair; val may be None for BOOL."""
    if isinstance(x, tuple):
        idx, val = x
        return _lib.Vec(_lib.VEC_SPARSE, n, int(idx.numel()), _ptr(idx), _ptr(val)), (idx, val)
    # the library checks the dense length against the matrix's n
    return _lib.Vec(_lib.VEC_DENSE, int(x.numel()), -1, None, _ptr(x)), (x,)


class Matrix:
    """Handle over a CSR matrix on the GPU plus its device-built CSC copy.

    The CSR tensors are borrowed (kept alive by this object); the CSC copy,
    features and workspaces belong to the library handle."""

    def __init__(self, row_ptr, col_idx, vals, m: int, n: int, dtype: int | None = None,
                 validate: bool = False, renumber: bool | None = None, stream=None, fmt: str | None = None):
        torch = _torch()
        self.row_ptr = row_ptr.contiguous()
        self.col_idx = col_idx.contiguous()
        self.vals = None if vals is None else vals.contiguous()
        self.m, self.n = int(m), int(n)
        self.nnz = int(self.col_idx.numel())
        if dtype is None:
            dtype = BOOL if vals is None else dtype_code(vals.dtype)
        self.dtype = dtype
        assert self.row_ptr.dtype == torch.int32 and self.col_idx.dtype == torch.int32
        self._csr = _lib.Csr(self.m, self.n, self.nnz, dtype, _ptr(self.row_ptr), _ptr(self.col_idx),
                             _ptr(self.vals))
        _ensure_default_selector()
        h = C.c_void_p()
        flags = (VALIDATE if validate else 0) | {None: 0, True: RENUMBER, False: NO_RENUMBER}[renumber]
        flags |= {None: 0, "csr": FORMAT_CSR, "sell": FORMAT_SELL, "ell": FORMAT_ELL, "csr5": FORMAT_CSR5,
                  "dia": FORMAT_DIA}[fmt]
        _lib.call("spx_matrix_create", C.byref(self._csr), flags, _stream(stream), C.byref(h))
        self._h = h
        if dtype == BOOL:
            for path in (_BOOL_SELECTOR, _BOOL_NNZ_S_SELECTOR):
                if __import__("os").path.exists(path):
                    _lib.call("spx_load_selector", self._h, path.encode())
        self._vals_version = None if self.vals is None else self.vals._version

    @classmethod
    def from_host(cls, A, dtype=None, device="cuda", validate=False, renumber=None, fmt=None):
        """From an object with m, n, row_ptr, col_idx, vals (numpy)."""
        torch = _torch()
        rp = torch.as_tensor(A.row_ptr, dtype=torch.int32, device=device)
        ci = torch.as_tensor(A.col_idx, dtype=torch.int32, device=device)
        if dtype == BOOL or A.vals is None:
            v = None
            dt = BOOL
        else:
            v = torch.as_tensor(A.vals, device=device)
            if dtype is not None:
                v = v.to(torch_dtype(dtype))
            dt = dtype_code(v.dtype) if dtype is None else dtype  # F32_MINPLUS shares float32
        return cls(rp, ci, v, A.m, A.n, dt, validate=validate, renumber=renumber, fmt=fmt)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().spx_matrix_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def out_tensor(self, batch: int | None = None):
        torch = _torch()
        shape = (self.m,) if batch is None else (batch, self.m)
        return torch.empty(shape, dtype=torch_dtype(self.dtype), device=self.row_ptr.device)

    def csc_pointers(self):
        c = _lib.Csc()
        _lib.call("spx_matrix_csc", self._h, C.byref(c))
        return c

    def csc(self):
        """Copies of the handle's CSC arrays as tensors (for tests)."""
        torch = _torch()
        c = self.csc_pointers()
        dev = self.row_ptr.device
        col_ptr = torch.empty(self.n + 1, dtype=torch.int32, device=dev)
        row_idx = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        _copy_raw(col_ptr, c.col_ptr)
        _copy_raw(row_idx, c.row_idx)
        vals = None
        if self.dtype != BOOL:
            vals = torch.empty(self.nnz, dtype=torch_dtype(self.dtype), device=dev)
            _copy_raw(vals, c.vals)
        return col_ptr, row_idx, vals

    def features(self) -> dict:
        out = (C.c_double * 9)()
        _lib.call("spx_matrix_features", self._h, out)
        keys = ("m", "n", "nnz", "max_row", "min_row", "avg_row", "relative_range", "var_nnz_row", "gini")
        return dict(zip(keys, list(out)))

    def vector_features(self, x, stream=None) -> dict:
        v, keep = _vec(x, self.n)
        out = (C.c_double * 4)()
        _lib.call("spx_vector_features", self._h, C.byref(v), out, _stream(stream))
        return dict(zip(("nnz_x", "x_sparsity", "nnz_s", "m_sparsity"), list(out)))

    def select(self, x, no_sync=False, stream=None) -> Plan:
        v, keep = _vec(x, self.n)
        p = Plan()
        _lib.call("select_kernel", self._h, C.byref(v), NO_SYNC if no_sync else 0, C.byref(p),
                  _stream(stream))
        return p

    def run(self, x, y=None, stream=None):
        v, keep = _vec(x, self.n)
        y = self.out_tensor() if y is None else y
        _lib.call("run", self._h, C.byref(v), _ptr(y), _stream(stream))
        return y

    def run_plan(self, x, p: Plan, y=None, stream=None):
        v, keep = _vec(x, self.n)
        y = self.out_tensor() if y is None else y
        _lib.call("run_plan", self._h, C.byref(v), _ptr(y), C.byref(p), _stream(stream))
        return y

    def last_plan(self) -> Plan:
        p = Plan()
        _lib.call("spx_last_plan", self._h, C.byref(p))
        return p

    def set_profiling(self, on: bool):
        _lib.call("spx_set_profiling", self._h, 1 if on else 0)

    def stage_times(self) -> dict:
        out = (C.c_double * 4)()
        _lib.call("spx_stage_times", self._h, out)
        return dict(zip(("features_ms", "model_ms", "conversion_ms", "kernel_ms"), list(out)))

    def run_times(self, cap: int = 1 << 16):
        """Per-run kernel times (ms) recorded while profiling was on."""
        out = (C.c_double * cap)()
        cnt = C.c_int32()
        _lib.call("spx_run_times", self._h, out, cap, C.byref(cnt))
        return list(out[:min(cnt.value, cap)])

    def values_updated(self, stream=None):
        _lib.call("spx_matrix_values_updated", self._h, _stream(stream))

    def storage_format(self):
        """("sell", "ell", "csr5" or "dia", padding ratio) when the handle
        keeps the sliced ELLPACK, the ELLPACK, the CSR5 or the diagonal copy
        that its SpMV plans run on, else ("csr", 0.0)."""
        f = C.c_int32(0)
        r = C.c_double(0.0)
        _lib.call("spx_matrix_format", self._h, C.byref(f), C.byref(r))
        return ("csr", "sell", "ell", "csr5", "dia")[f.value], float(r.value)

    def column_order(self, stream=None):
        """The column ranking of the renumbered row-major copy (device int32
        tensor, order[r] = column of rank r), or None if there is none."""
        torch = _torch()
        flag = C.c_int32(0)
        _lib.call("spx_matrix_column_order", self._h, None, C.byref(flag), _stream(stream))
        if not flag.value:
            return None
        out = torch.empty(self.n, dtype=torch.int32, device=self.row_ptr.device)
        _lib.call("spx_matrix_column_order", self._h, _ptr(out), C.byref(flag), _stream(stream))
        return out

    def load_selector(self, path: str | None):
        _lib.call("spx_load_selector", self._h, None if path is None else path.encode())

    def run_batch(self, vec_ptr, idx, val, Y=None, total_nnz_x=None, stream=None):
        B = int(vec_ptr.numel()) - 1
        Y = self.out_tensor(B) if Y is None else Y
        tot = int(idx.numel()) if total_nnz_x is None else int(total_nnz_x)
        _lib.call("run_batch", self._h, B, tot, _ptr(vec_ptr), _ptr(idx), _ptr(val), _ptr(Y), _stream(stream))
        return Y

    def sync_values(self, vals=None, stream=None):
        """Refreshes the CSC copy if the CSR value tensor changed in place
        since the last refresh (tracked by the tensor's version counter)."""
        v = self.vals if vals is None else vals
        if v is None:
            return
        ver = v._version
        if self._vals_version != ver:
            self.values_updated(stream)
            self._vals_version = ver

    def dense_rows_to_sparse(self, X, stream=None):
        """The rows of a dense X (B x n, the matrix dtype) as CSR-of-vectors:
        (vec_ptr int32[B+1], idx, val) on the device, trimmed to vec_ptr[B]."""
        torch = _torch()
        X2 = X.reshape(-1, self.n).contiguous()
        B = int(X2.shape[0])
        vp = torch.empty(B + 1, dtype=torch.int32, device=X.device)
        idx = torch.empty(max(1, B * self.n), dtype=torch.int32, device=X.device)
        val = None if self.dtype == BOOL else torch.empty(max(1, B * self.n), dtype=X.dtype, device=X.device)
        _lib.call("spx_dense_rows_to_sparse", self._h, B, _ptr(X2), _ptr(vp), _ptr(idx), _ptr(val),
                  _stream(stream))
        k = int(vp[B].item())
        return vp, idx[:k], (val[:k] if val is not None else None)

    def run_dense_batch(self, X, Y=None, stream=None):
        """Y[b] = A X[b] for the rows of a dense X (B x n): the rows become
        sparse vectors on the device, then run_batch."""
        torch = _torch()
        B = int(X.shape[0])
        key = (B, X.dtype)
        if getattr(self, "_dense_bufs", (None,))[0] != key:
            dev = X.device
            self._dense_bufs = (key, torch.empty(B + 1, dtype=torch.int32, device=dev),
                                torch.empty(max(1, B * self.n), dtype=torch.int32, device=dev),
                                None if self.dtype == BOOL else torch.empty(max(1, B * self.n), dtype=X.dtype,
                                                                            device=dev))
        _, vp, idx, val = self._dense_bufs
        _lib.call("spx_dense_rows_to_sparse", self._h, B, _ptr(X), _ptr(vp), _ptr(idx), _ptr(val), _stream(stream))
        return self.run_batch(vp, idx, val, Y, total_nnz_x=B * self.n, stream=stream)

    def spmv_batch(self, X, Y=None, stream=None):
        """Y[b] = A X[b] for the rows of a dense X (B x n) in one pass over
        A (F32/F64)."""
        X2 = X.reshape(-1, self.n).contiguous()
        B = int(X2.shape[0])
        Y = self.out_tensor(B) if Y is None else Y
        _lib.call("spmv_csr_batch", self._h, B, _ptr(X2), _ptr(Y), _stream(stream))
        return Y

    def bfs(self, source: int, max_levels: int = 1 << 30, plan: Plan | None = None, push_only: bool = False,
            stream=None):
        """Breadth-first levels from source (BOOL handle; entry (i, j) is the
        edge j -> i): returns (level tensor int32[n], the plan of every
        expansion). A search that runs to completion makes one expansion per
        level, the last of which finds no new vertex."""
        torch = _torch()
        level = torch.empty(self.n, dtype=torch.int32, device=self.row_ptr.device)
        nl = C.c_int32(0)
        cap = 4096
        plans = (Plan * cap)()
        for i in range(cap):
            plans[i].pattern = -1  # entries the search does not reach stay -1
        # a masked-pull level comes back with lanes = -1
        _lib.call("spx_bfs", self._h, int(source), _ptr(level), int(max_levels),
                  None if plan is None else C.byref(plan), _lib.BFS_PUSH_ONLY if push_only else 0, C.byref(nl),
                  plans, cap, _stream(stream))
        self.bfs_levels = nl.value
        return level, [plans[i] for i in range(cap) if plans[i].pattern >= 0]

    def pack_mask(self, rows_mask, stream=None):
        """A bool / uint8 tensor of m entries as the bitvector (int32 words,
        bit i of word i // 32) that spmspv_sparse takes (spx_pack_mask)."""
        torch = _torch()
        rows = rows_mask.reshape(-1)
        if rows.dtype not in (torch.bool, torch.uint8):
            raise TypeError("pack_mask: rows_mask must be bool or uint8")
        if rows.numel() != self.m:
            raise ValueError(f"pack_mask: {rows.numel()} entries for {self.m} rows")
        rows = rows.contiguous()
        words = torch.empty(max(1, (self.m + 31) // 32), dtype=torch.int32, device=rows.device)
        _lib.call("spx_pack_mask", int(self.m), _ptr(rows), _ptr(words), _stream(stream))
        return words

    def spmspv_sparse(self, x, mask=None, plan: Plan | None = None, with_values: bool = True, stream=None):
        """y = A x for a sparse x as a row list: (rows, values) of the rows an
        effective entry reaches, minus those set in mask (a packed bitvector
        from pack_mask, or a bool / uint8 tensor of m entries). Rows ascend
        within each bucket of rows; buckets come in any order."""
        torch = _torch()
        v, keep = _vec(x, self.n)
        if mask is not None and mask.dtype != torch.int32:
            mask = self.pack_mask(mask)
        self.sync_values(stream=stream)
        idx = torch.empty(max(1, self.m), dtype=torch.int32, device=self.row_ptr.device)
        val = torch.empty(max(1, self.m), dtype=torch_dtype(self.dtype),
                          device=self.row_ptr.device) if with_values else None
        cnt = C.c_int32(0)
        _lib.call("spmspv_sparse", self._h, C.byref(v), _ptr(mask), None if plan is None else C.byref(plan),
                  _ptr(idx), _ptr(val), C.byref(cnt), _stream(stream))
        k = cnt.value
        return idx[:k], (val[:k] if val is not None else None)

    def pagerank(self, damping: float = 0.85, eps: float | None = None, max_iters: int = 10000,
                 plan: Plan | None = None, want_residual: bool = False, stream=None):
        """Incremental (residual-push) PageRank on an F32/F64 handle (entry
        (i, j) = edge j -> i of weight a_ij >= 0). eps defaults to
        1e-3 (1 - damping) / n. Returns (rank, plans) or, with want_residual,
        (rank, residual, plans); self.pr_iters = the number of products."""
        if eps is None:
            eps = 1e-3 * (1.0 - damping) / max(1, self.n)
        self.sync_values(stream=stream)
        rank = self.out_tensor()
        res = self.out_tensor() if want_residual else None
        ni = C.c_int32(0)
        cap = 4096
        plans = (Plan * cap)()
        for i in range(cap):
            plans[i].pattern = -1
        _lib.call("spx_pagerank", self._h, float(damping), float(eps), int(max_iters),
                  None if plan is None else C.byref(plan), _ptr(rank), None if res is None else _ptr(res),
                  C.byref(ni), plans, cap, _stream(stream))
        self.pr_iters = ni.value
        out = [plans[i] for i in range(cap) if plans[i].pattern >= 0]
        return (rank, res, out) if want_residual else (rank, out)

    def batch_status(self, stream=None) -> int:
        f = C.c_int32()
        _lib.call("spx_batch_status", self._h, C.byref(f), _stream(stream))
        return f.value

    def transpose_matvec(self, G, dX=None, stream=None):
        """dX[b] = A^T G[b]; G is B x m (or m)."""
        torch = _torch()
        G2 = G.reshape(-1, self.m).contiguous()
        B = G2.shape[0]
        out = torch.empty((B, self.n), dtype=G.dtype, device=G.device) if dX is None else dX
        _lib.call("spmv_csr_transpose", self._h, B, _ptr(G2), _ptr(out), _stream(stream))
        return out.reshape(G.shape[:-1] + (self.n,)) if dX is None else out

    def dvals(self, G, X, out=None, stream=None):
        """dvals[k] = sum_b G[b, row k] X[b, col k]; G is B x m, X is B x n dense."""
        torch = _torch()
        G2 = G.reshape(-1, self.m).contiguous()
        X2 = X.reshape(-1, self.n).contiguous()
        out = torch.empty(self.nnz, dtype=G.dtype, device=G.device) if out is None else out
        _lib.call("dvals_pattern", self._h, G2.shape[0], _ptr(G2), _ptr(X2), _ptr(out), _stream(stream))
        return out


    def backward(self, G, X=None, want_dx=True, want_dvals=True, stream=None):
        """(dX, dvals) of one backward pass from one B-minor copy of G:
        dX[b] = A^T G[b] (B x n) and dvals[k] = sum_b G[b, row k] X[b, col k];
        either may be skipped (None is returned for it)."""
        torch = _torch()
        G2 = G.reshape(-1, self.m).contiguous()
        B = int(G2.shape[0])
        dX = torch.empty((B, self.n), dtype=G.dtype, device=G.device) if want_dx else None
        dv = torch.empty(self.nnz, dtype=G.dtype, device=G.device) if want_dvals else None
        X2 = X.reshape(-1, self.n).contiguous() if want_dvals else None
        _lib.call("spx_backward", self._h, B, _ptr(G2), _ptr(X2), _ptr(dX), _ptr(dv), _stream(stream))
        return dX, dv


def _copy_raw(dst, src_ptr: int):
    """Device-to-device copy from a raw device pointer into a tensor."""
    torch = _torch()
    import ctypes
    hip = _hip_runtime()
    nbytes = dst.numel() * dst.element_size()
    torch.cuda.synchronize()
    rc = hip.hipMemcpy(C.c_void_p(dst.data_ptr()), C.c_void_p(src_ptr), C.c_size_t(nbytes), 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed: {rc}")


_HIP = None


def _hip_runtime():
    global _HIP
    if _HIP is None:
        _lib.load()
        _HIP = C.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.restype = C.c_int
        _HIP.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return _HIP


# ----------------------------------------------------------------------------
# Candidate kernels called directly (explicit plan and workspace)
# ----------------------------------------------------------------------------

def workspace_size(m, n, nnz, nnz_x_max, dtype, p: Plan) -> int:
    return int(_lib.load().spx_workspace_size(m, n, nnz, nnz_x_max, dtype, C.byref(p)))


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def spmv_csr(A: Matrix, x, p: Plan, y=None, stream=None):
    y = A.out_tensor() if y is None else y
    ws = _workspace(workspace_size(A.m, A.n, A.nnz, A.n, A.dtype, p), x.device)
    _lib.call("spmv_csr", C.byref(A._csr), _ptr(x), _ptr(y), C.byref(p), _ptr(ws), ws.numel(), _stream(stream))
    return y


def spmspv_csr(A: Matrix, idx, val, p: Plan, y=None, stream=None):
    y = A.out_tensor() if y is None else y
    ws = _workspace(workspace_size(A.m, A.n, A.nnz, int(idx.numel()), A.dtype, p), idx.device)
    _lib.call("spmspv_csr", C.byref(A._csr), int(idx.numel()), _ptr(idx), _ptr(val), _ptr(y), C.byref(p),
              _ptr(ws), ws.numel(), _stream(stream))
    return y


def spmspv_csc(A: Matrix, idx, val, p: Plan, y=None, stream=None):
    y = A.out_tensor() if y is None else y
    c = A.csc_pointers()
    ws = _workspace(workspace_size(A.m, A.n, A.nnz, int(idx.numel()), A.dtype, p), idx.device)
    _lib.call("spmspv_csc", C.byref(c), int(idx.numel()), _ptr(idx), _ptr(val), _ptr(y), C.byref(p),
              _ptr(ws), ws.numel(), _stream(stream))
    return y


def spmspv_csc_noalloc(A: Matrix, idx, val, p: Plan, y, stream=None):
    """spmspv_csc without a workspace argument: the library's fixed device
    scratch serves instead (nothing is allocated; y must be given)."""
    c = A.csc_pointers()
    _lib.call("spmspv_csc_noalloc", C.byref(c), int(idx.numel()), _ptr(idx), _ptr(val), _ptr(y), C.byref(p),
              _stream(stream))
    return y


def noalloc_capacity() -> int:
    """Bytes of the fixed device scratch behind spmspv_csc_noalloc."""
    return int(_lib.load().spmspv_csc_noalloc_capacity())


def stream_copy(src, dst, stream=None):
    """dst <- src with the library's streaming copy kernel (the achievable
    bandwidth reference); both contiguous device tensors of equal byte size,
    16-byte aligned."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _lib.call("spx_stream_copy", _ptr(src), _ptr(dst), nbytes, _stream(stream))
    return dst

