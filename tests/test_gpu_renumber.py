"""The column-renumbered copy that the row-major kernels run on (columns
ranked by descending length, entries of a row by rank): its ranking, the
default choice of when to keep it, and parity of every row-major plan on it
with the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close, cfg_matrix, reference

pytestmark = pytest.mark.gpu

KINDS = {"f32": (spx.F32, np.float32), "f64": (spx.F64, np.float64), "i32": (spx.I32, np.int32),
         "bool": (spx.BOOL, None)}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _row_major_plans():
    return [p for p in spx.all_plans() if p.pattern != spx.PAT_CSC_SPMSPV] + [
        spx.plan("spmv", "balanced", tile=4096), spx.plan("csr_spmspv", "balanced", tile=4096),
        spx.plan("csr_spmspv", "balanced", tile=2048),
        spx.plan("csr_spmspv", "balanced", tile=1), spx.plan("spmv", "direct", lanes=1),
        spx.plan("csr_spmspv", "direct", lanes=64)]


def _with_kind(A, kind):
    if kind == "i32":
        return A.with_vals(np.clip(np.round(np.asarray(A.vals) * 4), -4, 4).astype(np.int32))
    if kind in ("f32", "f64"):
        return A.with_vals(np.asarray(A.vals).astype(KINDS[kind][1]))
    return A


def _check(M, A, kind, nnz_x, seed, dense):
    torch = _torch()
    code, npdt = KINDS[kind]
    v = synth.sparse_vector(A.n, nnz_x, seed)
    val = None
    if kind == "i32":
        val = np.random.default_rng(seed).integers(-5, 6, size=v.nnz).astype(np.int32)
    elif kind != "bool":
        val = np.asarray(v.val).astype(npdt)
    ref, S = reference(A, v.idx, val, kind)
    if dense:
        xd = np.zeros(A.n, dtype=npdt if npdt is not None else np.uint8)
        xd[v.idx] = val if kind != "bool" else 1
        x = torch.as_tensor(xd, device="cuda")
    else:
        x = (torch.as_tensor(v.idx, device="cuda"),
             None if kind == "bool" else torch.as_tensor(val, device="cuda"))
    for p in _row_major_plans():
        y = M.run_plan(x, p)
        torch.cuda.synchronize()
        assert_close(y.cpu().numpy(), ref, S, kind, f"{kind} nnz_x={nnz_x} dense={dense} {p}")


def test_column_order_is_the_stable_length_ranking():
    _torch()
    A = cfg_matrix("rmat16")
    M = spx.Matrix.from_host(A, renumber=True, fmt="csr")
    order = M.column_order()
    assert order is not None
    lens = np.diff(oracle.transpose(A, with_values=False).col_ptr)
    want = np.argsort(-lens, kind="stable")
    assert np.array_equal(order.cpu().numpy(), want)
    assert spx.Matrix.from_host(A, renumber=False).column_order() is None


def test_default_choice():
    """Kept for the skewed R-MAT column lengths, not for the 7-point stencil
    (uniform lengths, natural order already local) nor for small n."""
    _torch()
    assert spx.Matrix.from_host(cfg_matrix("cfg2")).column_order() is not None
    assert spx.Matrix.from_host(cfg_matrix("cfg3")).column_order() is None
    assert spx.Matrix.from_host(cfg_matrix("cfg1")).column_order() is None  # n < 65536


@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
def test_renumbered_plans_match_oracle(kind):
    _torch()
    A = _with_kind(cfg_matrix("rmat16"), kind)
    M = spx.Matrix.from_host(A, dtype=KINDS[kind][0], renumber=True, fmt="csr")
    for nnz_x in (0, 1, 300, A.n // 8, A.n):
        _check(M, A, kind, nnz_x, 40 + nnz_x, dense=False)
    for nnz_x in (1, A.n // 3):
        _check(M, A, kind, nnz_x, 50 + nnz_x, dense=True)


@pytest.mark.parametrize("kind", ["f32", "bool"])
def test_renumbered_ragged(kind):
    """Forced on small and ragged shapes: empty rows, empty columns, n not
    a multiple of 32 or 64, a single column."""
    _torch()
    for ci, (m, n, dens) in enumerate([(37, 53, 0.1), (3001, 2503, 0.004), (700, 9000, 0.002), (2, 1, 1.0)]):
        A = _with_kind(synth.random_csr(m, n, dens, 300 + ci, empty_rows=0.2), kind)
        M = spx.Matrix.from_host(A, dtype=KINDS[kind][0], renumber=True, fmt="csr")
        for nnz_x in sorted({1, max(1, n // 7), n}):
            _check(M, A, kind, nnz_x, 60 + ci, dense=False)
            _check(M, A, kind, nnz_x, 70 + ci, dense=True)


def test_renumbered_copy_follows_values_updated():
    torch = _torch()
    A = cfg_matrix("rmat16")
    M = spx.Matrix.from_host(A, renumber=True, fmt="csr")
    new = np.random.default_rng(8).uniform(-2, 2, A.nnz).astype(np.float32)
    M.vals.copy_(torch.as_tensor(new, device="cuda"))
    M.values_updated()
    B = A.with_vals(new)
    x = synth.dense_vector(A.n, 9)
    ref, S = oracle.spmv(B, x.astype(np.float64))
    for p in [spx.plan("spmv", "balanced"), spx.plan("spmv", "direct")]:
        y = M.run_plan(torch.as_tensor(x, device="cuda"), p)
        torch.cuda.synchronize()
        assert_close(y.cpu().numpy(), ref, S, "f32", f"after update {p}")
