"""Conversion buffers carried between calls on one handle.

A balanced row-major product clears, in its fix-up pass, the bitvector
words and dense-x entries that its sparse x was scattered to, and the next
sparse conversion then skips its fill. Every call of a mixed sequence on one
handle (sparse and dense x; balanced, direct and LDS-bitvector row-major
plans; column-major plans; supports growing, shrinking, empty) is checked
against the oracle, so a buffer left dirty shows up as stray entries of x in
a later product."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close, cfg_matrix, reference

pytestmark = pytest.mark.gpu

KINDS = {"f32": (spx.F32, np.float32), "f64": (spx.F64, np.float64), "i32": (spx.I32, np.int32),
         "bool": (spx.BOOL, None)}

PLANS = [
    spx.plan("spmv", "balanced"),
    spx.plan("csr_spmspv", "balanced"),
    spx.plan("spmv", "balanced", tile=4096),
    spx.plan("spmv", "direct"),
    spx.plan("csr_spmspv", "balanced", tile=1),
    spx.plan("csr_spmspv", "direct"),
    spx.plan("csc_spmspv", "balanced", "atomic"),
    spx.plan("csr_spmspv", "balanced", tile=4096),
]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _with_kind(A, kind):
    if kind == "i32":
        return A.with_vals(np.clip(np.round(np.asarray(A.vals) * 4), -4, 4).astype(np.int32))
    if kind in ("f32", "f64"):
        return A.with_vals(np.asarray(A.vals).astype(KINDS[kind][1]))
    return A


@pytest.mark.parametrize("renumber", [True, False])
@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
def test_mixed_call_sequence(kind, renumber):
    torch = _torch()
    code, npdt = KINDS[kind]
    A = _with_kind(cfg_matrix("rmat16"), kind)
    M = spx.Matrix.from_host(A, dtype=code, renumber=renumber, fmt="csr")
    rng = np.random.default_rng(17)
    sizes = [A.n // 8, 5, A.n // 2, 1, 0, 300, -(A.n // 3), A.n // 8, 2, -7, A.n]
    for i in range(3 * len(PLANS)):
        p = PLANS[i % len(PLANS)]
        nnz = sizes[(5 * i) % len(sizes)]
        dense = nnz < 0
        v = synth.sparse_vector(A.n, abs(nnz), 500 + i)
        val = None
        if kind == "i32":
            val = rng.integers(-5, 6, size=v.nnz).astype(np.int32)
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
        y = M.run_plan(x, p)
        torch.cuda.synchronize()
        assert_close(y.cpu().numpy(), ref, S, kind, f"call {i}: {p} nnz_x={nnz} renumber={renumber}")


def test_minplus_sequence_keeps_infinity():
    """Min-plus: the cleared dense-x entries go back to +inf, not 0 (a 0
    left behind would lower every row that holds that column)."""
    torch = _torch()
    A = cfg_matrix("rmat16")
    A = A.with_vals(np.asarray(A.vals, np.float32))
    M = spx.Matrix.from_host(A, dtype=spx.F32_MINPLUS, renumber=True, fmt="csr")
    plans = [spx.plan("spmv", "balanced"), spx.plan("csr_spmspv", "balanced"), spx.plan("spmv", "direct")]
    for i, nnz in enumerate([A.n // 4, 3, A.n // 2, 0, 40, A.n // 16, 1]):
        v = synth.sparse_vector(A.n, nnz, 700 + i)
        xv = np.asarray(v.val, np.float32)
        for p in plans:
            y = M.run_plan((torch.as_tensor(v.idx, device="cuda"), torch.as_tensor(xv, device="cuda")), p)
            torch.cuda.synchronize()
            got = y.cpu().numpy()
            want = oracle.minplus_spmspv(A, v.idx, xv)
            bad = np.nonzero(~((got == want) | (np.isnan(got) & np.isnan(want))))[0]
            assert bad.size == 0, f"call {i} {p} nnz_x={nnz}: {bad.size} rows differ, first {bad[:5]}"
