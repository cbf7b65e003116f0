"""Accumulation length: a hub row and a hub column of 2^19 entries.

One serial FP32 chain over 2^19 positive products misses the bound
|y_i - ref_i| <= 1e-5 * sum_j |a_ij x_j| (the CPU test below shows it on
the very inputs of the GPU tests), so every kernel that sums a row (or a
column, for dX = A^T g) must split it into bounded partial sums. The
write-backs that add one product at a time into y (atomic, LDS-atomic,
bucket) are one chain per row by construction; run() does not pick them in
FP32 for a matrix whose longest row exceeds 2^16 entries, and they are not
part of this check.
"""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close

N = (1 << 19) + 8192
HUB = 1 << 19


def _inputs():
    A = synth.hub_matrix(N, HUB, 4, 31)
    x = np.random.default_rng(32).uniform(0.0, 1.0, A.n).astype(np.float32)
    return A, x


def test_serial_chain_misses_the_bound():
    """The products of the hub row summed one after another in FP32 miss
    the bound that the GPU kernels must meet (so the GPU tests can fail)."""
    A, x = _inputs()
    ref, S = oracle.spmv(A, x.astype(np.float64))
    k1 = int(A.row_ptr[1])
    prod = A.vals[:k1].astype(np.float64) * x[A.col_idx[:k1]].astype(np.float64)
    serial = np.add.accumulate(prod.astype(np.float32), dtype=np.float32)[-1]
    assert abs(float(serial) - ref[0]) > 1e-5 * S[0]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _row_major_plans():
    out = [spx.plan("spmv", "balanced"), spx.plan("csr_spmspv", "balanced")]
    for L in (0, 1, 4, 32, 64):
        out.append(spx.plan("spmv", "direct", lanes=L))
        out.append(spx.plan("csr_spmspv", "direct", lanes=L))
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("renumber", [False, True])
def test_hub_row_row_major_and_tree_write_backs(renumber):
    torch = _torch()
    A, x = _inputs()
    ref, S = oracle.spmv(A, x.astype(np.float64))
    M = spx.Matrix.from_host(A, renumber=renumber, fmt="csr")
    xd = torch.as_tensor(x, device="cuda")
    idx = torch.arange(A.n, dtype=torch.int32, device="cuda")
    for p in _row_major_plans():
        y = M.run_plan(xd, p).cpu().numpy()
        assert_close(y, ref, S, "f32", f"dense x {p}")
    for p in _row_major_plans() + [spx.plan("csc_spmspv", d, "sort") for d in ("direct", "balanced")]:
        y = M.run_plan((idx, xd), p).cpu().numpy()
        assert_close(y, ref, S, "f32", f"sparse x {p}")
    for xin in (xd, (idx, xd)):
        y = M.run(xin).cpu().numpy()
        assert_close(y, ref, S, "f32", f"run() {M.last_plan()}")


@pytest.mark.gpu
def test_hub_row_and_column_batched_and_backward():
    """The fused batch forward (a wave per row) and dX = G A (a wave per
    column) over the hub row and the hub column; run_batch with dense-enough
    vectors (fused groups split the hub row into pieces)."""
    torch = _torch()
    A, _ = _inputs()
    M = spx.Matrix.from_host(A)
    rng = np.random.default_rng(33)
    B = 3
    X = rng.uniform(0.0, 1.0, (B, A.n)).astype(np.float32)
    G = rng.uniform(0.0, 1.0, (B, A.m)).astype(np.float32)
    Y = M.spmv_batch(torch.as_tensor(X, device="cuda")).cpu().numpy()
    for b in range(B):
        ref, S = oracle.spmv(A, X[b].astype(np.float64))
        assert_close(Y[b], ref, S, "f32", f"fused batch forward b={b}")
    dX = M.transpose_matvec(torch.as_tensor(G, device="cuda")).cpu().numpy()
    dX_ref, sdX, _ = oracle.grad(A, G, np.zeros((B, A.n)), want_dvals=False)
    for b in range(B):
        assert_close(dX[b], dX_ref[b], sdX[b], "f32", f"dX b={b}")
    vecs = [synth.sparse_vector(A.n, int(A.n * d), 400 + i, "uniform", np.float64)
            for i, d in enumerate((1.0, 0.5, 0.05))]
    vecs = [synth.SparseVec(v.n, v.idx, np.abs(v.val).astype(np.float32)) for v in vecs]
    ptr = torch.as_tensor(np.concatenate([[0], np.cumsum([v.nnz for v in vecs])]).astype(np.int32), device="cuda")
    idx = torch.as_tensor(np.concatenate([v.idx for v in vecs]), device="cuda")
    val = torch.as_tensor(np.concatenate([v.val for v in vecs]), device="cuda")
    Yb = M.run_batch(ptr, idx, val).cpu().numpy()
    assert M.batch_status() == 0
    for b, v in enumerate(vecs):
        xd = np.zeros(A.n)
        xd[v.idx] = v.val
        ref, S = oracle.spmv(A, xd)
        assert_close(Yb[b], ref, S, "f32", f"run_batch b={b} nnz_x={v.nnz}")
