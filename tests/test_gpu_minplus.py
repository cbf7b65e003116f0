"""Min-plus semiring (SPX_F32_MINPLUS) against the oracle, bit-exact: every
sum a_ij + x_j is one float32 addition on both sides and the minimum is
exact, so the order of the reduction cannot change a bit."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import cfg_matrix

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _f32(A):
    return A.with_vals(np.asarray(A.vals, np.float32))


def _same(got, want, what):
    got = got.cpu().numpy()
    bad = np.nonzero(~((got == want) | (np.isnan(got) & np.isnan(want))))[0]
    assert bad.size == 0, f"{what}: {bad.size} rows differ, first {bad[:5]}: {got[bad[:5]]} vs {want[bad[:5]]}"


@pytest.mark.parametrize("name", ["cfg1", "rmat16"])
def test_minplus_every_plan_dense_and_sparse(name):
    torch = _torch()
    A = _f32(cfg_matrix(name))
    M = spx.Matrix.from_host(A, dtype=spx.F32_MINPLUS)
    y = M.out_tensor()
    rng = np.random.default_rng(21)
    xd = rng.uniform(-1, 1, A.n).astype(np.float32)
    xd[rng.random(A.n) < 0.4] = np.inf
    want_d = oracle.minplus_spmv(A, xd)
    sparse = []
    for nnz in (1, 10, 300, 3000):
        v = synth.sparse_vector(A.n, nnz, 300 + nnz)
        sparse.append((v.idx, np.asarray(v.val, np.float32)))
    for p in spx.all_plans():
        for k, (xi, xv) in enumerate([(None, None)] + sparse):
            x = torch.as_tensor(xd, device="cuda") if xi is None else (torch.as_tensor(xi, device="cuda"),
                                                                        torch.as_tensor(xv, device="cuda"))
            try:
                M.run_plan(x, p, y)
            except spx.SpxError as e:
                if e.code == -5:
                    continue  # the write-back does not fit this matrix (LDS)
                raise
            want = want_d if xi is None else oracle.minplus_spmspv(A, xi, xv)
            _same(y, want, f"{name} {p} x{k}")
    # adaptive
    for xi, xv in sparse:
        M.run((torch.as_tensor(xi, device="cuda"), torch.as_tensor(xv, device="cuda")), y)
        _same(y, oracle.minplus_spmspv(A, xi, xv), f"{name} run()")


def test_minplus_bellman_ford_is_dijkstra():
    """Repeated relaxation d = min(d, A (x) d) on the GPU (run() picks the
    kernel per round as the frontier of changed distances grows and shrinks)
    reaches scipy's Dijkstra distances exactly (integer weights)."""
    torch = _torch()
    from scipy.sparse.csgraph import dijkstra
    A = synth.rmat(12, 8, 5)
    w = np.random.default_rng(2).integers(1, 16, A.nnz).astype(np.float32)
    A = A.with_vals(w)
    M = spx.Matrix.from_host(A, dtype=spx.F32_MINPLUS)
    G = sp.csr_matrix((w.astype(np.float64), A.col_idx, A.row_ptr), shape=(A.m, A.n)).T.tocsr()
    outdeg = np.bincount(A.col_idx, minlength=A.n)
    s0 = int(np.nonzero(outdeg > 0)[0][0])
    d = torch.full((A.n,), float("inf"), device="cuda")
    d[s0] = 0.0
    frontier = torch.tensor([s0], dtype=torch.int32, device="cuda")
    y = M.out_tensor()
    for _ in range(A.n):
        M.run((frontier, d[frontier.long()].contiguous()), y)
        better = y < d
        if not bool(better.any()):
            break
        d = torch.where(better, y, d)
        frontier = torch.nonzero(better).flatten().to(torch.int32)
    want = dijkstra(G, directed=True, indices=s0)
    assert np.array_equal(d.cpu().numpy().astype(np.float64), want)


def test_minplus_sparse_output_and_refusals():
    torch = _torch()
    A = _f32(cfg_matrix("rmat16"))
    M = spx.Matrix.from_host(A, dtype=spx.F32_MINPLUS)
    v = synth.sparse_vector(A.n, 500, 9)
    x = (torch.as_tensor(v.idx, device="cuda"), torch.as_tensor(np.asarray(v.val, np.float32), device="cuda"))
    rows, vals = M.spmspv_sparse(x)
    order = torch.argsort(rows)
    want_rows = np.nonzero(oracle.bool_spmspv(A, v.idx))[0]
    assert np.array_equal(rows[order].cpu().numpy(), want_rows)
    want = oracle.minplus_spmspv(A, v.idx, np.asarray(v.val, np.float32))[want_rows]
    assert np.array_equal(vals[order].cpu().numpy(), want)
    # an empty x reaches nothing: every row is +inf
    y = M.run((torch.zeros(0, dtype=torch.int32, device="cuda"), torch.zeros(0, device="cuda")))
    assert bool(torch.isinf(y).all())
    with pytest.raises(spx.SpxError) as e:
        M.run_batch(torch.tensor([0, 1], dtype=torch.int32, device="cuda"), x[0][:1], x[1][:1])
    assert e.value.code == -4
