"""Incremental PageRank driver (one adaptive SpMSpV per round) against the
oracle's residual-push loop. In FP64 the rounds take the same threshold
decisions as the oracle (a residual would have to land within rounding of
eps to flip one), so the product count must match and rank and residual
agree to rounding. In FP32 the two trajectories may part at a threshold;
both then still satisfy the residual identity, which bounds their
distance by the residual norms."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import cfg_matrix

pytestmark = pytest.mark.gpu

D = 0.85


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _f64(A):
    return A.with_vals(np.asarray(A.vals, np.float64))


def _close64(got, want, what):
    got = got.cpu().numpy()
    scale = np.abs(want).max() if want.size else 1.0
    err = np.abs(got - want).max() if want.size else 0.0
    assert err <= 1e-11 * scale, f"{what}: max error {err:.3e} against scale {scale:.3e}"


@pytest.mark.parametrize("tol", [1e-2, 1e-3])
def test_pagerank_fp64_matches_oracle(tol):
    _torch()
    A = _f64(cfg_matrix("rmat16"))
    M = spx.Matrix.from_host(A)
    eps = tol * (1 - D) / A.n
    rank, res, plans = M.pagerank(D, eps, want_residual=True)
    p, r, k = oracle.pagerank_incremental(A, D, eps, 10 ** 6)
    assert M.pr_iters == k and len(plans) == k
    _close64(rank, p, "rank")
    _close64(res, r, "residual")
    # the input density falls from about half the vertices to a handful,
    # so more than one pattern serves the rounds
    assert len({q.pattern for q in plans}) >= 2


@pytest.mark.parametrize("k", [0, 1, 3])
def test_pagerank_product_limit_folds_the_last_product(k):
    _torch()
    A = _f64(cfg_matrix("rmat16"))
    M = spx.Matrix.from_host(A)
    eps = 1e-3 * (1 - D) / A.n
    rank, res, plans = M.pagerank(D, eps, max_iters=k, want_residual=True)
    p, r, kk = oracle.pagerank_incremental(A, D, eps, k)
    assert M.pr_iters == kk == k
    _close64(rank, p, "rank")
    _close64(res, r, "residual")


def test_pagerank_every_fixed_plan_fp64():
    _torch()
    A = _f64(cfg_matrix("rmat16"))
    M = spx.Matrix.from_host(A)
    eps = 1e-2 * (1 - D) / A.n
    p, r, k = oracle.pagerank_incremental(A, D, eps, 10 ** 6)
    for plan in spx.all_plans():
        try:
            rank, plans = M.pagerank(D, eps, plan=plan)
        except spx.SpxError as e:
            if e.code == -5:
                continue  # the write-back does not fit this matrix (LDS)
            raise
        assert M.pr_iters == k, plan
        _close64(rank, p, f"rank under {plan}")


def test_pagerank_fp32_full_size():
    """R-MAT 2^20 (degree 16, weights U[0, 1]) in FP32: the GPU residual is
    below eps everywhere, and rank is within the residual bound of the
    oracle's: |p_gpu - p_ref|_1 <= (|r_gpu|_1 + |r_ref|_1) / (1 - d) plus
    FP32 rounding of the rank itself."""
    _torch()
    A = cfg_matrix("cfg2")
    M = spx.Matrix.from_host(A)
    eps = 1e-3 * (1 - D) / A.n
    rank, res, plans = M.pagerank(D, eps, want_residual=True)
    p, r, k = oracle.pagerank_incremental(_f64(A), D, eps, 10 ** 6)
    rg = res.cpu().numpy().astype(np.float64)
    pg = rank.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(rg) <= np.float32(eps))
    bound = (np.abs(rg).sum() + np.abs(r).sum()) / (1 - D) + 1e-5 * np.abs(p).sum()
    assert np.abs(pg - p).sum() <= bound
    assert abs(M.pr_iters - k) <= 3
    assert len({(q.pattern, q.distribution, q.writeback) for q in plans}) >= 2


def test_pagerank_edge_cases():
    torch = _torch()
    n = 6
    # no edges: every vertex dangling, one round moves r0 into p
    E = synth._coo_to_csr(n, n, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.float32))
    M = spx.Matrix.from_host(E)
    rank, res, plans = M.pagerank(D, 0.0, want_residual=True)
    assert M.pr_iters == 0 and plans == []
    assert np.allclose(rank.cpu().numpy(), (1 - D) / n, rtol=1e-7) and np.all(res.cpu().numpy() == 0)
    # one edge 0 -> 1 (vertex 1 dangling): p = (1-d)/2 * [1, 1 + d]
    A = synth._coo_to_csr(2, 2, np.array([1]), np.array([0]), np.array([0.5]))
    A = _f64(A)
    M = spx.Matrix.from_host(A)
    rank, _ = M.pagerank(D, 0.0)
    assert M.pr_iters == 1
    assert np.allclose(rank.cpu().numpy(), [(1 - D) / 2, (1 - D) / 2 * (1 + D)], rtol=1e-15)
    # negative weight, then fixed in place
    B = synth.random_csr(50, 50, 0.1, 3)
    B = B.with_vals(np.asarray(B.vals, np.float32))
    MB = spx.Matrix.from_host(B)
    if (np.asarray(B.vals) < 0).any():
        with pytest.raises(spx.SpxError) as e:
            MB.pagerank(D)
        assert e.value.code == -1
    with torch.no_grad():
        MB.vals.abs_()
    rank, _ = MB.pagerank(D, 0.0, max_iters=500)
    want, _, _ = oracle.pagerank_incremental(B.with_vals(np.abs(np.asarray(B.vals, np.float64))), D, 0.0, 500)
    assert np.allclose(rank.cpu().numpy(), want, rtol=1e-5, atol=1e-9)
    for bad in (1.0, -0.1, float("nan")):
        with pytest.raises(spx.SpxError) as e:
            MB.pagerank(bad)
        assert e.value.code == -1
    with pytest.raises(spx.SpxError) as e:
        spx.Matrix.from_host(B, dtype=spx.BOOL).pagerank(D)
    assert e.value.code == -4
    with pytest.raises(spx.SpxError) as e:
        spx.Matrix.from_host(synth.random_csr(8, 9, 0.3, 1)).pagerank(D)
    assert e.value.code == -2
