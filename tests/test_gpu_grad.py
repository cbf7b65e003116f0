"""Backward of the sparse layer: central differences in FP64 (the loss is
bilinear in (vals, X), so they are exact up to rounding), the oracle's
gradient, torch.autograd.gradcheck, and the pruned FC layer at full size."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _relu_batch(n, B, seed, dtype):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, n))
    X[rng.random((B, n)) < 0.6] = 0.0
    return np.abs(X).astype(dtype)


@pytest.mark.parametrize("mode", ["fused", "sparse"])
def test_fd_exact_fp64_and_oracle(mode):
    torch = _torch()
    from paper_2006_16767_amd.autograd import sparse_linear
    A = synth.bernoulli(64, 32, 0.05, 12, std=1.0, dtype=np.float64)
    M = spx.Matrix.from_host(A)
    vals = M.vals.requires_grad_(True)
    X = torch.as_tensor(_relu_batch(32, 3, 1, np.float64), device="cuda").requires_grad_(True)
    G = torch.as_tensor(np.random.default_rng(2).standard_normal((3, 64)), device="cuda")
    Y = sparse_linear(M, X, vals, mode)
    (Y * G).sum().backward()
    dvals = vals.grad.detach().cpu().numpy()
    dX = X.grad.detach().cpu().numpy()
    # oracle gradient
    dX_ref, _, dv_ref = oracle.grad(A, G.cpu().numpy(), X.detach().cpu().numpy())
    assert np.allclose(dX, dX_ref, rtol=1e-12, atol=1e-14)
    assert np.allclose(dvals, dv_ref, rtol=1e-12, atol=1e-14)
    # central differences of the GPU forward, h = 2^-10
    h = 2.0 ** -10
    with torch.no_grad():
        def L():
            return float((sparse_linear(M, X.detach(), vals, mode) * G).sum())
        for k in range(A.nnz):
            vals[k] += h
            lp = L()
            vals[k] -= 2 * h
            lm = L()
            vals[k] += h
            fd = (lp - lm) / (2 * h)
            assert abs(fd - dvals[k]) <= 1e-9 * max(1.0, abs(dvals[k]))
        Xd = X.detach().clone()
        for b in range(3):
            for j in range(32):
                Xp = Xd.clone(); Xp[b, j] += h
                Xm = Xd.clone(); Xm[b, j] -= h
                fd = (float((sparse_linear(M, Xp, vals, mode) * G).sum()) -
                      float((sparse_linear(M, Xm, vals, mode) * G).sum())) / (2 * h)
                assert abs(fd - dX[b, j]) <= 1e-9 * max(1.0, abs(dX[b, j]))


def test_gradcheck_small():
    torch = _torch()
    from paper_2006_16767_amd.autograd import SparseLinearFunction
    A = synth.bernoulli(20, 12, 0.3, 3, std=1.0, dtype=np.float64)
    M = spx.Matrix.from_host(A)
    vals = M.vals.requires_grad_(True)
    X = torch.as_tensor(_relu_batch(12, 2, 4, np.float64) + 0.1, device="cuda").requires_grad_(True)
    assert torch.autograd.gradcheck(lambda v, x: SparseLinearFunction.apply(v, x, M), (vals, X),
                                    eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("mode", ["fused", "sparse"])
def test_values_refresh_after_inplace_update(mode):
    torch = _torch()
    from paper_2006_16767_amd.autograd import sparse_linear
    A = synth.bernoulli(200, 100, 0.1, 5, dtype=np.float32)
    M = spx.Matrix.from_host(A)
    X = torch.as_tensor(_relu_batch(100, 4, 6, np.float32), device="cuda")
    with torch.no_grad():
        Y1 = sparse_linear(M, X, mode=mode).clone()
        M.vals.mul_(2.0)  # an optimizer-style in-place update
        Y2 = sparse_linear(M, X, mode=mode)
    torch.cuda.synchronize()
    # the forward may pick column-major plans, which read the CSC copy
    assert torch.allclose(Y2, 2.0 * Y1, rtol=1e-6, atol=1e-6)


@pytest.mark.slow
def test_pruned_fc_layer_full_size():
    """16384 x 4096 at 5% density, batch 64 with 50..95% zeros: forward,
    dX and dvals against the oracle in FP32."""
    torch = _torch()
    from paper_2006_16767_amd.autograd import sparse_linear
    A = synth.cfg5_matrix()
    M = spx.Matrix.from_host(A)
    acts = synth.cfg5_activations()
    Xh = np.zeros((64, A.n), np.float32)
    for b, v in enumerate(acts):
        Xh[b, v.idx] = v.val
    Gh = synth.cfg5_upstream()
    vals = M.vals.requires_grad_(True)
    X = torch.as_tensor(Xh, device="cuda").requires_grad_(True)
    G = torch.as_tensor(Gh, device="cuda")
    Y = sparse_linear(M, X, vals)
    (Y * G).sum().backward()
    with torch.no_grad():
        Ys = sparse_linear(M, X.detach(), mode="sparse")
    torch.cuda.synchronize()
    Yh = Y.detach().cpu().numpy()
    Ysh = Ys.cpu().numpy()
    for b in range(64):
        ref, S = oracle.spmv(A, Xh[b])
        assert_close(Yh[b], ref, S, "f32", f"fc forward (fused) b={b}")
        assert_close(Ysh[b], ref, S, "f32", f"fc forward (sparse) b={b}")
    dX_ref, sdX, dv_ref = oracle.grad(A, Gh, Xh)
    dX = X.grad.cpu().numpy()
    for b in range(64):
        assert_close(dX[b], dX_ref[b], sdX[b], "f32", f"fc dX b={b}")
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    sdv = (np.abs(Gh[:, rows].astype(np.float64)) * np.abs(Xh[:, A.col_idx].astype(np.float64))).sum(0)
    assert_close(vals.grad.cpu().numpy(), dv_ref, sdv, "f32", "fc dvals")


@pytest.mark.parametrize("kind", ["f32", "f64"])
def test_fused_batch_spmv_matches_oracle(kind):
    """spmv_csr_batch on ragged shapes: empty rows, rows shorter and longer
    than the 8-entry unroll, B = 1, below, at and above 64 (chunks of 64)."""
    torch = _torch()
    npdt = np.float32 if kind == "f32" else np.float64
    for ci, (m, n, dens) in enumerate([(37, 53, 0.1), (3001, 2503, 0.004), (700, 900, 0.05), (2, 1, 1.0)]):
        A = synth.random_csr(m, n, dens, 500 + ci, empty_rows=0.2)
        A = A.with_vals(np.asarray(A.vals).astype(npdt))
        M = spx.Matrix.from_host(A)
        for B in (1, 3, 64, 70, 130):
            X = _relu_batch(n, B, 10 * ci + B, npdt)
            Y = M.spmv_batch(torch.as_tensor(X, device="cuda")).cpu().numpy()
            for b in range(B):
                ref, S = oracle.spmv(A, X[b].astype(np.float64))
                assert_close(Y[b], ref, S, kind, f"{m}x{n} B={B} b={b}")


@pytest.mark.parametrize("B", [1, 7, 64, 130])
def test_fused_backward_matches_separate_calls_and_oracle(B):
    """spx_backward (one B-minor copy of G for both gradients) gives the same
    bits as spmv_csr_transpose and dvals_pattern called apart, matches the
    oracle's gradient, and skips either gradient on request; B past 64 runs
    the gather in chunks of 64 batch rows, with a ragged last chunk."""
    torch = _torch()
    A = synth.bernoulli(700, 301, 0.04, 31, std=1.0, dtype=np.float32)
    M = spx.Matrix.from_host(A)
    rng = np.random.default_rng(B)
    G = torch.as_tensor(rng.standard_normal((B, A.m)).astype(np.float32), device="cuda")
    X = torch.as_tensor(_relu_batch(A.n, B, B + 1, np.float32), device="cuda")
    dX, dv = M.backward(G, X)
    dX2 = M.transpose_matvec(G)
    dv2 = M.dvals(G, X)
    only_dx, none_dv = M.backward(G, want_dvals=False)
    none_dx, only_dv = M.backward(G, X, want_dx=False)
    torch.cuda.synchronize()
    assert none_dv is None and none_dx is None
    for a, b in ((dX, dX2), (dv, dv2), (dX, only_dx), (dv, only_dv)):
        assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))
    dX_ref, S_dx, dv_ref = oracle.grad(A, G.cpu().numpy(), X.cpu().numpy())
    got = dX.cpu().numpy()
    for b in range(B):
        assert_close(got[b], dX_ref[b], S_dx[b], "f32", f"dX row {b}")
    # dvals: B products per entry, each bounded by |g| |x|
    S_dv = oracle.grad(A.with_vals(np.ones(A.nnz)), np.abs(G.cpu().numpy()), np.abs(X.cpu().numpy()),
                       want_dx=False)[2]
    assert_close(dv.cpu().numpy(), dv_ref, S_dv, "f32", "dvals")
