"""Pins for the CPU oracle: checks against things other than the oracle
itself (hand-worked values, dense brute force, scipy, closed forms,
invariants, finite differences, an edge-list BFS step), plus planted
mistakes showing that each pin would catch a plausible oracle bug.

CPU only."""
import itertools
import json
import math
import os
from types import SimpleNamespace

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2006_16767_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLD, "tiny_worked.json")) as f:
        return json.load(f)


def _mat(m, n, row_ptr, col_idx, vals):
    return SimpleNamespace(m=m, n=n, row_ptr=np.asarray(row_ptr, np.int32),
                           col_idx=np.asarray(col_idx, np.int32),
                           vals=None if vals is None else np.asarray(vals))


def _dense(A, dtype=np.float64):
    D = np.zeros((A.m, A.n), dtype=dtype)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    D[rows, A.col_idx] = A.vals if A.vals is not None else 1
    return D


# ---------------------------------------------------------------- golden

def test_golden_spmv_spmspv():
    g = _golden()
    A = _mat(g["m"], g["n"], g["row_ptr"], g["col_idx"], g["vals"])
    y, s = oracle.spmv(A, g["x_dense"])
    assert y.tolist() == g["y_dense"]
    assert s.tolist() == g["s_dense"]
    csc = oracle.transpose(A)
    y2, _ = oracle.spmspv(csc, g["x_sparse_idx"], g["x_sparse_val"])
    assert y2.tolist() == g["y_sparse"]


def test_golden_bool_int():
    g = _golden()
    A = _mat(g["m"], g["n"], g["row_ptr"], g["col_idx"], None)
    for case in g["bool_cases"]:
        assert oracle.bool_spmspv(A, case["x_idx"]).tolist() == case["y"]
    Ai = _mat(g["m"], g["n"], g["row_ptr"], g["col_idx"], np.array(g["int_vals"], np.int32))
    assert oracle.int_spmv(Ai, g["int_x"]).tolist() == g["int_y"]
    w = g["int_wrap"]
    Aw = _mat(w["m"], w["n"], w["row_ptr"], w["col_idx"], np.array(w["vals"], np.int32))
    assert oracle.int_spmv(Aw, w["x"]).tolist() == w["y"]
    cscw = oracle.transpose(Aw, int_values=True)
    assert oracle.int_spmspv(cscw, [0, 1], w["x"]).tolist() == w["y"]


def test_golden_features_and_grad():
    g = _golden()
    A = _mat(g["m"], g["n"], g["row_ptr"], g["col_idx"], g["vals"])
    f = oracle.matrix_features(A)
    for k, v in g["features"].items():
        assert f[k] == pytest.approx(v, rel=1e-15, abs=0), k
    csc = oracle.transpose(A)
    vf = oracle.vector_features(csc, g["vector_features_idx"])
    for k, v in g["vector_features"].items():
        assert vf[k] == pytest.approx(v, rel=1e-15, abs=0), k
    dX, _, dv = oracle.grad(A, [g["g"]], [g["x_dense"]])
    assert dX[0].tolist() == g["dx"]
    assert dv.tolist() == g["dvals"]


# ------------------------------------------------------------ brute force

def _check_spmv_brute(spmv_fn, A, x):
    y, s = spmv_fn(A, x)
    D = _dense(A)
    ref = D @ np.asarray(x, np.float64)
    sref = np.abs(D) @ np.abs(np.asarray(x, np.float64))
    return np.allclose(y, ref, rtol=1e-13, atol=1e-13) and np.allclose(s, sref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("seed", range(6))
def test_spmv_dense_brute(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(1, 65)), int(rng.integers(1, 65))
    A = synth.random_csr(m, n, float(rng.uniform(0.02, 0.5)), seed, dtype=np.float32,
                         empty_rows=0.2)
    x = rng.uniform(-1, 1, n).astype(np.float32)
    assert _check_spmv_brute(oracle.spmv, A, x)


@pytest.mark.parametrize("seed", range(6))
def test_spmspv_dense_brute(seed):
    rng = np.random.default_rng(100 + seed)
    m, n = int(rng.integers(1, 65)), int(rng.integers(1, 65))
    A = synth.random_csr(m, n, float(rng.uniform(0.02, 0.5)), seed, empty_rows=0.2)
    csc = oracle.transpose(A)
    D = _dense(A)
    for nnz_x in sorted({0, 1, n // 3, n}):
        v = synth.sparse_vector(n, nnz_x, seed * 7 + nnz_x)
        y, s = oracle.spmspv(csc, v.idx, v.val)
        xh = v.dense(np.float64)
        assert np.allclose(y, D @ xh, rtol=1e-13, atol=1e-13)
        assert np.allclose(s, np.abs(D) @ np.abs(xh), rtol=1e-13, atol=0)
        # rows with no effective entry are exactly +0
        empty = (np.abs(D) @ (xh != 0)) == 0
        assert np.all(y[empty] == 0) and not np.any(np.signbit(y[empty]))


def test_spmspv_exhaustive_supports():
    """Every support of x for n = 10: SpMSpV equals the dense product with
    the zero-filled vector."""
    A = synth.random_csr(9, 10, 0.35, 7, empty_rows=0.1)
    csc = oracle.transpose(A)
    D = _dense(A)
    vals = np.linspace(-1.5, 1.75, 10)
    for mask in range(1 << 10):
        idx = np.array([j for j in range(10) if mask >> j & 1], np.int32)
        y, _ = oracle.spmspv(csc, idx, vals[idx])
        xh = np.zeros(10)
        xh[idx] = vals[idx]
        assert np.allclose(y, D @ xh, rtol=1e-14, atol=1e-14)
        yb = oracle.bool_spmspv(A, idx)
        assert yb.tolist() == ((D != 0).astype(int) @ (xh != 0).astype(int) > 0).astype(int).tolist()


@pytest.mark.parametrize("seed", range(4))
def test_int_dense_brute(seed):
    rng = np.random.default_rng(200 + seed)
    m, n = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    A = synth.random_csr(m, n, 0.3, seed, dtype=np.float64)
    vals = rng.integers(-2**31, 2**31, size=A.nnz).astype(np.int32)
    Ai = A.with_vals(vals)
    x = rng.integers(-2**31, 2**31, size=n).astype(np.int32)
    D = np.zeros((m, n), dtype=object)
    rows = np.repeat(np.arange(m), np.diff(A.row_ptr))
    for r, c, v in zip(rows, A.col_idx, vals):
        D[r, c] = int(v)
    ref = [(sum(D[i, j] * int(x[j]) for j in range(n)) % 2**32) for i in range(m)]
    ref = np.array([r - 2**32 if r >= 2**31 else r for r in ref], dtype=np.int64)
    assert np.array_equal(oracle.int_spmv(Ai, x).astype(np.int64), ref)
    csc = oracle.transpose(Ai, int_values=True)
    assert np.array_equal(oracle.int_spmspv(csc, np.arange(n), x).astype(np.int64), ref)


def test_scipy_library_routine():
    A = synth.uniform_rows(3000, 2500, 12, 5)
    x = synth.dense_vector(2500, 6)
    S = sp.csr_matrix((A.vals.astype(np.float64), A.col_idx, A.row_ptr), shape=(A.m, A.n))
    y, _ = oracle.spmv(A, x)
    assert np.allclose(y, S @ x.astype(np.float64), rtol=1e-12, atol=1e-14)
    v = synth.sparse_vector(2500, 300, 7)
    csc = oracle.transpose(A)
    y2, _ = oracle.spmspv(csc, v.idx, v.val)
    assert np.allclose(y2, S @ v.dense(np.float64), rtol=1e-12, atol=1e-14)


def test_compensated_sum():
    """A row whose terms cancel catastrophically: plain float64 left-to-right
    gives 0, the exact sum is 2."""
    A = _mat(1, 4, [0, 4], [0, 1, 2, 3], [1e16, 1.0, -1e16, 1.0])
    y, s = oracle.spmv(A, [1.0, 1.0, 1.0, 1.0])
    assert y[0] == 2.0
    assert s[0] == 2e16 + 2.0


def test_integer_valued_inputs_exact():
    A = synth.random_csr(50, 60, 0.3, 3, int_values=True, dtype=np.float32)
    x = synth.dense_vector(60, 4, "int")
    y, _ = oracle.spmv(A, x)
    Di = _dense(A, np.int64)
    assert np.array_equal(y, (Di @ x.astype(np.int64)).astype(np.float64))


# ------------------------------------------------------------ transpose

def test_transpose_structure():
    A = synth.random_csr(40, 33, 0.2, 9, empty_rows=0.2)
    csc = oracle.transpose(A)
    D = _dense(A)
    Dc = np.zeros_like(D)
    cols = np.repeat(np.arange(A.n), np.diff(csc.col_ptr))
    Dc[csc.row_idx, cols] = csc.vals
    assert np.array_equal(D, Dc)
    for j in range(A.n):
        seg = csc.row_idx[csc.col_ptr[j]:csc.col_ptr[j + 1]]
        assert np.all(np.diff(seg) > 0)
    assert np.array_equal(csc.vals, A.vals.astype(np.float64)[csc.perm])
    assert sorted(csc.perm.tolist()) == list(range(A.nnz))


# ------------------------------------------------------------ closed forms

def test_poisson_closed_form():
    """y = A * 1 on the 7-point Laplacian: 6 minus the number of in-grid
    neighbours, i.e. the number of coordinates on the grid boundary."""
    k = 128
    A = synth.poisson3d(k, np.float32)
    assert A.m == 2_097_152 and A.nnz == 14_581_760
    y, s = oracle.spmv(A, np.ones(A.n))
    idx = np.arange(A.n)
    cx, cy, cz = idx % k, (idx // k) % k, idx // (k * k)
    onb = sum(((c == 0) | (c == k - 1)).astype(np.int64) for c in (cx, cy, cz))
    # a coordinate at 0 or k-1 drops exactly one neighbour (k > 2)
    assert np.array_equal(y, onb.astype(np.float64))
    assert np.array_equal(s, 6.0 + (6 - onb))
    f = oracle.matrix_features(A)
    assert f["min_row"] == 4 and f["max_row"] == 7
    assert f["avg_row"] == 14_581_760 / 2_097_152 == 6.953125


def test_poisson_fp64_small():
    A = synth.poisson3d(6, np.float64)
    D = _dense(A)
    assert np.array_equal(D, D.T)
    # the Dirichlet Laplacian is positive definite
    assert np.linalg.eigvalsh(D).min() > 0
    x = synth.dense_vector(A.n, 1, "normal", np.float64)
    y, _ = oracle.spmv(A, x)
    assert np.allclose(y, D @ x, rtol=1e-14, atol=1e-14)


# ------------------------------------------------------------ features

def _gini_mean_abs_diff(r):
    r = np.asarray(r, np.float64)
    if r.sum() == 0:
        return 0.0
    return np.abs(r[:, None] - r[None, :]).sum() / (2 * r.size * r.sum())


@pytest.mark.parametrize("seed", range(4))
def test_features_brute(seed):
    A = synth.random_csr(37 + seed, 29, 0.25, seed, empty_rows=0.15)
    f = oracle.matrix_features(A)
    L = np.diff(A.row_ptr).astype(np.float64)
    assert f["m"] == A.m and f["n"] == A.n and f["nnz"] == A.nnz
    assert f["max_row"] == L.max() and f["min_row"] == L.min()
    assert f["avg_row"] == pytest.approx(L.mean(), rel=1e-15)
    assert f["relative_range"] == pytest.approx((L.max() - L.min()) / A.n, rel=1e-15)
    assert f["var_nnz_row"] == pytest.approx(L.std(ddof=0), rel=1e-13)
    assert f["gini"] == pytest.approx(_gini_mean_abs_diff(L), rel=1e-12, abs=1e-15)
    csc = oracle.transpose(A)
    D = _dense(A)
    v = synth.sparse_vector(A.n, 7, seed)
    vf = oracle.vector_features(csc, v.idx)
    assert vf["nnz_s"] == (D[:, v.idx] != 0).sum()
    assert vf["m_sparsity"] == pytest.approx(vf["nnz_s"] / A.nnz, rel=1e-15)
    assert vf["x_sparsity"] == pytest.approx(7 / A.n, rel=1e-15)


def test_features_special_cases():
    A = synth.uniform_rows(100, 50, 5, 1)
    f = oracle.matrix_features(A)
    assert f["var_nnz_row"] == 0 and f["gini"] == 0 and f["relative_range"] == 0
    m = 64
    A1 = _mat(m, 10, [0] * 10 + [4] * (m - 9), [0, 1, 2, 3], [1.0] * 4)
    f1 = oracle.matrix_features(A1)
    assert f1["gini"] == pytest.approx(1 - 1 / m, rel=1e-15)
    A0 = _mat(5, 5, [0] * 6, [], [])
    f0 = oracle.matrix_features(A0)
    assert f0["gini"] == 0 and f0["nnz"] == 0


# ------------------------------------------------------------ invariants

def test_spmspv_equals_spmv_of_zero_filled():
    A = synth.cfg1_matrix()
    csc = oracle.transpose(A)
    _, sparse = synth.cfg1_vectors()
    for v in sparse:
        y1, s1 = oracle.spmspv(csc, v.idx, v.val)
        y2, s2 = oracle.spmv(A, v.dense(np.float32))
        # both sums are compensated over exact products: equal to rounding
        assert np.allclose(y1, y2, rtol=0, atol=1e-15 * (1 + s2.max()))
        assert np.allclose(s1, s2, rtol=1e-15, atol=0)


def test_power_of_two_linearity_and_permutation():
    A = synth.uniform_rows(500, 400, 9, 2)
    csc = oracle.transpose(A)
    v = synth.sparse_vector(400, 90, 3)
    y, _ = oracle.spmspv(csc, v.idx, v.val)
    for k in (-3, 5):
        yk, _ = oracle.spmspv(csc, v.idx, v.val.astype(np.float64) * 2.0 ** k)
        assert np.array_equal(yk, y * 2.0 ** k)
    perm = np.random.default_rng(0).permutation(v.nnz)
    Ab = A.with_vals(None)
    assert np.array_equal(oracle.bool_spmspv(Ab, v.idx), oracle.bool_spmspv(Ab, v.idx[perm]))
    Ai = A.with_vals(np.random.default_rng(1).integers(-9, 9, A.nnz).astype(np.int32))
    csci = oracle.transpose(Ai, int_values=True)
    xi = np.random.default_rng(2).integers(-9, 9, v.nnz).astype(np.int32)
    assert np.array_equal(oracle.int_spmspv(csci, v.idx, xi),
                          oracle.int_spmspv(csci, v.idx[perm], xi[perm]))


def test_bool_equals_bfs_step():
    """The (OR, AND) product of the pattern with a frontier is one BFS
    expansion over the edge list (edge j -> i for every stored (i, j))."""
    A = synth.rmat(14, 16, 4242)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr)).astype(np.int32)
    src, dst = A.col_idx, rows
    fronts = synth.bfs_frontiers(A)
    assert len(fronts) >= 3
    for fr in fronts:
        nxt = oracle.bfs_step(src, dst, A.n, A.m, fr.idx)
        yb = oracle.bool_spmspv(A, fr.idx)
        assert np.array_equal(nxt, yb)


def test_transpose_identity():
    """<g, A x> = <A^T g, x> (the dx of the gradient)."""
    A = synth.bernoulli(300, 200, 0.05, 11)
    x = synth.dense_vector(200, 1, "normal", np.float64)
    g = synth.dense_vector(300, 2, "normal", np.float64)
    y, _ = oracle.spmv(A, x)
    dX, _, _ = oracle.grad(A, g[None, :], x[None, :], want_dvals=False)
    lhs = float(np.dot(g, y))
    rhs = float(np.dot(dX[0], x))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(g) @ np.abs(_dense(A)) @ np.abs(x))


def _fd_check(grad_fn, A, G, X, h=2.0 ** -10):
    """L(vals, X) = sum_b <G_b, A(vals) X_b> is bilinear, so central
    differences are exact up to float64 rounding."""
    vals = np.asarray(A.vals, np.float64)

    def L(v, Xm):
        Av = A.with_vals(v)
        return sum(float(np.dot(G[b], oracle.spmv(Av, Xm[b])[0])) for b in range(G.shape[0]))

    dX, _, dv = grad_fn(A, G, X)
    ok = True
    scale = sum(float(np.abs(G[b]) @ np.abs(_dense(A)) @ np.abs(X[b])) for b in range(G.shape[0]))
    for k in range(A.nnz):
        e = np.zeros_like(vals)
        e[k] = h
        fd = (L(vals + e, X) - L(vals - e, X)) / (2 * h)
        ok &= abs(fd - dv[k]) <= 1e-9 * abs(dv[k]) + 1e-12 * scale
    for b in range(X.shape[0]):
        for j in range(A.n):
            E = np.zeros_like(X)
            E[b, j] = h
            fd = (L(vals, X + E) - L(vals, X - E)) / (2 * h)
            ok &= abs(fd - dX[b, j]) <= 1e-9 * abs(dX[b, j]) + 1e-12 * scale
    return bool(ok)


def test_grad_finite_differences():
    A = synth.bernoulli(64, 32, 0.05, 12, std=1.0, dtype=np.float64)
    assert A.nnz > 40
    G = synth.dense_vector(2 * 64, 3, "normal", np.float64).reshape(2, 64)
    X = synth.dense_vector(2 * 32, 4, "normal", np.float64).reshape(2, 32)
    assert _fd_check(oracle.grad, A, G, X)


def test_grad_dense_brute():
    A = synth.random_csr(30, 20, 0.3, 13, empty_rows=0.2)
    G = np.random.default_rng(1).standard_normal((3, 30))
    X = np.random.default_rng(2).standard_normal((3, 20))
    dX, sdX, dv = oracle.grad(A, G, X)
    D = _dense(A)
    assert np.allclose(dX, G @ D, rtol=1e-13, atol=1e-13)
    assert np.allclose(sdX, np.abs(G) @ np.abs(D), rtol=1e-13)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    assert np.allclose(dv, (G[:, rows] * X[:, A.col_idx]).sum(0), rtol=1e-13, atol=1e-14)


# ------------------------------------------------------------ planted mistakes
# Each test below feeds the pin a deliberately wrong oracle and asserts the
# pin rejects it, showing the pins are sensitive to the usual slips.

def test_pin_catches_dropped_term():
    def bad_spmv(A, x):
        # drops the last stored entry of every row
        keep = np.ones(A.nnz, bool)
        ends = A.row_ptr[1:][np.diff(A.row_ptr) > 0] - 1
        keep[ends] = False
        rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))[keep]
        B = synth._coo_to_csr(A.m, A.n, rows, A.col_idx[keep], A.vals[keep])
        return oracle.spmv(B, x)

    A = synth.random_csr(20, 20, 0.3, 1)
    x = synth.dense_vector(20, 1)
    assert _check_spmv_brute(oracle.spmv, A, x)
    assert not _check_spmv_brute(bad_spmv, A, x)


def test_pin_catches_transposed_operand_and_sign():
    A = synth.random_csr(20, 20, 0.3, 2)
    x = synth.dense_vector(20, 2)

    def transposed(A, x):
        csc = oracle.transpose(A)
        At = SimpleNamespace(m=A.n, n=A.m, row_ptr=csc.col_ptr, col_idx=csc.row_idx, vals=csc.vals)
        return oracle.spmv(At, x)

    def sign(A, x):
        y, s = oracle.spmv(A, x)
        return -y, s

    def index_shift(A, x):
        return oracle.spmv(A, np.roll(x, 1))

    for bad in (transposed, sign, index_shift):
        assert not _check_spmv_brute(bad, A, x), bad.__name__


def test_pin_catches_bad_gradient():
    A = synth.bernoulli(16, 12, 0.3, 14, std=1.0, dtype=np.float64)
    G = np.random.default_rng(3).standard_normal((1, 16))
    X = np.random.default_rng(4).standard_normal((1, 12))

    def swapped(A, G, X):
        dX, s, dv = oracle.grad(A, G, X)
        return dX, s, dv[::-1].copy()

    def no_transpose(A, G, X):
        # A g (leading 12 x 12 block) in place of A^T g
        dX, s, dv = oracle.grad(A, G, X)
        D = _dense(A)
        return (D[:12, :12] @ G[0, :12])[None, :], s, dv

    assert _fd_check(oracle.grad, A, G, X)
    assert not _fd_check(swapped, A, G, X)
    assert not _fd_check(no_transpose, A, G, X)


def test_pin_catches_wrong_gini():
    L = np.array([0, 2, 2, 3, 9, 1])
    A = _mat(6, 10, np.concatenate([[0], np.cumsum(L)]), np.zeros(L.sum(), np.int32),
             np.ones(L.sum()))
    f = oracle.matrix_features(A)
    assert f["gini"] == pytest.approx(_gini_mean_abs_diff(L), rel=1e-12)
    # the usual slip: 0-based rank in (2i - m - 1)
    srt = np.sort(L)
    wrong = sum((2 * i - 6 - 1) * r for i, r in enumerate(srt)) / (6 * L.sum())
    assert wrong != pytest.approx(_gini_mean_abs_diff(L), rel=1e-6)


def test_bfs_levels_hand_worked():
    """Six vertices: 0 -> 1 -> 2 -> 3, 0 -> 2, 4 -> 0, and 5 alone.
    From 0: levels 0, 1, 1, 2, unreachable, unreachable. From 4: one more
    everywhere below it, 0 for itself."""
    src = np.array([0, 1, 2, 0, 4], np.int32)
    dst = np.array([1, 2, 3, 2, 0], np.int32)
    assert oracle.bfs_levels(src, dst, 6, 0).tolist() == [0, 1, 1, 2, -1, -1]
    assert oracle.bfs_levels(src, dst, 6, 4).tolist() == [1, 2, 2, 3, 0, -1]
    assert oracle.bfs_levels(src, dst, 6, 5).tolist() == [-1, -1, -1, -1, -1, 0]


def test_bfs_levels_vs_scipy_shortest_path():
    """Levels equal the unweighted directed shortest-path lengths of scipy's
    csgraph, on random graphs from dense enough to sparse enough to leave
    vertices unreachable."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(17)
    for n, deg in ((40, 0.5), (300, 1.2), (300, 4.0), (1000, 2.0)):
        ne = int(n * deg)
        src = rng.integers(0, n, ne).astype(np.int32)
        dst = rng.integers(0, n, ne).astype(np.int32)
        g = sp.csr_matrix((np.ones(ne), (src, dst)), shape=(n, n))
        for s in (0, n // 2, n - 1):
            want = shortest_path(g, directed=True, unweighted=True, indices=s)
            want = np.where(np.isinf(want), -1, want).astype(np.int64)
            got = oracle.bfs_levels(src, dst, n, s)
            assert np.array_equal(got, want), (n, deg, s)


# ---------------------------------------------------------------- PageRank
def _pr_dense(A, d):
    """I - d P as a dense matrix, P = A diag(1/W) (dangling columns zero)."""
    n = A.n
    D = np.zeros((n, n))
    for i in range(A.m):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col_idx[k]] += A.vals[k]
    W = D.sum(0)
    P = np.divide(D, W, out=np.zeros_like(D), where=W > 0)
    return np.eye(n) - d * P


def test_pagerank_hand_worked():
    d = 0.85
    # one edge 0 -> 1, vertex 1 dangling: p0 = (1 - d)/2, p1 = (1 - d)/2 + d p0,
    # reached after one product and a last round that only moves r1
    A = _mat(2, 2, [0, 0, 1], [0], [0.5])
    p, r, k = oracle.pagerank_incremental(A, d, 0.0, 100)
    assert k == 1
    assert np.allclose(p, [(1 - d) / 2, (1 - d) / 2 * (1 + d)], rtol=1e-15, atol=0)
    assert np.all(r == 0)
    # a directed 3-cycle: P is a permutation, so p = 1/3 everywhere
    A = _mat(3, 3, [0, 1, 2, 3], [2, 0, 1], [1.0, 2.0, 3.0])
    p, r, k = oracle.pagerank_incremental(A, d, 0.0, 400)
    assert k == 400
    assert np.allclose(p, 1 / 3, rtol=1e-13, atol=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pagerank_fixed_point_by_dense_solve(seed):
    """eps = 0: after k products the error is at most d^k / (1 - d) * sum r0,
    so 400 products reach the dense solve of (I - d P) p = (1 - d)/n to
    rounding; weighted edges, dangling and isolated vertices included."""
    A = synth.random_csr(60, 60, 0.06, 900 + seed, empty_rows=0.1)
    A = A.with_vals(np.abs(np.asarray(A.vals, np.float64)) + 0.1)
    d = 0.85
    p, r, k = oracle.pagerank_incremental(A, d, 0.0, 400)
    want = np.linalg.solve(_pr_dense(A, d), np.full(A.n, (1 - d) / A.n))
    assert np.allclose(p, want, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("eps_scale", [1e-1, 1e-3])
def test_pagerank_threshold_residual_identity(eps_scale):
    """eps > 0: the loop stops with every |r_v| <= eps, p below the fixed
    point, and p + (I - d P)^-1 r equal to it (the residual identity)."""
    A = synth.random_csr(80, 80, 0.05, 77, empty_rows=0.05)
    A = A.with_vals(np.abs(np.asarray(A.vals, np.float64)) + 0.05)
    d = 0.85
    eps = eps_scale * (1 - d) / A.n
    p, r, k = oracle.pagerank_incremental(A, d, eps, 10 ** 6)
    M = _pr_dense(A, d)
    want = np.linalg.solve(M, np.full(A.n, (1 - d) / A.n))
    assert k > 1
    assert np.all(np.abs(r) <= eps)
    assert np.all(p <= want + 1e-15)
    assert np.allclose(p + np.linalg.solve(M, r), want, rtol=1e-12, atol=1e-15)
    # and the unfinished state after a few products obeys the same identity
    p3, r3, k3 = oracle.pagerank_incremental(A, d, eps, 3)
    assert k3 == 3
    assert np.allclose(p3 + np.linalg.solve(M, r3), want, rtol=1e-12, atol=1e-15)


def test_pagerank_pins_catch_planted_mistakes(monkeypatch):
    """Mistakes planted in the oracle: a transposed product, and weights
    normalized by the out-degree instead of the column weight sum. The
    dense-solve pin fails on each."""
    A = synth.random_csr(40, 40, 0.1, 5, empty_rows=0.0)
    A = A.with_vals(np.abs(np.asarray(A.vals, np.float64)) + 0.1)
    d = 0.85
    want = np.linalg.solve(_pr_dense(A, d), np.full(A.n, (1 - d) / A.n))
    p, _, _ = oracle.pagerank_incremental(A, d, 0.0, 400)
    assert np.allclose(p, want, rtol=1e-12)

    good_spmv = oracle.spmv
    T = synth._coo_to_csr(A.n, A.m, np.asarray(A.col_idx, np.int64),
                          np.repeat(np.arange(A.m), np.diff(A.row_ptr)), np.asarray(A.vals, np.float64))
    with monkeypatch.context() as mp:
        mp.setattr(oracle, "spmv", lambda M, x: good_spmv(T, x))
        p, _, _ = oracle.pagerank_incremental(A, d, 0.0, 400)
    assert not np.allclose(p, want, rtol=1e-6)

    class _Np:
        def __getattr__(self, k):
            return getattr(np, k)
    shim = _Np()
    shim.add = SimpleNamespace(at=lambda W, idx, v: np.add.at(W, idx, 1.0))
    with monkeypatch.context() as mp:
        mp.setattr(oracle, "np", shim)
        p, _, _ = oracle.pagerank_incremental(A, d, 0.0, 400)
    assert not np.allclose(p, want, rtol=1e-6)


# ---------------------------------------------------------------- sparse output, complement mask
def test_sparse_output_hand_worked():
    """A (4 x 3): rows 0: (0, 2.0); 1: (1, -1.0), (2, 1.0); 2: (2, 3.0);
    3: (0, 1.0), (2, -1.0). x = {0: 1.0, 2: 1.0}. y = [2, 1, 3, 0]: row 3 is
    listed with value 0 (its products cancel), row 1 through column 2 only.
    With row 2 masked the list is rows 0, 1, 3."""
    A = _mat(4, 3, [0, 1, 3, 4, 6], [0, 1, 2, 2, 0, 2], [2.0, -1.0, 1.0, 3.0, 1.0, -1.0])
    rows, vals, _ = oracle.spmspv_sparse(A, [0, 2], [1.0, 1.0])
    assert rows.tolist() == [0, 1, 2, 3] and vals.tolist() == [2.0, 1.0, 3.0, 0.0]
    rows, vals, _ = oracle.spmspv_sparse(A, [0, 2], [1.0, 1.0], mask=[False, False, True, False])
    assert rows.tolist() == [0, 1, 3] and vals.tolist() == [2.0, 1.0, 0.0]
    rows, vals, _ = oracle.spmspv_sparse(A, [1], [5.0], kind="bool")
    assert rows.tolist() == [1] and vals.tolist() == [1]
    rows, vals, _ = oracle.spmspv_sparse(A, [], [])
    assert rows.size == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sparse_output_brute_force(seed):
    """Against a dense matrix: listed rows = rows with a stored entry in a
    selected column and no mask bit; values = the dense product."""
    rng = np.random.default_rng(seed)
    A = synth.random_csr(30, 25, 0.12, 40 + seed, empty_rows=0.2)
    D = np.zeros((A.m, A.n))
    P = np.zeros((A.m, A.n), bool)
    for i in range(A.m):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col_idx[k]] += A.vals[k]
            P[i, A.col_idx[k]] = True
    x_idx = np.sort(rng.choice(A.n, 6, replace=False)).astype(np.int32)
    x_val = rng.uniform(-1, 1, 6)
    mask = rng.random(A.m) < 0.3
    x = np.zeros(A.n)
    x[x_idx] = x_val
    sel = np.zeros(A.n, bool)
    sel[x_idx] = True
    want_rows = np.nonzero(P[:, sel].any(1) & ~mask)[0]
    rows, vals, _ = oracle.spmspv_sparse(A, x_idx, x_val, mask=mask)
    assert rows.tolist() == want_rows.tolist()
    assert np.allclose(vals, (D @ x)[want_rows], rtol=1e-14, atol=1e-15)


def test_sparse_output_pin_catches_numeric_listing(monkeypatch):
    """A planted mistake: listing the rows whose value is nonzero instead of
    the rows an effective entry reaches drops row 3 of the hand-worked case."""
    A = _mat(4, 3, [0, 1, 3, 4, 6], [0, 1, 2, 2, 0, 2], [2.0, -1.0, 1.0, 3.0, 1.0, -1.0])

    def numeric(M, xi):
        y, _ = oracle.spmspv(oracle.transpose(M), xi, np.ones(len(xi)))
        return (y != 0).astype(np.uint8)
    with monkeypatch.context() as mp:
        mp.setattr(oracle, "bool_spmspv", numeric)
        rows, _, _ = oracle.spmspv_sparse(A, [0, 2], [1.0, 1.0])
    assert rows.tolist() != [0, 1, 2, 3]


# ---------------------------------------------------------------- min-plus semiring
def test_minplus_hand_worked():
    """A (3 x 3): (0, 2) 1.5; (1, 0) 2.0, (1, 2) 0.25; (2, 1) 3.0; x = [0, inf, 1].
    Row 0: 1.5 + 1 = 2.5. Row 1: min(2 + 0, 0.25 + 1) = 1.25. Row 2 reads only
    the absent x_1: +inf."""
    A = _mat(3, 3, [0, 1, 3, 4], [2, 0, 2, 1], [1.5, 2.0, 0.25, 3.0])
    y = oracle.minplus_spmv(A, np.array([0.0, np.inf, 1.0], np.float32))
    assert y.tolist() == [2.5, 1.25, np.inf]
    y = oracle.minplus_spmspv(A, [0, 2], [0.0, 1.0])
    assert y.tolist() == [2.5, 1.25, np.inf]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_minplus_brute_force_float32(seed):
    """Against a dense table of float32 sums a_ij + x_j (numpy float32
    adds, one rounding each) and their minimum: bit-exact."""
    rng = np.random.default_rng(seed)
    A = synth.random_csr(40, 30, 0.15, 70 + seed, empty_rows=0.2)
    x = rng.uniform(-2, 2, A.n).astype(np.float32)
    x[rng.random(A.n) < 0.3] = np.inf
    want = np.full(A.m, np.inf, np.float32)
    for i in range(A.m):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = A.col_idx[k]
            if np.isfinite(x[j]):
                want[i] = min(want[i], np.float32(np.float32(A.vals[k]) + x[j]))
    assert np.array_equal(oracle.minplus_spmv(A, x), want)


def _bellman_ford(A, source, prod):
    d = np.full(A.n, np.inf, np.float32)
    d[source] = 0.0
    for _ in range(A.n):
        nd = np.minimum(d, prod(A, d))
        if np.array_equal(nd, d):
            break
        d = nd
    return d


def test_minplus_relaxation_is_shortest_paths():
    """Entry (i, j) is the edge j -> i, so repeated relaxation d = min(d, A (x) d)
    from a source reaches scipy's Dijkstra distances on the graph A^T, exactly
    (integer weights are exact in float32)."""
    from scipy.sparse.csgraph import dijkstra
    rng = np.random.default_rng(9)
    n = 60
    src = rng.integers(0, n, 300)
    dst = rng.integers(0, n, 300)
    key = np.unique(dst.astype(np.int64) * n + src)
    w = rng.integers(1, 20, key.size).astype(np.float32)
    A = synth._coo_to_csr(n, n, key // n, key % n, w)
    G = sp.csr_matrix((np.asarray(A.vals, np.float64), A.col_idx, A.row_ptr), shape=(n, n)).T.tocsr()
    for s0 in (0, 7, 33):
        want = dijkstra(G, directed=True, indices=s0)
        got = _bellman_ford(A, s0, oracle.minplus_spmv)
        assert np.array_equal(got.astype(np.float64), want)


def test_minplus_pins_catch_planted_mistakes(monkeypatch):
    """A transposed product (edges read the wrong way) breaks the
    shortest-path pin; a sum instead of the minimum breaks the hand-worked
    one."""
    from scipy.sparse.csgraph import dijkstra
    A = _mat(3, 3, [0, 1, 3, 4], [2, 0, 2, 1], [1.5, 2.0, 0.25, 3.0])
    T = _mat(3, 3, [0, 1, 2, 4], [1, 2, 0, 1], [2.0, 3.0, 1.5, 0.25])  # A^T
    G = sp.csr_matrix((np.asarray(A.vals, np.float64), A.col_idx, A.row_ptr), shape=(3, 3)).T.tocsr()
    want = dijkstra(G, directed=True, indices=0)
    good = oracle.minplus_spmv
    with monkeypatch.context() as mp:
        mp.setattr(oracle, "minplus_spmv", lambda M, x: good(T, x))
        got = _bellman_ford(A, 0, lambda M, d: oracle.minplus_spmv(M, d))
    assert not np.array_equal(got.astype(np.float64), want)

    def summed(M, x):
        y = np.zeros(M.m, np.float32)
        for i in range(M.m):
            for k in range(M.row_ptr[i], M.row_ptr[i + 1]):
                if np.isfinite(x[M.col_idx[k]]):
                    y[i] += M.vals[k] + x[M.col_idx[k]]
        return y
    with monkeypatch.context() as mp:
        mp.setattr(oracle, "minplus_spmv", summed)
        got = oracle.minplus_spmv(A, np.array([0.0, np.inf, 1.0], np.float32))
    assert got.tolist() != [2.5, 1.25, np.inf]


def test_row_range_and_openmp_scatter_equal_the_column_scatter():
    """The row-range scatter (binary searches cut each column to the range)
    and its OpenMP driver give the column scatter's bits: every row receives
    the same terms in the same order. Ranges: empty, one row, the first and
    last rows, ragged splits; matrices with empty rows and columns, and
    R-MAT with hub columns."""
    from paper_2006_16767_amd import synth
    mats = [synth.random_csr(97, 61, 0.08, 5, empty_rows=0.2), synth.rmat(14, 8, 99)]
    for A in mats:
        csc = oracle.transpose(A)
        for nnz in (0, 1, A.n // 7, A.n):
            v = synth.sparse_vector(A.n, nnz, 40 + nnz)
            y, s = oracle.spmspv(csc, v.idx, v.val)
            yo, so = oracle.spmspv_omp(csc, v.idx, v.val)
            assert np.array_equal(y, yo) and np.array_equal(s, so)
            for r0, r1 in ((0, 0), (0, 1), (A.m - 1, A.m), (3, 3), (0, A.m), (A.m // 3, 2 * A.m // 3 + 1)):
                yr, sr = oracle.spmspv_rows(csc, v.idx, v.val, r0, r1)
                assert np.array_equal(yr, y[r0:r1]) and np.array_equal(sr, s[r0:r1])
    assert oracle.omp_threads() >= 1
