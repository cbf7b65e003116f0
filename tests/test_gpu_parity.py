"""Parity of every candidate kernel with the CPU oracle, through the C ABI.

Bit-exact for BOOL and I32 (and for FP inputs with small integer values);
FP32 within 1e-5 * sum_j |a_ij x_j| and FP64 within 1e-12 * the same, with
exact zeros where no entry is effective. Sizes span several tiles with
ragged tails; the workload configurations run at full size."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close, cfg_matrix, dev_sparse, reference

pytestmark = pytest.mark.gpu

KINDS = {"f32": (spx.F32, np.float32), "f64": (spx.F64, np.float64), "i32": (spx.I32, np.int32),
         "bool": (spx.BOOL, None)}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _matrix(A, kind):
    code, npdt = KINDS[kind]
    if kind == "i32":
        vals = np.asarray(A.vals)
        if vals.dtype != np.int32:
            vals = np.clip(np.round(vals * 4), -4, 4).astype(np.int32)
        A = A.with_vals(vals)
    elif kind in ("f32", "f64"):
        A = A.with_vals(np.asarray(A.vals).astype(npdt))
    return A, spx.Matrix.from_host(A, dtype=code, fmt="csr")


def _vec_vals(v, kind, rng=None):
    if kind == "bool":
        return None
    if kind == "i32":
        if v.val is not None and v.val.dtype == np.int32:
            return v.val
        r = np.random.default_rng(v.nnz + 7)
        return r.integers(-5, 6, size=v.nnz).astype(np.int32)
    return np.asarray(v.val).astype(KINDS[kind][1])


def _plans(m, kind):
    out = []
    for p in spx.all_plans():
        out.append(p)
    return out


def _run_and_check(M, A, v_idx, v_val, kind, plans, what, dense=False):
    torch = _torch()
    code, npdt = KINDS[kind]
    ref, S = reference(A, v_idx, v_val if kind != "bool" else None, kind)
    if dense:
        xd = np.zeros(A.n, dtype=npdt if npdt is not None else np.uint8)
        if len(v_idx):
            xd[v_idx] = v_val if kind != "bool" else 1
        x = torch.as_tensor(xd, device="cuda")
    else:
        idx = torch.as_tensor(np.asarray(v_idx, np.int32), device="cuda")
        val = None if kind == "bool" else torch.as_tensor(np.asarray(v_val, npdt), device="cuda")
        x = (idx, val)
    for p in plans:
        try:
            y = M.run_plan(x, p)
        except spx.SpxError as e:
            if e.code == -5 and p.writeback == spx.WB_LDS_ATOMIC:
                continue  # y does not fit in LDS for this m
            raise
        torch.cuda.synchronize()
        assert_close(y.cpu().numpy(), ref, S, kind, f"{what} {p}")


# ------------------------------------------------------------------ structure

@pytest.mark.parametrize("name", ["cfg1", "rmat16"])
def test_transpose_matches_oracle(name):
    torch = _torch()
    A = cfg_matrix(name)
    M = spx.Matrix.from_host(A, fmt="csr")
    col_ptr, row_idx, vals = M.csc()
    ref = oracle.transpose(A)
    assert np.array_equal(col_ptr.cpu().numpy(), ref.col_ptr)
    assert np.array_equal(row_idx.cpu().numpy(), ref.row_idx)
    assert np.array_equal(vals.cpu().numpy().astype(np.float64), ref.vals)


def test_transpose_ragged_and_empty():
    torch = _torch()
    for m, n, dens, seed in [(37, 53, 0.1, 1), (1, 1, 1.0, 2), (300, 7, 0.5, 3), (5, 400, 0.01, 4)]:
        A = synth.random_csr(m, n, dens, seed, empty_rows=0.3)
        M = spx.Matrix.from_host(A, fmt="csr")
        col_ptr, row_idx, vals = M.csc()
        ref = oracle.transpose(A)
        assert np.array_equal(col_ptr.cpu().numpy(), ref.col_ptr)
        assert np.array_equal(row_idx.cpu().numpy(), ref.row_idx)
    # a matrix with no entries at all
    A0 = synth.CSR(6, 9, np.zeros(7, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    M0 = spx.Matrix.from_host(A0, fmt="csr")
    assert np.array_equal(M0.csc()[0].cpu().numpy(), np.zeros(10, np.int32))
    y = M0.run((torch.as_tensor(np.array([1, 4], np.int32), device="cuda"),
                torch.ones(2, dtype=torch.float32, device="cuda")))
    assert np.array_equal(y.cpu().numpy(), np.zeros(6, np.float32))


@pytest.mark.parametrize("name", ["cfg1", "rmat16", "cfg3"])
def test_features_match_oracle(name):
    _torch()
    A = cfg_matrix(name)
    M = spx.Matrix.from_host(A, fmt="csr")
    f = M.features()
    ref = oracle.matrix_features(A)
    for k, v in ref.items():
        assert f[k] == pytest.approx(v, rel=1e-12, abs=1e-15), k
    csc = oracle.transpose(A, with_values=False)
    v = synth.sparse_vector(A.n, max(1, A.n // 50), 3)
    vf = M.vector_features(dev_sparse(v, np.float32))
    for k, val in oracle.vector_features(csc, v.idx).items():
        assert vf[k] == pytest.approx(val, rel=1e-15), k


# ------------------------------------------------------------------ small and ragged

@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
def test_ragged_all_plans(kind):
    _torch()
    cases = [(37, 53, 0.1), (3001, 2503, 0.004), (700, 9000, 0.002), (2, 1, 1.0)]
    for ci, (m, n, dens) in enumerate(cases):
        A = synth.random_csr(m, n, dens, 100 + ci, empty_rows=0.2)
        A, M = _matrix(A, kind)
        for nnz_x in sorted({0, 1, max(1, n // 7), n}):
            v = synth.sparse_vector(n, nnz_x, 1000 + nnz_x + ci)
            val = _vec_vals(v, kind)
            _run_and_check(M, A, v.idx, val, kind, _plans(m, kind), f"{kind} {m}x{n} nnz_x={nnz_x}")
            if nnz_x in (1, n):
                _run_and_check(M, A, v.idx, val, kind, _plans(m, kind), f"{kind} dense {m}x{n}", dense=True)


def test_hub_rows_and_columns():
    """A row and a column far longer than a tile: merge-path splits them
    across workgroups and the fix-up joins them."""
    _torch()
    m = n = 5000
    rng = np.random.default_rng(5)
    rows = [np.full(n, 17), rng.integers(0, m, 4000), np.arange(m)]
    cols = [np.arange(n), np.full(4000, 23), rng.integers(0, n, m)]
    rr = np.concatenate(rows)
    cc = np.concatenate(cols)
    key = np.unique(rr.astype(np.int64) * n + cc)
    A = synth._coo_to_csr(m, n, key // n, key % n, rng.uniform(-1, 1, key.size).astype(np.float32))
    for kind in ("f32", "i32", "bool"):
        A2, M = _matrix(A, kind)
        for nnz_x in (1, 300, n):
            v = synth.sparse_vector(n, nnz_x, nnz_x)
            idx = np.unique(np.concatenate([v.idx, [23]])).astype(np.int32)
            vv = synth.SparseVec(n, idx, np.random.default_rng(1).uniform(-1, 1, idx.size).astype(np.float32))
            _run_and_check(M, A2, vv.idx, _vec_vals(vv, kind), kind, _plans(m, kind), f"hub {kind} {nnz_x}")


def test_integer_valued_fp32_bitexact():
    """FP32 inputs with small integer values: every partial sum is exact, so
    every kernel must match the oracle bit for bit."""
    torch = _torch()
    A = synth.random_csr(4000, 3000, 0.003, 9, dtype=np.float32, int_values=True, empty_rows=0.1)
    M = spx.Matrix.from_host(A, fmt="csr")
    for nnz_x in (5, 300, 3000):
        v = synth.sparse_vector(3000, nnz_x, nnz_x, dist="int")
        ref, S = reference(A, v.idx, v.val, "f32")
        for p in spx.all_plans():
            try:
                y = M.run_plan(dev_sparse(v, np.float32), p)
            except spx.SpxError as e:
                if e.code == -5:
                    continue
                raise
            assert np.array_equal(y.cpu().numpy().astype(np.float64), ref), str(p)


# ------------------------------------------------------------------ workload configs

def test_cfg1_all_plans():
    _torch()
    A = cfg_matrix("cfg1")
    for kind in ("f32", "f64", "i32", "bool"):
        A2, M = _matrix(A, kind)
        dense, sparse = synth.cfg1_vectors()
        for v in sparse:
            _run_and_check(M, A2, v.idx, _vec_vals(v, kind), kind, _plans(A.m, kind), f"cfg1 {kind} {v.nnz}")
        full = synth.SparseVec(A.n, np.arange(A.n, dtype=np.int32), dense)
        _run_and_check(M, A2, full.idx, _vec_vals(full, kind), kind, _plans(A.m, kind), f"cfg1 {kind} dense",
                       dense=True)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_cfg3_poisson_closed_form(dt):
    """A * 1 on the 7-point Laplacian is the count of boundary coordinates:
    exact in any order, so bit-exact."""
    torch = _torch()
    A = cfg_matrix("cfg3" if dt == "f32" else "cfg3_f64")
    M = spx.Matrix.from_host(A, fmt="csr")
    k = 128
    idx = np.arange(A.n)
    onb = sum(((c == 0) | (c == k - 1)).astype(np.int64) for c in (idx % k, (idx // k) % k, idx // (k * k)))
    npdt = np.float32 if dt == "f32" else np.float64
    ones = torch.ones(A.n, dtype=torch.float32 if dt == "f32" else torch.float64, device="cuda")
    all_idx = torch.arange(A.n, dtype=torch.int32, device="cuda")
    for p in spx.all_plans():
        if p.writeback == spx.WB_LDS_ATOMIC:
            continue
        y = M.run_plan(ones, p)
        assert np.array_equal(y.cpu().numpy(), onb.astype(npdt)), str(p)
        y2 = M.run_plan((all_idx, ones), p)
        assert np.array_equal(y2.cpu().numpy(), onb.astype(npdt)), str(p)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_cfg3_dense_and_sparse(dt):
    _torch()
    npdt = np.float32 if dt == "f32" else np.float64
    A = cfg_matrix("cfg3" if dt == "f32" else "cfg3_f64")
    M = spx.Matrix.from_host(A, fmt="csr")
    dense, sparse = synth.cfg3_vectors(dtype=npdt)
    plans = [p for p in spx.all_plans() if p.writeback != spx.WB_LDS_ATOMIC]
    full = np.arange(A.n, dtype=np.int32)
    _run_and_check(M, A, full, dense, dt, plans, f"cfg3 {dt} dense", dense=True)
    _run_and_check(M, A, sparse.idx, sparse.val, dt, plans, f"cfg3 {dt} 1%")


@pytest.mark.slow
def test_cfg2_rmat_sweep():
    """R-MAT 2^20, degree 16, at every density of the sweep, FP32 and the
    boolean pattern (bit-exact)."""
    _torch()
    A = cfg_matrix("cfg2")
    Mf = spx.Matrix.from_host(A, fmt="csr")
    Mb = spx.Matrix.from_host(A, dtype=spx.BOOL, fmt="csr")
    plans = [p for p in spx.all_plans() if p.writeback != spx.WB_LDS_ATOMIC]
    for v in synth.cfg2_vectors():
        _run_and_check(Mf, A, v.idx, v.val, "f32", plans, f"cfg2 f32 nnz_x={v.nnz}")
        _run_and_check(Mb, A, v.idx, None, "bool", plans, f"cfg2 bool nnz_x={v.nnz}")


def test_bool_bfs_frontiers():
    """(OR, AND) products of the pattern with BFS frontiers equal the
    edge-list expansion of each frontier."""
    torch = _torch()
    A = cfg_matrix("rmat16")
    M = spx.Matrix.from_host(A, dtype=spx.BOOL, fmt="csr")
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr)).astype(np.int32)
    plans = [p for p in spx.all_plans() if p.writeback != spx.WB_LDS_ATOMIC]
    for fr in synth.bfs_frontiers(A, max_levels=12):
        nxt = oracle.bfs_step(A.col_idx, rows, A.n, A.m, fr.idx)
        x = (torch.as_tensor(fr.idx, device="cuda"), None)
        for p in plans:
            y = M.run_plan(x, p)
            assert np.array_equal(y.cpu().numpy(), nxt), f"frontier {fr.nnz} {p}"
        assert np.array_equal(M.run(x).cpu().numpy(), nxt)


def test_int_invariant_spmspv_equals_spmv():
    """SpMSpV equals SpMV of the zero-filled vector, bitwise in the integer
    semiring, for every kernel."""
    torch = _torch()
    A = cfg_matrix("rmat16")
    A2, M = _matrix(A, "i32")
    v = synth.sparse_vector(A.n, 3000, 11)
    val = _vec_vals(v, "i32")
    xd = np.zeros(A.n, np.int32)
    xd[v.idx] = val
    base = M.run_plan(torch.as_tensor(xd, device="cuda"), spx.plan("spmv")).cpu().numpy()
    for p in spx.all_plans():
        if p.writeback == spx.WB_LDS_ATOMIC:
            continue
        y = M.run_plan((torch.as_tensor(v.idx, device="cuda"), torch.as_tensor(val, device="cuda")), p)
        assert np.array_equal(y.cpu().numpy(), base), str(p)


def test_direct_entry_points():
    """spmv_csr / spmspv_csr / spmspv_csc called directly with a workspace."""
    torch = _torch()
    A = cfg_matrix("cfg1")
    M = spx.Matrix.from_host(A, fmt="csr")
    dense, sparse = synth.cfg1_vectors()
    x = torch.as_tensor(dense, device="cuda")
    ref, S = reference(A, np.arange(A.n), dense, "f32")
    for d in ("direct", "balanced"):
        y = spx.spmv_csr(M, x, spx.plan("spmv", d))
        assert_close(y.cpu().numpy(), ref, S, "f32", f"spmv_csr {d}")
    v = sparse[1]
    ref, S = reference(A, v.idx, v.val, "f32")
    idx, val = dev_sparse(v, np.float32)
    for d in ("direct", "balanced"):
        y = spx.spmspv_csr(M, idx, val, spx.plan("csr_spmspv", d))
        assert_close(y.cpu().numpy(), ref, S, "f32", f"spmspv_csr {d}")
        for wb in ("atomic", "lds_atomic", "sort"):
            y = spx.spmspv_csc(M, idx, val, spx.plan("csc_spmspv", d, wb))
            assert_close(y.cpu().numpy(), ref, S, "f32", f"spmspv_csc {d} {wb}")


def test_adaptive_run_cfg1_and_rmat16():
    torch = _torch()
    for name in ("cfg1", "rmat16"):
        A = cfg_matrix(name)
        M = spx.Matrix.from_host(A)
        for i, d in enumerate((1e-4, 1e-3, 1e-2, 0.1, 0.5, 1.0)):
            v = synth.sparse_vector(A.n, max(1, round(d * A.n)), 50 + i)
            y = M.run(dev_sparse(v, np.float32))
            ref, S = reference(A, v.idx, v.val, "f32")
            assert_close(y.cpu().numpy(), ref, S, "f32", f"run {name} d={d} plan={M.last_plan()}")
            p = M.select(dev_sparse(v, np.float32))
            assert 0 <= p.pattern <= 2
            pn = M.select(dev_sparse(v, np.float32), no_sync=True)
            assert 0 <= pn.pattern <= 2


def test_errors_on_device():
    torch = _torch()
    A = cfg_matrix("cfg1")
    M = spx.Matrix.from_host(A, fmt="csr")
    with pytest.raises(spx.SpxError) as e:
        M.run(torch.zeros(A.n + 1, device="cuda"))
    # the binding passes n of the matrix; a wrong-length sparse index set is
    # caught by the nnz_x bound
    with pytest.raises(spx.SpxError):
        M.run((torch.zeros(A.n + 5, dtype=torch.int32, device="cuda"), torch.zeros(A.n + 5, device="cuda")))
    bad = synth.CSR(3, 3, np.array([0, 1, 2, 3], np.int32), np.array([0, 5, 1], np.int32),
                    np.ones(3, np.float32))
    with pytest.raises(spx.SpxError) as e:
        spx.Matrix.from_host(bad, validate=True)
    assert e.value.code == -3
    bad2 = synth.CSR(3, 3, np.array([0, 2, 1, 3], np.int32), np.array([0, 1, 1], np.int32),
                     np.ones(3, np.float32))
    with pytest.raises(spx.SpxError) as e:
        spx.Matrix.from_host(bad2, validate=True)
    assert e.value.code == -2


# ------------------------------------------------------------------ backward

@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_backward_matches_oracle(dt):
    torch = _torch()
    npdt = np.float32 if dt == "f32" else np.float64
    tdt = torch.float32 if dt == "f32" else torch.float64
    A = synth.bernoulli(3000, 1200, 0.03, 21, std=0.5, dtype=npdt)
    M = spx.Matrix.from_host(A, fmt="csr")
    B = 5
    G = np.random.default_rng(1).standard_normal((B, A.m)).astype(npdt)
    X = np.zeros((B, A.n), npdt)
    for b in range(B):
        v = synth.sparse_vector(A.n, 100 * (b + 1), b, "halfnormal", npdt)
        X[b, v.idx] = v.val
    dX_ref, sdX, dv_ref = oracle.grad(A, G, X)
    dX = M.transpose_matvec(torch.as_tensor(G, device="cuda")).cpu().numpy()
    for b in range(B):
        assert_close(dX[b], dX_ref[b], sdX[b], dt, f"dx b={b}")
    dv = M.dvals(torch.as_tensor(G, device="cuda"), torch.as_tensor(X, device="cuda")).cpu().numpy()
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    sdv = (np.abs(G[:, rows].astype(np.float64)) * np.abs(X[:, A.col_idx].astype(np.float64))).sum(0)
    assert_close(dv, dv_ref, sdv, dt, "dvals")


# ------------------------------------------------------------------ launch parameters

def _variant_plans():
    out = []
    for L in (1, 2, 4, 8, 16, 32, 64):
        out += [spx.plan("spmv", "direct", lanes=L), spx.plan("csr_spmspv", "direct", lanes=L)]
        for wb in ("atomic", "lds_atomic", "sort", "bucket"):
            out.append(spx.plan("csc_spmspv", "direct", wb, lanes=L))
    for T in (2048, 4096):
        out += [spx.plan("spmv", "balanced", tile=T), spx.plan("csr_spmspv", "balanced", tile=T)]
    out.append(spx.plan("csr_spmspv", "balanced", tile=1))
    for R in (64, 256, 1024, 8192):
        out += [spx.plan("csc_spmspv", "balanced", "bucket", bucket_rows=R),
                spx.plan("csc_spmspv", "direct", "bucket", bucket_rows=R)]
    return out


@pytest.mark.parametrize("kind", ["f32", "i32"])
@pytest.mark.parametrize("name", ["cfg1", "rmat16"])
def test_launch_parameter_variants(name, kind):
    """Every explicit lane count, merge tile and bucket height gives the
    oracle's result (the automatic choices cover only one of each)."""
    _torch()
    A, M = _matrix(cfg_matrix(name), kind)
    for nnz_x in (max(1, A.n // 100), A.n // 2):
        v = synth.sparse_vector(A.n, nnz_x, 900 + nnz_x)
        _run_and_check(M, A, v.idx, _vec_vals(v, kind), kind, _variant_plans(), f"{name} {kind} nnz_x={nnz_x}")


def test_dense_x_never_takes_the_column_major_pattern():
    """A vector handed over dense counts as dense and is read as it is: the
    selection keeps it off the column-major pattern, which would first
    compact it with a host round trip."""
    torch = _torch()
    for name in ("cfg1", "rmat16"):
        A = cfg_matrix(name)
        M = spx.Matrix.from_host(A)
        x = synth.dense_vector(A.n, 3)
        xt = torch.as_tensor(x, device="cuda")
        p = M.select(xt)
        assert p.pattern != spx.PAT_CSC_SPMSPV, (name, p)
        y = M.run(xt)
        torch.cuda.synchronize()
        assert M.last_plan().pattern == p.pattern
        ref, S = oracle.spmv(A, x.astype(np.float64))
        assert_close(y.cpu().numpy(), ref, S, "f32", f"run {name} dense x {M.last_plan()}")
