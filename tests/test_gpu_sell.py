"""Sliced ELLPACK and ELLPACK copies (the storage-format pre-selection):
every SpMV plan on a handle that keeps a copy runs on it. Parity with the oracle's SpMV
for every dtype, dense and sparse x, ragged shapes (m not a multiple of the
64-row slice, empty rows, a row much longer than its slice neighbours), the
renumbered copy, a value refresh, and the refusal of a too-skewed matrix."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close, cfg_matrix, reference

pytestmark = pytest.mark.gpu

KINDS = {"f32": (spx.F32, np.float32), "f64": (spx.F64, np.float64), "i32": (spx.I32, np.int32),
         "bool": (spx.BOOL, None)}
SPMV_PLANS = [spx.plan("spmv", "direct"), spx.plan("spmv", "balanced"), spx.plan("spmv", "balanced", tile=4096)]


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


def _matrices():
    out = [("poisson32", synth.poisson3d(32, np.float32)),
           ("cfg1", cfg_matrix("cfg1")),
           ("ragged", synth.random_csr(3001, 2503, 0.004, 91, empty_rows=0.2)),
           ("tiny", synth.random_csr(37, 53, 0.1, 92, empty_rows=0.2))]
    # one row far longer than the others of its slice
    A = synth.random_csr(20000, 3000, 0.002, 93)
    rows = [np.asarray(A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]) for i in range(A.m)]
    rows[130] = np.arange(0, 3000, 3, dtype=np.int32)
    rp = np.zeros(A.m + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    vals = np.random.default_rng(94).uniform(-1, 1, ci.size).astype(np.float32)
    out.append(("long_row", synth.CSR(A.m, A.n, rp, ci, vals)))
    return out


def _run_all(M, A, kind, tag):
    torch = _torch()
    code, npdt = KINDS[kind]
    rng = np.random.default_rng(5)
    for nnz_x in sorted({0, 1, max(1, A.n // 10), A.n}):
        v = synth.sparse_vector(A.n, nnz_x, 800 + nnz_x)
        val = None
        if kind == "i32":
            val = rng.integers(-5, 6, size=v.nnz).astype(np.int32)
        elif kind != "bool":
            val = np.asarray(v.val).astype(npdt)
        ref, S = reference(A, v.idx, val, kind)
        xd = np.zeros(A.n, dtype=npdt if npdt is not None else np.uint8)
        xd[v.idx] = val if kind != "bool" else 1
        xs = [torch.as_tensor(xd, device="cuda"),
              (torch.as_tensor(v.idx, device="cuda"), None if kind == "bool" else torch.as_tensor(val, device="cuda"))]
        for x in xs:
            for p in SPMV_PLANS:
                y = M.run_plan(x, p)
                torch.cuda.synchronize()
                assert_close(y.cpu().numpy(), ref, S, kind, f"{tag} {kind} nnz_x={nnz_x} {p}")


@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
def test_sell_spmv_matches_oracle(kind):
    _torch()
    for name, A0 in _matrices():
        A = _with_kind(A0, kind)
        M = spx.Matrix.from_host(A, dtype=KINDS[kind][0], fmt="sell", renumber=False)
        fmt, ratio = M.storage_format()
        assert fmt == "sell" and ratio >= 1.0, (name, fmt, ratio)
        _run_all(M, A, kind, name)


def test_sell_on_the_renumbered_copy():
    _torch()
    A = _with_kind(synth.random_csr(5000, 70000, 0.0005, 95), "f32")
    M = spx.Matrix.from_host(A, fmt="sell", renumber=True)
    assert M.column_order() is not None and M.storage_format()[0] == "sell"
    _run_all(M, A, "f32", "renumbered")


def test_sell_minplus_bit_exact():
    torch = _torch()
    A = synth.poisson3d(16, np.float32)
    A = A.with_vals(np.random.default_rng(3).uniform(-1, 1, A.nnz).astype(np.float32))
    M = spx.Matrix.from_host(A, dtype=spx.F32_MINPLUS, fmt="sell")
    assert M.storage_format()[0] == "sell"
    xd = np.random.default_rng(4).uniform(-1, 1, A.n).astype(np.float32)
    xd[np.random.default_rng(5).random(A.n) < 0.5] = np.inf
    want = oracle.minplus_spmv(A, xd)
    for p in SPMV_PLANS:
        got = M.run_plan(torch.as_tensor(xd, device="cuda"), p).cpu().numpy()
        assert np.array_equal(got, want), p


def test_sell_follows_values_updated():
    torch = _torch()
    A = synth.poisson3d(24, np.float32)
    M = spx.Matrix.from_host(A, fmt="sell")
    new = np.random.default_rng(8).uniform(-2, 2, A.nnz).astype(np.float32)
    M.vals.copy_(torch.as_tensor(new, device="cuda"))
    M.values_updated()
    B = A.with_vals(new)
    x = synth.dense_vector(A.n, 9)
    ref, S = oracle.spmv(B, x.astype(np.float64))
    y = M.run_plan(torch.as_tensor(x, device="cuda"), spx.plan("spmv", "direct"))
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), ref, S, "f32", "after update")


def test_sell_refused_when_too_skewed():
    _torch()
    A = cfg_matrix("rmat16")
    with pytest.raises(spx.SpxError) as e:
        spx.Matrix.from_host(A, fmt="sell")
    assert e.value.code == -5
    assert spx.Matrix.from_host(A, fmt="csr").storage_format()[0] == "csr"
    assert spx.Matrix.from_host(synth.poisson3d(16, np.float32), fmt="csr").storage_format() == ("csr", 0.0)


def test_padding_ratio_matches_the_layout_definition():
    """The library's cells / nnz equals the layout's definition recomputed
    in numpy (slices of 64 rows, rows sorted by descending length within
    windows of 4096, each slice padded to its longest row)."""
    _torch()
    from paper_2006_16767_amd import tune
    for name, A in _matrices():
        M = spx.Matrix.from_host(A, fmt="sell", renumber=False)
        assert M.storage_format()[1] == pytest.approx(tune.sell_padding(A), rel=1e-12), name


def test_auto_format_follows_the_tree():
    """Up to 1.17M entries: rows of at most 7 entries go to ELL, up to 1158 to
    the sliced copy, longer to CSR5. Beyond: nearly equal rows to ELL up to
    15.7M entries and to the sliced copy past that, rows longer than 17 % of
    n to CSR5, the large R-MAT graphs stay in CSR. The stencils lie on 7
    diagonals and take the DIA copy, which is tried before the tree."""
    _torch()
    assert spx.Matrix.from_host(synth.uniform_rows(65536, 65536, 8, 11)).storage_format()[0] == "sell"
    assert spx.Matrix.from_host(synth.uniform_rows(16384, 16384, 4, 44)).storage_format()[0] == "ell"
    assert spx.Matrix.from_host(cfg_matrix("cfg1")).storage_format()[0] == "sell"
    assert spx.Matrix.from_host(cfg_matrix("rmat16")).storage_format()[0] == "csr5"
    assert spx.Matrix.from_host(synth.poisson3d(64, np.float32)).storage_format()[0] == "dia"
    assert spx.Matrix.from_host(cfg_matrix("cfg3")).storage_format()[0] == "dia"
    assert spx.Matrix.from_host(synth.powerlaw_rows(100_000, 50_000, 40.0, 31)).storage_format()[0] == "csr5"
    assert spx.Matrix.from_host(synth.rmat(18, 8, 5)).storage_format()[0] == "csr"


def test_sell_full_size_uniform_rows():
    """A full-size matrix the format tree sends to the sliced copy (2^20
    rows of 16 entries): run() on dense and sparse x against the oracle."""
    torch = _torch()
    A = synth.uniform_rows(1 << 20, 1 << 20, 16, 13)
    M = spx.Matrix.from_host(A)
    assert M.storage_format()[0] == "sell"
    x = synth.dense_vector(A.n, 14)
    ref, S = oracle.spmv(A, x.astype(np.float64))
    y = M.run(torch.as_tensor(x, device="cuda"))
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), ref, S, "f32", "uniform 2^20 dense x")
    v = synth.sparse_vector(A.n, A.n // 2, 15)
    ref, S = reference(A, v.idx, np.asarray(v.val, np.float32), "f32")
    y = M.run_plan((torch.as_tensor(v.idx, device="cuda"), torch.as_tensor(np.asarray(v.val, np.float32), device="cuda")),
                   spx.plan("spmv", "balanced"))
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), ref, S, "f32", "uniform 2^20 sparse x")


# ---------------------------------------------------------------- ELLPACK copy
@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
def test_ell_spmv_matches_oracle(kind):
    """The ELL copy (rows padded to the longest, a thread per row): every
    SpMV plan runs on it; ragged m, empty rows, dense and sparse x."""
    for name, A in _matrices():
        if name == "long_row":
            continue  # padding to its 1000-entry row exceeds the ELL limit (refusal tested below)
        A = _with_kind(A, kind)
        M = spx.Matrix.from_host(A, dtype=KINDS[kind][0], fmt="ell", renumber=False)
        fmt, ratio = M.storage_format()
        assert fmt == "ell", (name, fmt)
        lens = np.diff(np.asarray(A.row_ptr))
        assert ratio == pytest.approx(lens.max() * A.m / A.nnz, rel=1e-12), name
        _run_all(M, A, kind, f"ell {name}")


def test_ell_on_the_renumbered_copy_and_minplus():
    torch = _torch()
    A = synth.uniform_rows(70000, 70000, 6, 31)
    M = spx.Matrix.from_host(A, fmt="ell", renumber=True)
    assert M.column_order() is not None and M.storage_format()[0] == "ell"
    _run_all(M, A, "f32", "ell renumbered")
    B = synth.poisson3d(12, np.float32)
    W = np.abs(np.asarray(B.vals)) + 0.5
    Bm = B.with_vals(W.astype(np.float32))
    Mm = spx.Matrix.from_host(Bm, dtype=spx.F32_MINPLUS, fmt="ell")
    assert Mm.storage_format()[0] == "ell"
    d = np.full(B.n, np.inf, np.float32)
    d[::7] = np.random.default_rng(3).uniform(0, 4, len(d[::7])).astype(np.float32)
    ref = oracle.minplus_spmv(Bm, d)
    y = Mm.run_plan(torch.as_tensor(d, device="cuda"), spx.plan("spmv", "direct"))
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), ref)


def test_ell_follows_values_updated():
    torch = _torch()
    A = synth.poisson3d(24, np.float32)
    M = spx.Matrix.from_host(A, fmt="ell")
    new = np.random.default_rng(18).uniform(-2, 2, A.nnz).astype(np.float32)
    M.vals.copy_(torch.as_tensor(new, device="cuda"))
    M.values_updated()
    B = A.with_vals(new)
    x = synth.dense_vector(A.n, 19)
    ref, S = oracle.spmv(B, x.astype(np.float64))
    y = M.run_plan(torch.as_tensor(x, device="cuda"), spx.plan("spmv", "balanced"))
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), ref, S, "f32", "ell after update")


def test_ell_refused_when_padding_too_large():
    _torch()
    with pytest.raises(spx.SpxError) as e:
        spx.Matrix.from_host(cfg_matrix("rmat16"), fmt="ell")
    assert e.value.code == -5
    A = dict(_matrices())["long_row"]
    with pytest.raises(spx.SpxError) as e:
        spx.Matrix.from_host(A, fmt="ell")
    assert e.value.code == -5


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_ell_poisson_128_full_size(dt):
    """The 7-point Poisson matrix on 128^3 (2,097,152 rows) on the ELL copy:
    every row of A x for x ~ N(0, 1) against the oracle, and the closed form
    A 1 = 6 - (in-grid neighbours), exact."""
    torch = _torch()
    A = synth.cfg3_matrix(dt)
    M = spx.Matrix.from_host(A, fmt="ell")
    assert M.storage_format()[0] == "ell"
    xd, _ = synth.cfg3_vectors(dtype=dt)
    ref, S = oracle.spmv(A, np.asarray(xd, np.float64))
    y = M.run_plan(torch.as_tensor(np.asarray(xd, dt), device="cuda"), spx.plan("spmv", "direct"))
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), ref, S, "f32" if dt == np.float32 else "f64", "poisson 128^3 ell")
    ones = torch.ones(A.n, dtype=torch.float32 if dt == np.float32 else torch.float64, device="cuda")
    y1 = M.run_plan(ones, spx.plan("spmv", "direct")).cpu().numpy()
    want = np.asarray(A.vals, np.float64)
    want = np.add.reduceat(want, np.asarray(A.row_ptr[:-1]))
    assert np.array_equal(y1.astype(np.float64), want)
