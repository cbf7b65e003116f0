"""The diagonal (DIA) copy of the storage-format pre-selection: every SpMV
plan on a handle that keeps it runs on it. Parity with the oracle's SpMV for
the value types it takes, on banded shapes that stress its cells: diagonals
with holes, rectangular matrices whose diagonals end early, the two corner
diagonals, empty rows, a single row, a diagonal as long as a row span; the
automatic choice and its refusals, min-plus bit for bit (cells without an
entry take no part, also against an infinite x), a value refresh, and the
full-size Poisson matrix."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close, cfg_matrix, reference

pytestmark = pytest.mark.gpu

KINDS = {"f32": (spx.F32, np.float32), "f64": (spx.F64, np.float64), "i32": (spx.I32, np.int32)}
SPMV_PLANS = [spx.plan("spmv", "direct"), spx.plan("spmv", "balanced")]
# another pattern on the same handles keeps its own kernels
PLANS = SPMV_PLANS + [spx.plan("csr_spmspv", "balanced")]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _banded(m, n, offsets, hole, seed, empty_rows=()):
    """Entries (i, i + o) for every offset o that lands in [0, n), each kept
    with probability 1 - hole; the listed rows left empty."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for o in sorted(offsets):
        i = np.arange(max(0, -o), min(m, n - o))
        keep = rng.random(i.size) >= hole
        rows.append(i[keep])
        cols.append(i[keep] + o)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    drop = np.isin(r, np.asarray(empty_rows, np.int64))
    r, c = r[~drop], c[~drop]
    order = np.lexsort((c, r))
    r, c = r[order], c[order]
    rp = np.zeros(m + 1, np.int32)
    np.add.at(rp, r + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    vals = rng.uniform(-1, 1, r.size).astype(np.float32)
    return synth.CSR(m, n, rp, c.astype(np.int32), vals)


def _with_kind(A, kind):
    if kind == "i32":
        return A.with_vals(np.clip(np.round(np.asarray(A.vals) * 4), -4, 4).astype(np.int32))
    return A.with_vals(np.asarray(A.vals).astype(KINDS[kind][1]))


def _matrices():
    return [
        ("poisson24", synth.poisson3d(24, np.float32)),
        ("tridiagonal_holes", _banded(5000, 5000, (-1, 0, 1), 0.3, 61)),
        ("rectangular", _banded(3000, 4500, (-2, 0, 5, 1200), 0.1, 62)),
        ("corners", _banded(2000, 2000, (-1999, 0, 1999), 0.0, 63)),
        ("empty_rows", _banded(4096, 4096, (-64, -1, 0, 1, 64), 0.05, 64, empty_rows=(0, 1, 700, 701, 4095))),
        ("one_row", _banded(1, 40, (0, 3, 17, 39), 0.0, 65)),
        ("tall", _banded(9000, 300, (0, -8000, -4500), 0.2, 66)),
    ]


def _run_all(M, A, kind, tag):
    torch = _torch()
    code, npdt = KINDS[kind]
    rng = np.random.default_rng(5)
    for nnz_x in sorted({0, 1, max(1, A.n // 10), A.n}):
        v = synth.sparse_vector(A.n, nnz_x, 900 + nnz_x)
        val = rng.integers(-5, 6, size=v.nnz).astype(np.int32) if kind == "i32" else np.asarray(v.val).astype(npdt)
        ref, S = reference(A, v.idx, val, kind)
        xd = np.zeros(A.n, dtype=npdt)
        xd[v.idx] = val
        xs = [torch.as_tensor(xd, device="cuda"), (torch.as_tensor(v.idx, device="cuda"), torch.as_tensor(val, device="cuda"))]
        for x in xs:
            for p in PLANS:
                y = M.run_plan(x, p)
                torch.cuda.synchronize()
                assert_close(y.cpu().numpy(), ref, S, kind, f"{tag} {kind} nnz_x={nnz_x} {p}")


@pytest.mark.parametrize("kind", ["f32", "f64", "i32"])
def test_dia_spmv_matches_oracle(kind):
    _torch()
    for name, A0 in _matrices():
        A = _with_kind(A0, kind)
        M = spx.Matrix.from_host(A, dtype=KINDS[kind][0], fmt="dia", renumber=False)
        fmt, ratio = M.storage_format()
        ndiag = len(np.unique(np.asarray(A.col_idx, np.int64) - np.repeat(np.arange(A.m), np.diff(A.row_ptr))))
        assert fmt == "dia" and ratio == pytest.approx(ndiag * A.m / A.nnz, rel=1e-12), (name, fmt, ratio, ndiag)
        _run_all(M, A, kind, f"dia {name}")


def test_dia_chosen_only_where_it_applies():
    _torch()
    assert spx.Matrix.from_host(synth.poisson3d(32, np.float32)).storage_format()[0] == "dia"
    assert spx.Matrix.from_host(_banded(5000, 5000, (-1, 0, 1), 0.3, 61)).storage_format()[0] == "dia"
    # random rows, Boolean values, too many diagonals, too many holes: no DIA copy
    assert spx.Matrix.from_host(cfg_matrix("cfg1")).storage_format()[0] != "dia"
    assert spx.Matrix.from_host(synth.poisson3d(32, np.float32), dtype=spx.BOOL).storage_format()[0] != "dia"
    wide = _banded(4096, 4096, tuple(range(-20, 21)), 0.0, 67)
    assert spx.Matrix.from_host(wide).storage_format()[0] != "dia"
    sparse_band = _banded(4096, 4096, (-3, 0, 3), 0.8, 68)
    assert spx.Matrix.from_host(sparse_band).storage_format()[0] != "dia"


def test_dia_refusals():
    import ctypes as C
    torch = _torch()
    for A, dt in ((synth.poisson3d(8, np.float32), spx.BOOL), (_banded(4096, 4096, tuple(range(-20, 21)), 0.0, 67), spx.F32),
                  (cfg_matrix("cfg1"), spx.F32)):
        with pytest.raises(spx.SpxError) as e:
            spx.Matrix.from_host(A, dtype=dt, fmt="dia")
        assert e.value.code == -5
    A = synth.poisson3d(8, np.float32)
    rp, ci, v = (torch.as_tensor(a, device="cuda") for a in (A.row_ptr, A.col_idx, A.vals))
    csr = spx._lib.Csr(A.m, A.n, A.nnz, spx.F32, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
    lib = spx._lib.load()
    for flags in (spx.FORMAT_DIA | spx.FORMAT_ELL, spx.FORMAT_DIA | spx.FORMAT_CSR5):
        out = C.c_void_p()
        assert lib.spx_matrix_create(C.byref(csr), flags, None, C.byref(out)) == -1
        assert not out.value


def test_dia_minplus_bit_exact():
    torch = _torch()
    for A in (synth.poisson3d(16, np.float32), _banded(3000, 4500, (-2, 0, 5, 1200), 0.1, 62)):
        A = A.with_vals(np.random.default_rng(3).uniform(-1, 1, A.nnz).astype(np.float32))
        M = spx.Matrix.from_host(A, dtype=spx.F32_MINPLUS, renumber=False)
        assert M.storage_format()[0] == "dia"
        xd = np.random.default_rng(4).uniform(-1, 1, A.n).astype(np.float32)
        xd[np.random.default_rng(5).random(A.n) < 0.5] = np.inf
        want = oracle.minplus_spmv(A, xd)
        for p in SPMV_PLANS:
            got = M.run_plan(torch.as_tensor(xd, device="cuda"), p).cpu().numpy()
            assert np.array_equal(got, want), p


def test_dia_follows_values_updated_and_repeats_its_bits():
    torch = _torch()
    A = synth.poisson3d(24, np.float32)
    M = spx.Matrix.from_host(A)
    assert M.storage_format()[0] == "dia"
    new = np.random.default_rng(8).uniform(-2, 2, A.nnz).astype(np.float32)
    M.vals.copy_(torch.as_tensor(new, device="cuda"))
    M.values_updated()
    B = A.with_vals(new)
    x = synth.dense_vector(A.n, 9)
    ref, S = oracle.spmv(B, x.astype(np.float64))
    xt = torch.as_tensor(x, device="cuda")
    y0 = M.run_plan(xt, spx.plan("spmv", "balanced")).cpu().numpy()
    assert_close(y0, ref, S, "f32", "after update")
    for _ in range(3):
        y1 = M.run_plan(xt, spx.plan("spmv", "balanced")).cpu().numpy()
        assert np.array_equal(y0.view(np.uint32), y1.view(np.uint32))


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_dia_poisson_128_full_size(dt):
    """The 128^3 Poisson matrix (14.6M entries on 7 diagonals) through run():
    every row against the oracle."""
    torch = _torch()
    A = cfg_matrix("cfg3")
    npdt = KINDS[dt][1]
    A = A.with_vals(np.asarray(A.vals).astype(npdt))
    M = spx.Matrix.from_host(A, dtype=KINDS[dt][0])
    assert M.storage_format()[0] == "dia"
    x = synth.dense_vector(A.n, 17).astype(npdt)
    ref, S = oracle.spmv(A, x.astype(np.float64))
    y = M.run(torch.as_tensor(x, device="cuda"))
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), ref, S, dt, f"poisson128 {dt}")
