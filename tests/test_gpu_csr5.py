"""The CSR5 copy (the fourth storage format of the pre-selection): every
SpMV plan on a handle that keeps it runs on it (the other patterns keep
their kernels, checked here on the same handles). Parity with the oracle's
SpMV for every dtype on dense and sparse x, over shapes that stress the tile
logic: rows that cross lanes and tiles, rows of exactly a lane or a tile,
empty rows first, last and in runs, a row spanning hundreds of tiles, no
entries at all, one row; the renumbered copy, min-plus bit for bit, a value
refresh, and repeatable bits."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close, cfg_matrix, reference

pytestmark = pytest.mark.gpu

KINDS = {"f32": (spx.F32, np.float32), "f64": (spx.F64, np.float64), "i32": (spx.I32, np.int32),
         "bool": (spx.BOOL, None)}
SPMV_PLANS = [spx.plan("spmv", "direct"), spx.plan("spmv", "balanced")]
# the bitvector SpMSpV on the same handles: consecutive calls with other
# supports check the bitvector and value buffers left clean between calls
PLANS = SPMV_PLANS + [spx.plan("csr_spmspv", "balanced"), spx.plan("csr_spmspv", "direct")]
TILE = 1024  # 64 lanes x 16 entries


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _from_lengths(lens, n, seed):
    lens = np.asarray(lens, np.int64)
    rng = np.random.default_rng(seed)
    rp = np.zeros(len(lens) + 1, np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(rng.choice(n, size=int(k), replace=False)) for k in lens] or
                        [np.zeros(0, np.int64)]).astype(np.int32)
    vals = rng.uniform(-1, 1, ci.size).astype(np.float32)
    return synth.CSR(len(lens), n, rp, ci, vals)


def _with_kind(A, kind):
    if kind == "i32":
        return A.with_vals(np.clip(np.round(np.asarray(A.vals) * 4), -4, 4).astype(np.int32))
    if kind in ("f32", "f64"):
        return A.with_vals(np.asarray(A.vals).astype(KINDS[kind][1]))
    return A


def _matrices():
    rng = np.random.default_rng(71)
    return [
        ("cfg1", cfg_matrix("cfg1")),
        ("poisson24", synth.poisson3d(24, np.float32)),
        # empty rows first, last and in runs; rows of 16 (a lane) and 1024 (a tile)
        ("edges", _from_lengths([0, 0, 3, 16, 0, 1024, 17, 0, 0, 1, 1023, 1025, 15, 0] * 9 + [0, 0], 4000, 72)),
        ("ragged", synth.random_csr(3001, 2503, 0.004, 91, empty_rows=0.2)),
        ("short_rows", _from_lengths(rng.integers(0, 3, 20000), 5000, 73)),
        ("one_row", _from_lengths([777], 1000, 74)),
        ("hub", synth.hub_matrix(70000, 60000, 3, 75)),
    ]


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
            for p in PLANS:
                y = M.run_plan(x, p)
                torch.cuda.synchronize()
                assert_close(y.cpu().numpy(), ref, S, kind, f"{tag} {kind} nnz_x={nnz_x} {p}")


@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
def test_csr5_spmv_matches_oracle(kind):
    _torch()
    for name, A0 in _matrices():
        A = _with_kind(A0, kind)
        M = spx.Matrix.from_host(A, dtype=KINDS[kind][0], fmt="csr5", renumber=False)
        fmt, ratio = M.storage_format()
        tiles = -(-A.nnz // TILE)
        assert fmt == "csr5" and ratio == pytest.approx(tiles * TILE / max(1, A.nnz), rel=1e-12), (name, fmt, ratio)
        _run_all(M, A, kind, f"csr5 {name}")


def test_csr5_without_entries_writes_zeros():
    torch = _torch()
    A = synth.CSR(300, 50, np.zeros(301, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    M = spx.Matrix.from_host(A, fmt="csr5", renumber=False)
    assert M.storage_format()[0] == "csr5"
    x = torch.ones(A.n, device="cuda")
    y = torch.full((A.m,), 7.0, device="cuda")
    M.run_plan(x, spx.plan("spmv", "balanced"), y)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), np.zeros(A.m, np.float32))


def test_csr5_on_the_renumbered_copy():
    _torch()
    A = _with_kind(synth.rmat(17, 8, 22), "f32")
    M = spx.Matrix.from_host(A, fmt="csr5", renumber=True)
    assert M.column_order() is not None and M.storage_format()[0] == "csr5"
    _run_all(M, A, "f32", "csr5 renumbered")


def test_csr5_minplus_bit_exact():
    torch = _torch()
    A = _from_lengths(np.random.default_rng(76).integers(0, 40, 5000), 3000, 77)
    A = A.with_vals(np.random.default_rng(3).uniform(-1, 1, A.nnz).astype(np.float32))
    M = spx.Matrix.from_host(A, dtype=spx.F32_MINPLUS, fmt="csr5", renumber=False)
    assert M.storage_format()[0] == "csr5"
    xd = np.random.default_rng(4).uniform(-1, 1, A.n).astype(np.float32)
    xd[np.random.default_rng(5).random(A.n) < 0.5] = np.inf
    want = oracle.minplus_spmv(A, xd)
    for p in SPMV_PLANS:
        got = M.run_plan(torch.as_tensor(xd, device="cuda"), p).cpu().numpy()
        assert np.array_equal(got, want), p


def test_csr5_follows_values_updated_and_repeats_its_bits():
    torch = _torch()
    A = synth.rmat(15, 16, 78)
    M = spx.Matrix.from_host(A, fmt="csr5")
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


def test_csr5_long_row_meets_the_fp32_bound():
    """A row of 2^19 positive products spans 512 tiles: the per-tile
    partials are added 64 at a time by a tree, so the row stays within the
    1e-5 * sum |a x| bound that one serial FP32 chain misses."""
    torch = _torch()
    N = (1 << 19) + 8192
    A = synth.hub_matrix(N, 1 << 19, 4, 31)
    x = np.random.default_rng(32).uniform(0.0, 1.0, A.n).astype(np.float32)
    M = spx.Matrix.from_host(A, fmt="csr5", renumber=False)
    ref, S = oracle.spmv(A, x.astype(np.float64))
    y = M.run_plan(torch.as_tensor(x, device="cuda"), spx.plan("spmv", "balanced"))
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), ref, S, "f32", "hub row")


def test_format_flags_exclude_each_other():
    import ctypes as C
    torch = _torch()
    A = synth.poisson3d(8, np.float32)
    rp, ci, v = (torch.as_tensor(a, device="cuda") for a in (A.row_ptr, A.col_idx, A.vals))
    csr = spx._lib.Csr(A.m, A.n, A.nnz, spx.F32, rp.data_ptr(), ci.data_ptr(), v.data_ptr())
    lib = spx._lib.load()
    for flags in (spx.FORMAT_CSR5 | spx.FORMAT_ELL, spx.FORMAT_CSR5 | spx.FORMAT_SELL):
        out = C.c_void_p()
        assert lib.spx_matrix_create(C.byref(csr), flags, None, C.byref(out)) == -1
        assert not out.value
