"""Sparse-output SpMSpV with a complement mask against the oracle: the
listed rows are unique (compared exactly after sorting); values follow the
tolerance of their semiring. Both bucket forms run: the one-launch walk
(short x, direct distribution) and the scatter + accumulate pair."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close, cfg_matrix

pytestmark = pytest.mark.gpu

KIND = {"f32": np.float32, "f64": np.float64, "i32": np.int32, "bool": None}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _as(A, kind):
    if kind == "bool":
        return A.with_vals(None) if hasattr(A, "with_vals") else A
    if kind == "i32":
        rng = np.random.default_rng(5)
        return A.with_vals(rng.integers(-4, 5, A.nnz).astype(np.int32))
    return A.with_vals(np.asarray(A.vals).astype(KIND[kind]))


def _x(n, nnz, kind, seed):
    v = synth.sparse_vector(n, nnz, seed)
    if kind == "bool":
        return v.idx, None
    if kind == "i32":
        return v.idx, np.random.default_rng(seed).integers(-4, 5, v.nnz).astype(np.int32)
    return v.idx, np.asarray(v.val).astype(KIND[kind])


def _check(M, A, kind, idx, val, mask, plan):
    torch = _torch()
    x = (torch.as_tensor(idx, device="cuda"), None if val is None else torch.as_tensor(val, device="cuda"))
    tmask = None if mask is None else torch.as_tensor(mask, device="cuda")
    rows, vals = M.spmspv_sparse(x, mask=tmask, plan=plan)
    rows = rows.cpu().numpy()
    order = np.argsort(rows)
    rows = rows[order]
    okind = {"f32": "f64", "f64": "f64", "i32": "i32", "bool": "bool"}[kind]
    want_rows, want_vals, S = oracle.spmspv_sparse(A, idx, None if val is None else val.astype(
        np.float64 if okind == "f64" else np.int32), mask=mask, kind=okind)
    assert np.array_equal(rows, want_rows), (kind, plan, len(rows), len(want_rows))
    got = vals.cpu().numpy()[order]
    if kind in ("i32", "bool"):
        assert np.array_equal(got.astype(np.int64), want_vals.astype(np.int64))
    else:
        assert_close(got, want_vals, S, kind, f"sparse output {plan}")
    return want_rows


PLANS = [None, spx.plan("csc_spmspv", "direct", "bucket"), spx.plan("csc_spmspv", "balanced", "bucket")]


@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
@pytest.mark.parametrize("name", ["cfg1", "rmat16"])
def test_sparse_output_matches_oracle(name, kind):
    _torch()
    A = _as(cfg_matrix(name), kind)
    M = spx.Matrix.from_host(A, dtype=spx.BOOL if kind == "bool" else None)
    rng = np.random.default_rng(11)
    for nnz in (1, 7, 300, 3000):  # short x takes the walk under the direct plan
        idx, val = _x(A.n, nnz, kind, 100 + nnz)
        for mask in (None, rng.random(A.m) < 0.3):
            for plan in PLANS:
                _check(M, A, kind, idx, val, mask, plan)


def test_sparse_output_edge_cases():
    torch = _torch()
    A = cfg_matrix("cfg1")
    M = spx.Matrix.from_host(A)
    # empty x: nothing listed
    rows, vals = M.spmspv_sparse((torch.zeros(0, dtype=torch.int32, device="cuda"),
                                  torch.zeros(0, dtype=torch.float32, device="cuda")))
    assert rows.numel() == 0 and vals.numel() == 0
    # every row masked
    idx, val = _x(A.n, 500, "f32", 3)
    x = (torch.as_tensor(idx, device="cuda"), torch.as_tensor(val, device="cuda"))
    rows, _ = M.spmspv_sparse(x, mask=torch.ones(A.m, dtype=torch.bool, device="cuda"))
    assert rows.numel() == 0
    # a row reached only by entries that cancel is still listed (structural)
    B = synth._coo_to_csr(3, 2, np.array([0, 0, 1]), np.array([0, 1, 1]), np.array([1.0, -1.0, 2.0], np.float32))
    MB = spx.Matrix.from_host(B)
    x = (torch.tensor([0, 1], dtype=torch.int32, device="cuda"), torch.tensor([1.0, 1.0], device="cuda"))
    rows, vals = MB.spmspv_sparse(x)
    order = torch.argsort(rows)
    assert rows[order].tolist() == [0, 1] and vals[order].tolist() == [0.0, 2.0]
    # values can be skipped; a dense x is refused
    rows2, none = M.spmspv_sparse((torch.as_tensor(idx, device="cuda"), torch.as_tensor(val, device="cuda")),
                                  with_values=False)
    assert none is None and rows2.numel() > 0
    with pytest.raises(spx.SpxError) as e:
        M.spmspv_sparse(torch.zeros(A.n, device="cuda"))
    assert e.value.code == -1
    with pytest.raises(spx.SpxError) as e:
        M.spmspv_sparse((torch.as_tensor(idx, device="cuda"), torch.as_tensor(val, device="cuda")),
                        plan=spx.plan("csc_spmspv", "direct", "atomic"))
    assert e.value.code == -1


def test_sparse_output_full_size_rmat20():
    """R-MAT 2^20 at the sweep's sparse densities, against the oracle with
    a mask of the rows the previous vector reached (frontier chaining)."""
    torch = _torch()
    A = cfg_matrix("cfg2")
    M = spx.Matrix.from_host(A)
    vecs = synth.cfg2_vectors(A.n)
    prev = None
    for v in vecs[:9]:
        mask = None
        if prev is not None:
            mask = np.zeros(A.m, bool)
            mask[prev] = True
        listed = _check(M, A, "f32", v.idx, np.asarray(v.val, np.float32), mask, None)
        prev = listed if mask is None else np.union1d(listed, prev)


@pytest.mark.parametrize("m", [1, 31, 32, 33, 64, 65, 1000, 4097])
def test_pack_mask_matches_bit_definition(m):
    """spx_pack_mask: bit i of word i // 32 is rows[i] != 0, high bits of the
    last word clear (numpy's little-endian bit packing as the definition)."""
    torch = _torch()
    rng = np.random.default_rng(16767 + m)
    A = synth.uniform_rows(m, 8, 1, 3)
    M = spx.Matrix.from_host(A.with_vals(np.asarray(A.vals).astype(np.float32)))
    rows = rng.integers(0, 4, m).astype(np.uint8)  # any nonzero byte sets the bit
    want = np.packbits(rows != 0, bitorder="little")
    want = np.concatenate([want, np.zeros((-len(want)) % 4, np.uint8)]).view("<u4")
    for t in (torch.as_tensor(rows, device="cuda"), torch.as_tensor(rows != 0, device="cuda")):
        got = M.pack_mask(t).cpu().numpy().view(np.uint32)
        assert np.array_equal(got[:len(want)], want[:(m + 31) // 32])
