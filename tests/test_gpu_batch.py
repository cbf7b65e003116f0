"""Batched SpMSpV (one graph-captured persistent launch, plans chosen on
the device) against the CPU oracle and against per-vector run()."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import assert_close, cfg_matrix, reference

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pack(vecs, kind, npdt):
    torch = _torch()
    ptr = np.zeros(len(vecs) + 1, np.int32)
    ptr[1:] = np.cumsum([v.nnz for v in vecs])
    idx = np.concatenate([v.idx for v in vecs]).astype(np.int32) if ptr[-1] else np.zeros(0, np.int32)
    val = None
    if kind != "bool":
        val = np.concatenate([np.asarray(v.val, npdt) for v in vecs]) if ptr[-1] else np.zeros(0, npdt)
    t = lambda a: torch.as_tensor(a, device="cuda")
    return t(ptr), t(idx), (None if val is None else t(val))


def _vectors(n, B, seed, kind, dense_frac=True):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(B):
        if b == 0:
            nnz = 0
        elif b == 1:
            nnz = n
        else:
            nnz = max(1, int(round(n * 10 ** rng.uniform(-4, np.log10(0.5)))))
        dist = "int" if kind == "i32" else "uniform"
        v = synth.sparse_vector(n, nnz, seed * 1000 + b, dist, np.int32 if kind == "i32" else np.float64)
        out.append(v)
    return out


@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
def test_batch_matches_oracle_small(kind):
    torch = _torch()
    npdt = {"f32": np.float32, "f64": np.float64, "i32": np.int32, "bool": None}[kind]
    code = {"f32": spx.F32, "f64": spx.F64, "i32": spx.I32, "bool": spx.BOOL}[kind]
    for name in ("cfg1", "rmat16"):
        A = cfg_matrix(name)
        if kind == "i32":
            A = A.with_vals(np.clip(np.round(A.vals * 4), -4, 4).astype(np.int32))
        elif npdt is not None:
            A = A.with_vals(A.vals.astype(npdt))
        M = spx.Matrix.from_host(A, dtype=code)
        vecs = _vectors(A.n, 40, 3, kind)
        ptr, idx, val = _pack(vecs, kind, npdt)
        Y = M.run_batch(ptr, idx, val)
        torch.cuda.synchronize()
        assert M.batch_status() == 0
        Yh = Y.cpu().numpy()
        for b, v in enumerate(vecs):
            ref, S = reference(A, v.idx, None if kind == "bool" else np.asarray(v.val, npdt), kind)
            assert_close(Yh[b], ref, S, kind, f"batch {name} {kind} b={b} nnz_x={v.nnz}")


def test_batch_graph_replays_and_recapture():
    """Replays of the captured graph, with eager work and syncs between
    them, each checked; new values in the same arrays; then different
    arrays (re-capture) and a larger batch (re-allocation)."""
    torch = _torch()
    A = cfg_matrix("rmat16")
    M = spx.Matrix.from_host(A)
    vecs = _vectors(A.n, 24, 5, "f32")
    ptr, idx, val = _pack(vecs, "f32", np.float32)
    Y = M.out_tensor(len(vecs))
    refs = [reference(A, v.idx, np.asarray(v.val, np.float32), "f32") for v in vecs]
    for rep in range(3):
        M.run_batch(ptr, idx, val, Y)
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy()
        for b in range(len(vecs)):
            assert_close(Yh[b], refs[b][0], refs[b][1], "f32", f"replay {rep} b={b}")
    # same arrays, new values (graph replay reads the new contents)
    val.mul_(-2.0)
    M.run_batch(ptr, idx, val, Y)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy()
    for b in range(len(vecs)):
        assert_close(Yh[b], -2.0 * refs[b][0], 2.0 * refs[b][1], "f32", f"new values b={b}")
    # different arrays and a larger batch
    vecs2 = _vectors(A.n, 50, 6, "f32")
    p2, i2, v2 = _pack(vecs2, "f32", np.float32)
    Y2 = M.run_batch(p2, i2, v2)
    torch.cuda.synchronize()
    Yh2 = Y2.cpu().numpy()
    for b, v in enumerate(vecs2):
        ref, S = reference(A, v.idx, np.asarray(v.val, np.float32), "f32")
        assert_close(Yh2[b], ref, S, "f32", f"recapture b={b}")
    assert M.batch_status() == 0


def _oracle_rows(A, vecs):
    """The oracle's column-scatter product (over its own transpose) for
    every vector: its cost follows nnz_s, so a whole batch takes seconds."""
    csc = oracle.transpose(A)
    for v in vecs:
        yield oracle.spmspv(csc, v.idx, np.asarray(v.val, np.float64))


@pytest.mark.slow
def test_batch_cfg4_rmat_matches_looped_run():
    """512 vectors of log-uniform density on R-MAT 2^18 (degree 32): every
    row of the batched result and every per-vector run() result is within
    the FP32 bound of the oracle (so the two agree within twice the bound)."""
    torch = _torch()
    A = cfg_matrix("cfg4_rmat")
    M = spx.Matrix.from_host(A)
    vecs = synth.cfg4_rmat_batch(A.n, 512)
    ptr, idx, val = _pack(vecs, "f32", np.float32)
    Y = M.run_batch(ptr, idx, val)
    torch.cuda.synchronize()
    assert M.batch_status() == 0
    Yh = Y.cpu().numpy()
    Yl = M.out_tensor(len(vecs))
    hp = ptr.cpu().numpy()
    for b in range(len(vecs)):
        M.run((idx[hp[b]:hp[b + 1]], val[hp[b]:hp[b + 1]]), Yl[b])
    Ylh = Yl.cpu().numpy()
    for b, (ref, S) in enumerate(_oracle_rows(A, vecs)):
        nx = vecs[b].nnz
        assert_close(Yh[b], ref, S, "f32", f"cfg4 rmat batched b={b} nnz_x={nx}")
        assert_close(Ylh[b], ref, S, "f32", f"cfg4 rmat looped run() b={b} nnz_x={nx}")


@pytest.mark.slow
def test_batch_cfg4_svm_rows():
    """256 rows of the 100k x 50k power-law matrix as sparse x against the
    same matrix: every batched row and every looped run() row against the
    oracle."""
    torch = _torch()
    A = cfg_matrix("cfg4_svm")
    M = spx.Matrix.from_host(A)
    vecs = synth.cfg4_svm_batch(A, 256)
    ptr, idx, val = _pack(vecs, "f32", np.float32)
    Y = M.run_batch(ptr, idx, val)
    torch.cuda.synchronize()
    assert M.batch_status() == 0
    Yh = Y.cpu().numpy()
    Yl = M.out_tensor(len(vecs))
    hp = ptr.cpu().numpy()
    for b in range(len(vecs)):
        M.run((idx[hp[b]:hp[b + 1]], val[hp[b]:hp[b + 1]]), Yl[b])
    Ylh = Yl.cpu().numpy()
    for b, (ref, S) in enumerate(_oracle_rows(A, vecs)):
        assert_close(Yh[b], ref, S, "f32", f"cfg4 svm batched b={b}")
        assert_close(Ylh[b], ref, S, "f32", f"cfg4 svm looped run() b={b}")


@pytest.mark.parametrize("kind", ["f32", "f64", "i32"])
def test_batch_fused_groups(kind):
    """Dense-enough vectors share passes over A in groups of 64: three
    groups (the last partial), hub rows cut into pieces (R-MAT), empty rows
    and a ragged row count, next to sparse vectors on per-vector plans."""
    torch = _torch()
    npdt = {"f32": np.float32, "f64": np.float64, "i32": np.int32}[kind]
    code = {"f32": spx.F32, "f64": spx.F64, "i32": spx.I32}[kind]
    rng = np.random.default_rng(11)
    for name, A in (("rmat16", cfg_matrix("rmat16")),
                    ("ragged", synth.random_csr(3001, 2503, 0.01, 77, empty_rows=0.3))):
        if kind == "i32":
            A = A.with_vals(np.clip(np.round(np.asarray(A.vals) * 4), -4, 4).astype(np.int32))
        else:
            A = A.with_vals(np.asarray(A.vals).astype(npdt))
        M = spx.Matrix.from_host(A, dtype=code)
        dens = np.concatenate([10 ** rng.uniform(-1.7, 0, 150), 10 ** rng.uniform(-4, -2.5, 20)])
        dens[0], dens[1] = 1.0, 0.5
        vecs = []
        for b, d in enumerate(dens):
            nnz = max(1, int(round(A.n * d)))
            dist = "int" if kind == "i32" else "uniform"
            vecs.append(synth.sparse_vector(A.n, nnz, 7000 + b, dist, np.int32 if kind == "i32" else np.float64))
        ptr, idx, val = _pack(vecs, kind, npdt)
        Y = M.run_batch(ptr, idx, val)
        torch.cuda.synchronize()
        assert M.batch_status() == 0
        Yh = Y.cpu().numpy()
        for b in range(len(vecs)):
            v = vecs[b]
            ref, S = reference(A, v.idx, np.asarray(v.val, npdt), kind)
            assert_close(Yh[b], ref, S, kind, f"fused {name} {kind} b={b} nnz_x={v.nnz}")
        # a second run on the same arrays: the group slabs were cleared
        Y2 = M.run_batch(ptr, idx, val).cpu().numpy()
        for b in (0, 1, 64, 149):
            v = vecs[b]
            ref, S = reference(A, v.idx, np.asarray(v.val, npdt), kind)
            assert_close(Y2[b], ref, S, kind, f"fused rerun {name} {kind} b={b}")


@pytest.mark.parametrize("kind", ["f32", "f64", "i32"])
def test_batch_fused_groups_with_unsorted_members(kind):
    """Fused groups take their members' entries in any order. Three runs
    on the same arrays (one captured graph): all ascending, one vector's
    entries shuffled in place, ascending again; every row checked on every
    run, so a slab or a split row of Y left dirty by one run shows up in the
    next."""
    torch = _torch()
    npdt = {"f32": np.float32, "f64": np.float64, "i32": np.int32}[kind]
    code = {"f32": spx.F32, "f64": spx.F64, "i32": spx.I32}[kind]
    A = cfg_matrix("rmat16")
    if kind == "i32":
        A = A.with_vals(np.clip(np.round(np.asarray(A.vals) * 4), -4, 4).astype(np.int32))
    else:
        A = A.with_vals(np.asarray(A.vals).astype(npdt))
    M = spx.Matrix.from_host(A, dtype=code)
    rng = np.random.default_rng(13)
    dist = "int" if kind == "i32" else "uniform"
    vecs = [synth.sparse_vector(A.n, max(1, int(round(A.n * d))), 8000 + b, dist,
                                np.int32 if kind == "i32" else np.float64)
            for b, d in enumerate(10 ** rng.uniform(-1.5, -0.3, 130))]
    ptr, idx, val = _pack(vecs, kind, npdt)
    hp = ptr.cpu().numpy()
    idx_sorted, val_sorted = idx.clone(), val.clone()
    refs = [reference(A, v.idx, np.asarray(v.val, npdt), kind) for v in vecs]
    for run in range(3):
        if run == 1:
            s0, s1 = int(hp[70]), int(hp[71])
            perm = torch.as_tensor(np.random.default_rng(14).permutation(s1 - s0), device="cuda")
            idx[s0:s1] = idx_sorted[s0:s1][perm]
            val[s0:s1] = val_sorted[s0:s1][perm]
        elif run == 2:
            idx.copy_(idx_sorted)
            val.copy_(val_sorted)
        Y = M.run_batch(ptr, idx, val)
        torch.cuda.synchronize()
        assert M.batch_status() == 0
        Yh = Y.cpu().numpy()
        for b, (ref, S) in enumerate(refs):
            assert_close(Yh[b], ref, S, kind, f"unsorted members run {run} {kind} b={b} nnz_x={vecs[b].nnz}")


def _one_per_row(m, n, seed):
    """m rows of one entry each in a random column: columns average m / n
    entries, many are empty."""
    rng = np.random.default_rng(seed)
    rp = np.arange(m + 1, dtype=np.int32)
    ci = rng.integers(0, n, m).astype(np.int32)
    return synth.CSR(m, n, rp, ci, rng.uniform(-1, 1, m).astype(np.float32))


@pytest.mark.parametrize("kind", ["f32", "f64", "i32", "bool"])
def test_batch_column_major_write_backs(kind):
    """Sparse vectors (below the fused-group density) on column-major plans,
    where the columns are long (R-MAT 2^15, hub columns) and where they are
    short (200,000 rows of one entry, two per column on average, many
    columns empty). Empty vectors and a support of empty columns included;
    every row is checked, on two runs (the second reuses the zero fill of
    Y and the queue heads)."""
    torch = _torch()
    npdt = {"f32": np.float32, "f64": np.float64, "i32": np.int32, "bool": None}[kind]
    code = {"f32": spx.F32, "f64": spx.F64, "i32": spx.I32, "bool": spx.BOOL}[kind]
    rng = np.random.default_rng(12)
    for name, A in (("rmat15", synth.rmat(15, 16, 23)), ("one_per_row", _one_per_row(200_000, 100_000, 24))):
        if kind == "i32":
            A = A.with_vals(np.clip(np.round(np.asarray(A.vals) * 4), -4, 4).astype(np.int32))
        elif npdt is not None:
            A = A.with_vals(np.asarray(A.vals).astype(npdt))
        M = spx.Matrix.from_host(A, dtype=code)
        dist = "int" if kind == "i32" else "uniform"
        vecs = [synth.SparseVec(A.n, np.zeros(0, np.int32), np.zeros(0, np.float64))]
        empty_cols = np.nonzero(np.bincount(A.col_idx, minlength=A.n) == 0)[0]
        if empty_cols.size:
            vecs.append(synth.SparseVec(A.n, empty_cols[:5].astype(np.int32), np.ones(min(5, empty_cols.size))))
        for b, d in enumerate(10 ** rng.uniform(-4, -2.2, 40)):
            nnz = max(1, int(round(A.n * d)))
            vecs.append(synth.sparse_vector(A.n, nnz, 9000 + b, dist, np.int32 if kind == "i32" else np.float64))
        ptr, idx, val = _pack(vecs, kind, npdt)
        for rep in range(2):
            Y = M.run_batch(ptr, idx, val)
            torch.cuda.synchronize()
            assert M.batch_status() == 0
            Yh = Y.cpu().numpy()
            for b, v in enumerate(vecs):
                ref, S = reference(A, v.idx, None if kind == "bool" else np.asarray(v.val, npdt), kind)
                assert_close(Yh[b], ref, S, kind, f"column-major {name} {kind} run {rep} b={b} nnz_x={v.nnz}")


@pytest.mark.parametrize("B,n", [(1, 1), (3, 100), (2, 2049), (64, 4096), (1, 1 << 20)])
def test_dense_rows_to_sparse(B, n):
    """Compaction of dense rows (long rows span many workgroups): indices in
    order and values exactly as numpy's nonzero finds them; -0.0 is a zero,
    NaN a nonzero; empty rows keep an empty range."""
    torch = _torch()
    rng = np.random.default_rng(B * 7 + n)
    X = rng.standard_normal((B, n)).astype(np.float32)
    X[rng.random((B, n)) < 0.7] = 0.0
    X[0, :: max(1, n // 5)] = -0.0
    if n > 3:
        X[0, 3] = np.nan
    if B > 1:
        X[1] = 0.0
    A = synth.random_csr(4, n, 0.5, 1)
    M = spx.Matrix.from_host(A)
    vp, idx, val = M.dense_rows_to_sparse(torch.as_tensor(X, device="cuda"))
    vp, idx, val = vp.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()
    assert vp[0] == 0
    for b in range(B):
        nz = np.nonzero(X[b] != 0)[0]  # NaN != 0 holds, -0.0 != 0 does not
        assert np.array_equal(idx[vp[b]:vp[b + 1]], nz)
        got, want = val[vp[b]:vp[b + 1]], X[b, nz]
        assert np.array_equal(np.isnan(got), np.isnan(want))
        assert np.array_equal(got[~np.isnan(got)], want[~np.isnan(want)])
