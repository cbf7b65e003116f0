"""Shared helpers of the GPU parity tests: device upload of the seeded
inputs, the oracle reference for a given vector, and the comparison rule
for each value type."""
from __future__ import annotations

import functools

import numpy as np

import oracle
from paper_2006_16767_amd import synth

FP32_TOL = 1e-5   # |y - ref| <= 1e-5 * sum |a_ij x_j|
FP64_TOL = 1e-12


def torch():
    import torch as t
    return t


def dev_sparse(v, dtype=None):
    t = torch()
    idx = t.as_tensor(v.idx, dtype=t.int32, device="cuda")
    val = None
    if v.val is not None and dtype is not None:
        val = t.as_tensor(np.asarray(v.val).astype(dtype), device="cuda")
    return idx, val


def reference(A, v_idx, v_val, kind: str):
    """Oracle y (and S) for a sparse x given as (idx, val); kind in
    f32/f64/i32/bool. The oracle computes SpMV on the zero-filled x; the
    column-scatter form is pinned equal to it on the CPU."""
    if kind == "bool":
        return oracle.bool_spmspv(A, v_idx), None
    xd = np.zeros(A.n, dtype=np.float64 if kind != "i32" else np.int32)
    if len(v_idx):
        xd[np.asarray(v_idx)] = v_val
    if kind == "i32":
        return oracle.int_spmv(A, xd), None
    return oracle.spmv(A, xd)


def assert_close(y, ref, S, kind: str, what: str = ""):
    y = np.asarray(y)
    if kind in ("bool", "i32"):
        bad = np.nonzero(y.astype(np.int64) != np.asarray(ref).astype(np.int64))[0]
        assert bad.size == 0, f"{what}: {bad.size} mismatches, first rows {bad[:5]} got {y[bad[:5]]} want {np.asarray(ref)[bad[:5]]}"
        return
    tol = FP32_TOL if kind == "f32" else FP64_TOL
    y64 = y.astype(np.float64)
    err = np.abs(y64 - ref)
    zero_rows = S == 0
    assert np.all(y64[zero_rows] == 0), f"{what}: rows with no effective entry must be exactly 0"
    lim = tol * S
    bad = np.nonzero(err > lim)[0]
    if bad.size:
        i = bad[np.argmax((err[bad] / np.maximum(S[bad], 1e-300)))]
        raise AssertionError(f"{what}: {bad.size} rows over {tol}*S; worst row {i}: got {y64[i]!r} "
                             f"want {ref[i]!r} S={S[i]!r} rel={err[i] / S[i]:.3e}")


@functools.lru_cache(maxsize=None)
def cfg_matrix(name: str):
    if name == "cfg1":
        return synth.cfg1_matrix()
    if name == "cfg2":
        return synth.cfg2_matrix()
    if name == "cfg3":
        return synth.cfg3_matrix()
    if name == "cfg3_f64":
        return synth.cfg3_matrix(np.float64)
    if name == "cfg4_rmat":
        return synth.cfg4_rmat()
    if name == "cfg4_svm":
        return synth.cfg4_svm()
    if name == "cfg5":
        return synth.cfg5_matrix()
    if name == "rmat16":
        return synth.rmat(16, 16, 777)
    raise KeyError(name)
