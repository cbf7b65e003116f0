"""run()'s lazy trees on the device (Section 6.3: features evaluated lazily,
cheap rules first).

select_kernel walks the shipped lazy cascade with nnz_s counted on the
device only where a node asks for it; it must pick what the tuner's walk of
the same trees picks from features computed here on the host (nnz_s from
the column lengths), and run() must then match the oracle. The matrix and
vectors are the training sweep's power-law matrix (100K x 50K, mean row
length 40) with its uniform, hub-weighted and low-degree supports: on this
matrix the shipped trees ask on some vectors and not on others.
"""
import json

import numpy as np
import pytest

import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth, tune

from parity_util import assert_close, dev_sparse, reference

LAZY = spx.LAZY_SELECTOR
K_ATOMIC_CHAIN_MAX = 1 << 16  # longest FP32 row the one-at-a-time write-backs may sum


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _expected(sel, mf, A, col_len, idx):
    """The tuner's walk of the trees on host-computed features, with the
    library's two capability rules applied after it (the LDS-atomic
    write-back needs y in 64 KiB of LDS; FP32 rows longer than 2^16 entries
    leave the one-at-a-time write-backs for the sort)."""
    nx = int(idx.size)
    ns = int(col_len[idx].sum())
    f = dict(mf)
    f.update({"nnz_x": float(nx), "x_sparsity": nx / A.n, "nnz_s": float(ns), "m_sparsity": ns / A.nnz})
    pat, dist, wb, asked = tune._walk_cascade(sel, tune._feature_row({"features": f}))
    if pat != 2:
        wb = 0
    else:
        if wb == tune.WBS.index("lds_atomic") and A.m * 4 > 65536:
            wb = tune.WBS.index("sort")
        if mf["max_row"] > K_ATOMIC_CHAIN_MAX and tune.WBS[wb] in ("atomic", "lds_atomic", "bucket"):
            wb = tune.WBS.index("sort")
    return (pat, dist, wb), asked


def _rerun_report(M, x, plan, ref, S):
    """On a mismatch: whether the same call and the same plan given
    explicitly reproduce it (tells a wrong plan from a wrong execution)."""
    out = []
    for label, fn in (("run", lambda: M.run(x)), ("run_plan", lambda: M.run_plan(x, plan))):
        for _ in range(3):
            y = fn().cpu().numpy().astype(np.float64)
            bad = int(np.count_nonzero(np.abs(y - ref) > 1e-5 * S))
            out.append(f"{label}: {bad} rows off")
    return "; ".join(out)


@pytest.mark.gpu
def test_lazy_trees_pick_what_the_tuner_walks_and_match_the_oracle():
    _torch()
    with open(LAZY) as fh:
        sel = json.load(fh)
    assert sel.get("lazy") is True
    A = synth.powerlaw_rows(100_000, 50_000, 40.0, 31)
    M = spx.Matrix.from_host(A)
    M.load_selector(LAZY)
    mf = M.features()
    col_len = np.bincount(np.asarray(A.col_idx), minlength=A.n)
    asked = not_asked = 0
    checked = 0
    for kind in tune.SUPPORTS:
        for key, v in tune._vectors(A, kind):
            want, ask = _expected(sel, mf, A, col_len, np.asarray(v.idx, np.int64))
            x = dev_sparse(v, np.float32)
            p = M.select(x)
            got = (p.pattern, p.distribution, p.writeback)
            assert got == want, f"{kind} {key}: select_kernel {got}, tuner walk {want} (asked={ask})"
            asked += int(ask)
            not_asked += int(not ask)
            # run() on every vector that asked and on every fourth other one
            if ask or checked % 4 == 0:
                y = M.run(x)
                lp = M.last_plan()
                ref, S = reference(A, v.idx, v.val, "f32")
                try:
                    assert_close(y.cpu().numpy(), ref, S, "f32", f"run {kind} {key} plan={lp}")
                except AssertionError as err:
                    raise AssertionError(f"{err}\n{_rerun_report(M, x, lp, ref, S)}") from None
                assert (lp.pattern, lp.distribution, lp.writeback) == want, f"{kind} {key}: run() took {lp}"
            checked += 1
    assert asked >= 2 and not_asked >= 2, (asked, not_asked)
