"""Run-to-run determinism of the write-backs that have no write conflict.

The paper's reason for the write-back strategies is the write conflict of
the column-major pattern (Section 4.2.2): products of one row arrive from
many threads. The row-major patterns write each row once, the sort
write-back reduces the sorted pairs by key with per-tile carries joined in
tile order, and the merge write-back sums each row's sorted runs in a fixed
order, so all of them must give the same bits on every call. The atomic
write-backs (atomic, LDS-atomic, bucket) are not covered: their order of
additions is the order in which the hardware serves the atomics.
"""
import numpy as np
import pytest

import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import cfg_matrix

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _deterministic_plans():
    out = []
    for d in ("direct", "balanced"):
        out.append(spx.plan("spmv", d))
        out.append(spx.plan("csr_spmspv", d))
        if d == "balanced":
            out.append(spx.plan("csr_spmspv", d, tile=2048))
        out.append(spx.plan("csc_spmspv", d, "sort"))
        if hasattr(spx, "WB_MERGE"):
            out.append(spx.plan("csc_spmspv", d, "merge"))
    return out


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["f32", "f64"])
def test_sweep_bitwise_repeatable(kind):
    """R-MAT 2^20 (degree 16) with the sweep's vectors from 10 to 524,288
    entries: three calls of every conflict-free plan give identical bits."""
    torch = _torch()
    A = cfg_matrix("cfg2")
    npdt = np.float32 if kind == "f32" else np.float64
    M = spx.Matrix.from_host(A.with_vals(A.vals.astype(npdt)), fmt="csr")
    vecs = synth.cfg2_vectors(A.n)
    for v in vecs[::2] + [vecs[-1]]:
        x = (torch.as_tensor(v.idx, device="cuda"), torch.as_tensor(np.asarray(v.val, npdt), device="cuda"))
        for p in _deterministic_plans():
            ys = [M.run_plan(x, p) for _ in range(3)]
            torch.cuda.synchronize()
            bits = [y.cpu().numpy().view(np.uint32 if kind == "f32" else np.uint64) for y in ys]
            assert np.array_equal(bits[0], bits[1]) and np.array_equal(bits[0], bits[2]), \
                f"{kind} nnz_x={v.nnz} {p}: results differ between calls"
