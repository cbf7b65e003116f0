"""Differentiable sparse layer: Y = X A(vals)^T, i.e. y_b = A(vals) x_b for
each row x_b of a dense batch X (B x n), e.g. a pruned fully-connected
layer applied to post-ReLU activations.

Forward, two ways: "fused" (default) runs the row-major SpMV of every row
of X in one pass over A (spmv_csr_batch); "sparse" converts each row of X
to a sparse vector on the device and runs the batched SpMSpV, with the plan
of each vector chosen on the device (run_batch).
Backward (F32/F64), one library call (spx_backward): dX = G A (gather
along the CSC columns, no atomics) and dvals_k = sum_b G[b, row k] X[b, col k]
over the stored pattern; both kernels read the matrix once for the whole
batch and share one B-minor copy of G.

The matrix handle borrows its CSR value tensor; pass that tensor as
`vals` so autograd tracks it. Every forward re-derives the CSC copy of the
values (one gather through the CSC-to-CSR permutation), because the values
may have changed in place in ways the tensor's version counter does not
record (writes through .data, as optimizers and gradcheck do).
"""
from __future__ import annotations

import torch

from . import Matrix


class SparseLinearFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, X, M: Matrix, mode: str = "fused"):
        if vals.data_ptr() != M.vals.data_ptr():
            raise ValueError("vals must be the value tensor the matrix handle was built on")
        M.values_updated()
        Xc = X.contiguous()
        if mode == "fused":
            Y = M.spmv_batch(Xc)
        elif mode == "sparse":
            Y = M.run_dense_batch(Xc)
        else:
            raise ValueError(f"mode must be 'fused' or 'sparse', not {mode!r}")
        ctx.save_for_backward(Xc)
        ctx.M = M
        return Y

    @staticmethod
    def backward(ctx, G):
        (X,) = ctx.saved_tensors
        M = ctx.M
        G = G.contiguous()
        want_dvals, want_dx = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_dvals or want_dx):
            return None, None, None, None
        # one call: the B-minor copy of G serves both gradients
        dX, dvals = M.backward(G, X, want_dx=want_dx, want_dvals=want_dvals)
        if dX is not None:
            dX = dX.reshape(G.shape[:-1] + (M.n,))
        return dvals, dX, None, None


def sparse_linear(M: Matrix, X: torch.Tensor, vals: torch.Tensor | None = None,
                  mode: str = "fused") -> torch.Tensor:
    """Y[b] = A(vals) X[b] for every row of X (B x n) -> (B x m)."""
    return SparseLinearFunction.apply(M.vals if vals is None else vals, X, M, mode)
