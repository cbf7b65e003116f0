"""Seeded input generators: determinism, shapes and the structural facts
the workloads are defined by. CPU only."""
import numpy as np
import pytest

from paper_2006_16767_amd import synth


def _valid_csr(A):
    assert A.row_ptr.dtype == np.int32 and A.col_idx.dtype == np.int32
    assert A.row_ptr[0] == 0 and np.all(np.diff(A.row_ptr) >= 0)
    assert A.col_idx.size == A.nnz
    if A.nnz:
        assert A.col_idx.min() >= 0 and A.col_idx.max() < A.n
    for i in range(0, A.m, max(1, A.m // 200)):
        seg = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_cfg1_shapes_and_determinism():
    A = synth.cfg1_matrix()
    B = synth.cfg1_matrix()
    _valid_csr(A)
    assert A.m == A.n == 4096 and A.nnz == 65536
    assert np.array_equal(A.col_idx, B.col_idx) and np.array_equal(A.vals, B.vals)
    assert np.all(np.diff(A.row_ptr) == 16)
    assert A.vals.min() >= -1 and A.vals.max() <= 1
    dense, sparse = synth.cfg1_vectors()
    assert [v.nnz for v in sparse] == [4096, 410, 41, 4]
    for v in sparse:
        assert np.all(np.diff(v.idx) > 0)


def test_rmat_small_structure():
    A = synth.rmat(12, 16, 5)
    _valid_csr(A)
    assert A.m == A.n == 4096
    assert A.nnz <= 16 * 4096
    L = np.diff(A.row_ptr)
    # skewed degree distribution: max far above mean, many empty rows
    assert L.max() > 10 * L.mean() and (L == 0).mean() > 0.2
    assert A.vals.min() >= 0 and A.vals.max() <= 1


def test_poisson_structure():
    A = synth.poisson3d(5)
    _valid_csr(A)
    D = np.zeros((A.m, A.n))
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    D[rows, A.col_idx] = A.vals
    assert np.array_equal(D, D.T)
    assert np.all(np.diag(D) == 6)


def test_powerlaw_and_bernoulli():
    A = synth.powerlaw_rows(20000, 5000, 40.0, 3)
    _valid_csr(A)
    assert abs(np.diff(A.row_ptr).mean() - 40.0) <= 0.5
    C = synth.powerlaw_cols(5000, 20000, 40.0, 3)
    _valid_csr(C)
    # the column lengths are the row lengths of the row generator, transposed
    assert np.array_equal(np.sort(np.bincount(C.col_idx, minlength=C.n)), np.sort(np.diff(A.row_ptr)))
    W = synth.bernoulli(512, 256, 0.05, 4)
    _valid_csr(W)
    assert abs(W.nnz / (512 * 256) - 0.05) < 0.005


def test_vectors():
    v = synth.sparse_vector(1000, 37, 1)
    assert v.nnz == 37 and np.all(np.diff(v.idx) > 0) and v.idx.max() < 1000
    v0 = synth.sparse_vector(1000, 0, 1)
    assert v0.nnz == 0
    vn = synth.sparse_vector(100, 100, 1)
    assert np.array_equal(vn.idx, np.arange(100))
    acts = synth.cfg5_activations(n=256, B=8)
    assert [a.nnz for a in acts][0] == 128 and all(np.all(a.val >= 0) for a in acts)
