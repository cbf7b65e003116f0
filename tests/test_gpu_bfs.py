"""Breadth-first search driver (one adaptive (OR, AND) SpMSpV per level)
against the oracle's queue traversal: levels are unique, so they must match
exactly, whatever kernel each level picks."""
import numpy as np
import pytest

import oracle
import paper_2006_16767_amd as spx
from paper_2006_16767_amd import synth

from parity_util import cfg_matrix

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _edges(A):
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr)).astype(np.int32)
    return A.col_idx, rows  # stored (i, j) is the edge j -> i


def _source(A):
    outdeg = np.bincount(A.col_idx, minlength=A.n)
    return 0 if outdeg[0] > 0 else int(np.nonzero(outdeg > 0)[0][0])


@pytest.mark.parametrize("push_only", [False, True])
@pytest.mark.parametrize("name", ["rmat16", "cfg2"])
def test_bfs_adaptive_matches_oracle(name, push_only):
    _torch()
    A = cfg_matrix(name)
    M = spx.Matrix.from_host(A, dtype=spx.BOOL)
    s = _source(A)
    level, plans = M.bfs(s, push_only=push_only)
    want = oracle.bfs_levels(*_edges(A), A.n, s)
    assert np.array_equal(level.cpu().numpy(), want)
    assert M.bfs_levels == int(want.max()) + 1
    assert len(plans) == M.bfs_levels  # the last expansion finds no new vertex
    pulls = sum(p.lanes == -1 for p in plans)
    if push_only:
        assert pulls == 0
    elif name == "cfg2":
        assert pulls > 0  # the dense middle levels of the R-MAT search pull


def test_bfs_pull_on_graphs_with_unreachable_parts():
    """Several components and sinks: the masked pull must leave every
    vertex outside the source's reach at -1 and stop rows at the first
    frontier neighbour without skipping any level."""
    _torch()
    rng = np.random.default_rng(3)
    n = 20000
    src = rng.integers(0, n // 2, 120000).astype(np.int32)  # edges only among the first half
    dst = rng.integers(0, n // 2, 120000).astype(np.int32)
    key = np.unique(dst.astype(np.int64) * n + src)
    A = synth._coo_to_csr(n, n, key // n, key % n, None)
    M = spx.Matrix.from_host(A, dtype=spx.BOOL)
    s = int(src[0])
    want = oracle.bfs_levels(A.col_idx, np.repeat(np.arange(n), np.diff(A.row_ptr)).astype(np.int32), n, s)
    level, plans = M.bfs(s)
    assert np.array_equal(level.cpu().numpy(), want)
    assert any(p.lanes == -1 for p in plans)


def test_bfs_every_fixed_plan_matches_oracle():
    _torch()
    A = cfg_matrix("rmat16")
    M = spx.Matrix.from_host(A, dtype=spx.BOOL)
    s = _source(A)
    want = oracle.bfs_levels(*_edges(A), A.n, s)
    for p in spx.all_plans():
        try:
            level, plans = M.bfs(s, plan=p)
        except spx.SpxError as e:
            if e.code == -5 and p.writeback == spx.WB_LDS_ATOMIC:
                continue  # y does not fit in LDS for this m
            raise
        assert np.array_equal(level.cpu().numpy(), want), p
        assert all(q.pattern == p.pattern and q.writeback == p.writeback for q in plans)


def test_bfs_edge_cases():
    torch = _torch()
    # a graph with an isolated vertex, a chain and a cycle
    src = np.array([0, 1, 2, 3, 5], np.int32)
    dst = np.array([1, 2, 3, 1, 6], np.int32)
    n = 8
    A = synth._coo_to_csr(n, n, dst.astype(np.int64), src.astype(np.int64), None)
    M = spx.Matrix.from_host(A, dtype=spx.BOOL)
    level, _ = M.bfs(0)
    assert level.cpu().numpy().tolist() == [0, 1, 2, 3, -1, -1, -1, -1]
    level, _ = M.bfs(4)  # no out-edge
    assert level.cpu().numpy().tolist() == [-1, -1, -1, -1, 0, -1, -1, -1] and M.bfs_levels == 1
    level, plans = M.bfs(0, max_levels=2)  # levels 0 and 1 only
    assert level.cpu().numpy().tolist() == [0, 1, -1, -1, -1, -1, -1, -1] and M.bfs_levels == 2
    with pytest.raises(spx.SpxError) as e:
        M.bfs(n)
    assert e.value.code == -3
    F = spx.Matrix.from_host(synth.random_csr(8, 8, 0.3, 1))
    with pytest.raises(spx.SpxError) as e:
        F.bfs(0)
    assert e.value.code == -4
    R = spx.Matrix.from_host(synth.random_csr(8, 9, 0.3, 1), dtype=spx.BOOL)
    with pytest.raises(spx.SpxError) as e:
        R.bfs(0)
    assert e.value.code == -2
