"""Seeded synthetic inputs shaped like the paper's workloads.

This module builds matrices and vectors only. It holds none of the method's
arithmetic (no product, no transpose, no feature): both the CPU oracle and
the HIP path consume what it returns, and neither depends on the other.

Every generator is deterministic in its seed (numpy PCG64). Index sets are
drawn without replacement and stored sorted. Matrices are returned in CSR
form (row_ptr int32[m+1], col_idx int32[nnz], vals) because CSR is the
format in which the paper's problem statement hands a matrix over
(Section 2, storage formats); every other layout is derived downstream.

Workloads (the paper's own datasets are not available; these stand in):
  * uniform:  m x n with a fixed number of distinct uniform columns per row
  * rmat:     R-MAT graph (quadrant probabilities a, b, c, d), deduplicated,
              randomly relabelled; A[i, j] = 1 iff edge j -> i, so a column
              is a vertex's out-edges (push) and a row its in-edges (pull)
  * poisson3d: 7-point Laplacian on a k^3 grid, Dirichlet, x-fastest order
  * powerlaw: rows with Pareto(1.5) lengths (SVM-like data matrix); the
              column variant skews column lengths instead
  * bernoulli: each entry present with probability p (pruned FC layer)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 16767


def seed_for(cfg: int, k: int = 0) -> int:
    """Seed convention: 16767 + 100*cfg + k."""
    return SEED_BASE + 100 * cfg + k


@dataclass
class CSR:
    m: int
    n: int
    row_ptr: np.ndarray  # int32[m+1]
    col_idx: np.ndarray  # int32[nnz]
    vals: np.ndarray | None  # float32/float64/int32[nnz] or None (pattern only)
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def with_vals(self, vals: np.ndarray) -> "CSR":
        return CSR(self.m, self.n, self.row_ptr, self.col_idx, vals, dict(self.meta))


@dataclass
class SparseVec:
    n: int
    idx: np.ndarray  # int32[nnz_x], unique, sorted
    val: np.ndarray | None

    @property
    def nnz(self) -> int:
        return int(self.idx.shape[0])

    def dense(self, dtype=None) -> np.ndarray:
        """Zero-filled dense copy (a format change, not arithmetic)."""
        dt = dtype or (self.val.dtype if self.val is not None else np.uint8)
        out = np.zeros(self.n, dtype=dt)
        out[self.idx] = self.val if self.val is not None else 1
        return out


def _coo_to_csr(m: int, n: int, rows: np.ndarray, cols: np.ndarray,
                vals: np.ndarray | None) -> CSR:
    """Order (row, col) pairs row-major and build row pointers."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    rows = rows[order]
    cols = cols[order]
    if vals is not None:
        vals = vals[order]
    counts = np.bincount(rows, minlength=m).astype(np.int64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return CSR(m, n, row_ptr.astype(np.int32), cols.astype(np.int32), vals)


def _rows_of_distinct_cols(rng, m: int, n: int, lengths: np.ndarray) -> np.ndarray:
    """For each row r, draw lengths[r] distinct columns uniformly from [0, n),
    sorted. Returns the rows' columns concatenated in row order."""
    out = np.empty(int(lengths.sum()), dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(lengths)])
    for L in np.unique(lengths):
        L = int(L)
        rows = np.nonzero(lengths == L)[0]
        if L == 0:
            continue
        if L * 4 <= n and L <= 256:
            # draw with replacement, redraw the rows that hit a duplicate
            block = rng.integers(0, n, size=(rows.size, L), dtype=np.int64)
            block.sort(axis=1)
            while True:
                dup = np.any(block[:, 1:] == block[:, :-1], axis=1)
                if not dup.any():
                    break
                redo = np.nonzero(dup)[0]
                nb = rng.integers(0, n, size=(redo.size, L), dtype=np.int64)
                nb.sort(axis=1)
                block[redo] = nb
        else:
            block = np.stack([np.sort(rng.choice(n, size=L, replace=False)) for _ in rows])
        for i, r in enumerate(rows):
            out[starts[r]:starts[r] + L] = block[i]
    return out


def uniform_rows(m: int, n: int, per_row: int, seed: int, dtype=np.float32,
                 lo: float = -1.0, hi: float = 1.0) -> CSR:
    """m x n matrix, each row has `per_row` distinct uniform columns,
    values U[lo, hi]."""
    rng = np.random.default_rng(seed)
    block = rng.integers(0, n, size=(m, per_row), dtype=np.int64)
    block.sort(axis=1)
    while True:
        dup = np.any(block[:, 1:] == block[:, :-1], axis=1)
        if not dup.any():
            break
        redo = np.nonzero(dup)[0]
        nb = rng.integers(0, n, size=(redo.size, per_row), dtype=np.int64)
        nb.sort(axis=1)
        block[redo] = nb
    cols = block.reshape(-1).astype(np.int32)
    row_ptr = (np.arange(m + 1, dtype=np.int64) * per_row).astype(np.int32)
    vals = rng.uniform(lo, hi, size=m * per_row).astype(dtype)
    return CSR(m, n, row_ptr, cols, vals, {"kind": "uniform", "per_row": per_row, "seed": seed})


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19,
         relabel: bool = True, dtype=np.float32) -> CSR:
    """R-MAT graph with 2^scale vertices and edge_factor * 2^scale sampled
    edges. Each edge picks one of four quadrants per level (a: (0,0),
    b: (0,1), c: (1,0), d: (1,1) for (source bit, target bit)).
    Duplicates are removed, self loops kept. A seeded random permutation
    relabels the vertices. A[i, j] = 1 iff edge j -> i. Weights U[0, 1]
    are drawn per unique edge."""
    rng = np.random.default_rng(seed)
    nv = 1 << scale
    E = edge_factor * nv
    src = np.zeros(E, dtype=np.int64)
    dst = np.zeros(E, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    for lvl in range(scale):
        r = rng.random(E, dtype=np.float32)
        sbit = r >= ab
        tbit = ((r >= a) & (r < ab)) | (r >= abc)
        bit = np.int64(1) << (scale - 1 - lvl)
        src |= sbit.astype(np.int64) * bit
        dst |= tbit.astype(np.int64) * bit
    if relabel:
        perm = rng.permutation(nv).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
    key = np.unique(dst * nv + src)  # sorted by (row=dst, col=src), deduped
    rows = (key // nv).astype(np.int64)
    cols = (key % nv).astype(np.int32)
    counts = np.bincount(rows, minlength=nv)
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    vals = rng.random(key.size, dtype=np.float64).astype(dtype)
    return CSR(nv, nv, row_ptr.astype(np.int32), cols, vals,
               {"kind": "rmat", "scale": scale, "edge_factor": edge_factor,
                "a": a, "b": b, "c": c, "relabel": relabel, "seed": seed,
                "sampled_edges": E})


def poisson3d(k: int, dtype=np.float32) -> CSR:
    """7-point Laplacian on a k^3 grid with natural x-fastest ordering
    (index = x + k*y + k*k*z), 6 on the diagonal and -1 for each in-grid
    neighbour (Dirichlet: out-of-grid neighbours are dropped)."""
    N = k * k * k
    idx = np.arange(N, dtype=np.int64)
    x = idx % k
    y = (idx // k) % k
    z = idx // (k * k)
    offs = [(-k * k, z > 0), (-k, y > 0), (-1, x > 0), (0, np.ones(N, bool)),
            (1, x < k - 1), (k, y < k - 1), (k * k, z < k - 1)]
    present = np.stack([mask for _, mask in offs], axis=1)  # N x 7, column-ascending order
    colmat = idx[:, None] + np.array([o for o, _ in offs], dtype=np.int64)[None, :]
    valmat = np.where(np.array([o == 0 for o, _ in offs])[None, :], 6.0, -1.0)
    valmat = np.broadcast_to(valmat, present.shape)
    counts = present.sum(axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    cols = colmat[present].astype(np.int32)
    vals = valmat[present].astype(dtype)
    return CSR(N, N, row_ptr.astype(np.int32), cols, vals, {"kind": "poisson3d", "k": k})


def powerlaw_rows(m: int, n: int, mean_len: float, seed: int, alpha: float = 1.5,
                  dtype=np.float32) -> CSR:
    """Rows with lengths L = min(n, ceil(x_min * U^(-1/alpha))), x_min tuned
    by bisection so that mean(L) is within 0.5 of mean_len; uniform
    distinct columns; values U[0, 1]."""
    rng = np.random.default_rng(seed)
    u = rng.random(m)
    base = u ** (-1.0 / alpha)

    def lens(xm):
        return np.minimum(n, np.ceil(xm * base)).astype(np.int64)

    lo, hi = 0.01, float(mean_len)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if lens(mid).mean() < mean_len:
            lo = mid
        else:
            hi = mid
    xm = 0.5 * (lo + hi)
    L = lens(xm)
    cols = _rows_of_distinct_cols(rng, m, n, L)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(L, out=row_ptr[1:])
    vals = rng.random(int(L.sum())).astype(dtype)
    return CSR(m, n, row_ptr.astype(np.int32), cols.astype(np.int32), vals,
               {"kind": "powerlaw", "alpha": alpha, "x_min": xm, "mean": float(L.mean()),
                "seed": seed})


def powerlaw_cols(m: int, n: int, mean_len: float, seed: int, alpha: float = 1.5,
                  dtype=np.float32) -> CSR:
    """Columns with Pareto(alpha) lengths of mean mean_len and uniformly
    placed distinct rows (feature-popularity skew): the column draws of
    powerlaw_rows with the roles of m and n swapped, stored as CSR."""
    D = powerlaw_rows(n, m, mean_len, seed, alpha, dtype)
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(D.row_ptr))
    A = _coo_to_csr(m, n, np.asarray(D.col_idx, np.int64), cols, D.vals)
    A.meta = {"kind": "powerlaw_cols", "mean_len": mean_len, "alpha": alpha, "seed": seed}
    return A


def bernoulli(m: int, n: int, p: float, seed: int, std: float = 0.02,
              dtype=np.float32) -> CSR:
    """Each entry present independently with probability p; values
    N(0, std^2)."""
    rng = np.random.default_rng(seed)
    rows_l = []
    cols_l = []
    blk = max(1, (1 << 24) // max(n, 1))
    for r0 in range(0, m, blk):
        r1 = min(m, r0 + blk)
        mask = rng.random((r1 - r0, n), dtype=np.float32) < p
        rr, cc = np.nonzero(mask)
        rows_l.append(rr + r0)
        cols_l.append(cc)
    rows = np.concatenate(rows_l).astype(np.int64)
    cols = np.concatenate(cols_l).astype(np.int64)
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    vals = (rng.standard_normal(rows.size) * std).astype(dtype)
    return CSR(m, n, row_ptr.astype(np.int32), cols.astype(np.int32), vals,
               {"kind": "bernoulli", "p": p, "seed": seed})


def random_csr(m: int, n: int, density: float, seed: int, dtype=np.float32,
               int_values: bool = False, empty_rows: float = 0.0) -> CSR:
    """Small random matrix for brute-force checks: Bernoulli pattern with a
    fraction of rows forced empty; values U[-1, 1] or integers in [-4, 4]."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    if empty_rows > 0:
        mask[rng.random(m) < empty_rows, :] = False
    rr, cc = np.nonzero(mask)
    if int_values:
        vals = rng.integers(-4, 5, size=rr.size).astype(dtype)
    else:
        vals = rng.uniform(-1, 1, size=rr.size).astype(dtype)
    return _coo_to_csr(m, n, rr.astype(np.int64), cc.astype(np.int64), vals)


def hub_matrix(n: int, hub_len: int, per_row: int, seed: int, dtype=np.float32) -> CSR:
    """Square n x n matrix with one hub row and one hub column for the
    accumulation-length checks: row 0 holds columns 0 .. hub_len - 1,
    column 1 holds rows 1 .. hub_len, and every other row gets per_row
    distinct uniform columns (a row's draw may hit column 1 again only as
    that row's hub entry). Values U[0, 1] (one sign, so rounding errors do
    not cancel)."""
    rng = np.random.default_rng(seed)
    rows = [np.zeros(hub_len, np.int64), np.arange(1, hub_len + 1, dtype=np.int64)]
    cols = [np.arange(hub_len, dtype=np.int64), np.ones(hub_len, np.int64)]
    r = np.repeat(np.arange(1, n, dtype=np.int64), per_row)
    c = rng.integers(0, n, size=r.size, dtype=np.int64)
    rows.append(r)
    cols.append(c)
    rr = np.concatenate(rows)
    cc = np.concatenate(cols)
    key = np.unique(rr * n + cc)  # distinct entries
    rr, cc = key // n, key % n
    vals = rng.uniform(0.0, 1.0, size=rr.size).astype(dtype)
    return _coo_to_csr(n, n, rr, cc, vals)


def weighted_sparse_vector(n: int, nnz: int, weights: np.ndarray, seed: int, lo=0.0, hi=1.0,
                           dtype=np.float32) -> SparseVec:
    """nnz distinct indices drawn without replacement with probability
    proportional to weights (Efraimidis-Spirakis keys U^(1/w)); indices of
    zero weight only once the positive ones run out. Sorted; values
    U[lo, hi]. Used for supports shaped like graph frontiers: weights =
    column lengths favours hubs, 1 / (length + 1) the low-degree tail."""
    rng = np.random.default_rng(seed)
    nnz = int(min(max(nnz, 0), n))
    w = np.asarray(weights, np.float64)
    u = rng.random(n)
    with np.errstate(divide="ignore"):
        key = np.where(w > 0, np.log(u) / np.where(w > 0, w, 1.0), -np.inf)
    idx = np.sort(np.argpartition(-key, nnz - 1)[:nnz]) if 0 < nnz < n else np.arange(nnz)
    val = rng.uniform(lo, hi, size=nnz).astype(dtype)
    return SparseVec(n, idx.astype(np.int32), val)


def sparse_vector(n: int, nnz: int, seed: int, dist: str = "uniform",
                  dtype=np.float32, lo=-1.0, hi=1.0) -> SparseVec:
    """nnz distinct uniform indices in [0, n), sorted; values drawn from
    U[lo, hi] ('uniform'), N(0, 1) ('normal'), |N(0, 1)| ('halfnormal'),
    integers in [-4, 4] ('int'), or None ('pattern')."""
    rng = np.random.default_rng(seed)
    nnz = int(min(max(nnz, 0), n))
    if nnz * 8 < n:
        idx = np.empty(0, dtype=np.int64)
        while idx.size < nnz:
            extra = rng.integers(0, n, size=2 * (nnz - idx.size) + 8)
            idx = np.unique(np.concatenate([idx, extra]))
        idx = rng.permutation(idx)[:nnz]
        idx.sort()
    else:
        idx = np.sort(rng.choice(n, size=nnz, replace=False))
    idx = idx.astype(np.int32)
    if dist == "pattern":
        val = None
    elif dist == "uniform":
        val = rng.uniform(lo, hi, size=nnz).astype(dtype)
    elif dist == "normal":
        val = rng.standard_normal(nnz).astype(dtype)
    elif dist == "halfnormal":
        val = np.abs(rng.standard_normal(nnz)).astype(dtype)
    elif dist == "int":
        val = rng.integers(-4, 5, size=nnz).astype(dtype)
    else:
        raise ValueError(dist)
    return SparseVec(n, idx, val)


def dense_vector(n: int, seed: int, dist: str = "uniform", dtype=np.float32,
                 lo=-1.0, hi=1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        return rng.uniform(lo, hi, size=n).astype(dtype)
    if dist == "normal":
        return rng.standard_normal(n).astype(dtype)
    if dist == "int":
        return rng.integers(-4, 5, size=n).astype(dtype)
    raise ValueError(dist)


# ---------------------------------------------------------------------------
# The five workload configurations
# ---------------------------------------------------------------------------

CFG1_DENSITIES = (1.0, 0.1, 0.01, 0.001)
CFG2_DENSITIES = tuple(float(d) for d in np.geomspace(1e-5, 0.5, 12))


def cfg1_matrix() -> CSR:
    """4096 x 4096, 16 distinct uniform columns per row, values U[-1, 1]."""
    return uniform_rows(4096, 4096, 16, seed_for(1, 0))


def cfg1_vectors():
    """Dense x U[-1,1] plus sparse x at densities 1, 0.1, 0.01, 0.001."""
    n = 4096
    dense = dense_vector(n, seed_for(1, 1))
    sparse = [sparse_vector(n, round(d * n), seed_for(1, 2 + i)) for i, d in enumerate(CFG1_DENSITIES)]
    return dense, sparse


def cfg2_matrix(scale: int = 20, edge_factor: int = 16) -> CSR:
    """R-MAT (0.57, 0.19, 0.19, 0.05), 2^20 vertices, edge factor 16,
    FP32 weights U[0, 1]."""
    return rmat(scale, edge_factor, seed_for(2, 0))


def cfg2_vectors(n: int = 1 << 20, densities=CFG2_DENSITIES):
    """Sparse vectors with nnz fraction log-spaced over [1e-5, 0.5]; values
    U[0, 1]."""
    return [sparse_vector(n, max(1, round(d * n)), seed_for(2, 1 + i), lo=0.0, hi=1.0)
            for i, d in enumerate(densities)]


def cfg3_matrix(dtype=np.float32, k: int = 128) -> CSR:
    return poisson3d(k, dtype)


def cfg3_vectors(n: int = 128 ** 3, dtype=np.float32):
    dense = dense_vector(n, seed_for(3, 1), "normal", dtype)
    sparse = sparse_vector(n, round(0.01 * n), seed_for(3, 2), "normal", dtype)
    return dense, sparse


def cfg4_rmat() -> CSR:
    """R-MAT 2^18 vertices, edge factor 32, FP32 weights U[0, 1]."""
    return rmat(18, 32, seed_for(4, 0))


def cfg4_rmat_batch(n: int = 1 << 18, B: int = 512):
    """B sparse vectors, densities 10^U[-4, log10 0.5], uniform supports,
    values U[0, 1]."""
    rng = np.random.default_rng(seed_for(4, 1))
    dens = 10.0 ** rng.uniform(-4.0, math.log10(0.5), size=B)
    return [sparse_vector(n, max(1, round(d * n)), seed_for(4, 1000 + i), lo=0.0, hi=1.0)
            for i, d in enumerate(dens)]


def cfg4_svm() -> CSR:
    """100,000 x 50,000 with Pareto(1.5) row lengths of mean 40, values
    U[0, 1]."""
    return powerlaw_rows(100_000, 50_000, 40.0, seed_for(4, 2))


def cfg4_svm_batch(A: CSR, B: int = 256):
    """B distinct rows of A (chosen uniformly) used as sparse vectors of
    length A.n."""
    rng = np.random.default_rng(seed_for(4, 3))
    rows = np.sort(rng.choice(A.m, size=B, replace=False))
    out = []
    for r in rows:
        s, e = int(A.row_ptr[r]), int(A.row_ptr[r + 1])
        out.append(SparseVec(A.n, A.col_idx[s:e].copy(), A.vals[s:e].copy()))
    return out


def cfg5_matrix(m: int = 16384, n: int = 4096, p: float = 0.05) -> CSR:
    """Pruned FC weights: Bernoulli(0.05) pattern, N(0, 0.02^2) values."""
    return bernoulli(m, n, p, seed_for(5, 0))


def cfg5_activations(n: int = 4096, B: int = 64):
    """B post-ReLU activation vectors: zero fraction 0.5 + 0.45 b/(B-1),
    uniform supports, values |N(0, 1)|."""
    out = []
    for b in range(B):
        z = 0.5 + 0.45 * b / max(B - 1, 1)
        out.append(sparse_vector(n, round((1 - z) * n), seed_for(5, 1 + b), "halfnormal"))
    return out


def cfg5_upstream(m: int = 16384, B: int = 64) -> np.ndarray:
    rng = np.random.default_rng(seed_for(5, 999))
    return rng.standard_normal((B, m)).astype(np.float32)


def bfs_frontiers(A: CSR, max_levels: int = 64):
    """Frontiers of a breadth-first search from the lowest-id vertex with an
    out-edge, with a visited mask (levels of the search). A[i, j] != 0 is
    an edge j -> i, so the out-neighbours of j are the rows that list j.
    Returned as pattern sparse vectors. This is an input generator for
    BFS-like test vectors; the expansion arithmetic it uses is a plain
    edge-list walk."""
    rows = np.repeat(np.arange(A.m, dtype=np.int64), np.diff(A.row_ptr.astype(np.int64)))
    cols = A.col_idx.astype(np.int64)
    order = np.argsort(cols, kind="stable")
    src_sorted = cols[order]
    dst_sorted = rows[order]
    starts = np.searchsorted(src_sorted, np.arange(A.n + 1))
    outdeg = np.diff(starts)
    src0 = 0 if outdeg[0] > 0 else int(np.nonzero(outdeg > 0)[0][0])
    visited = np.zeros(A.m, dtype=bool)
    frontier = np.array([src0], dtype=np.int64)
    visited[src0] = True
    out = []
    for _ in range(max_levels):
        if frontier.size == 0:
            break
        out.append(SparseVec(A.n, frontier.astype(np.int32), None))
        seg = [dst_sorted[starts[j]:starts[j + 1]] for j in frontier]
        nxt = np.unique(np.concatenate(seg)) if seg else np.empty(0, np.int64)
        nxt = nxt[~visited[nxt]]
        visited[nxt] = True
        frontier = nxt
    return out
