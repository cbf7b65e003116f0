"""Kernel-selector training on timings from this GPU (Section 5.2).

    python -m paper_2006_16767_amd.tune sweep --out sweep.jsonl   # on the GPU
    python -m paper_2006_16767_amd.tune train sweep.jsonl --out selector.json
    (sweep --dtype bool times the (OR, AND) semiring, for the trees BOOL
    handles load)

sweep  builds a synthetic corpus (uniform, R-MAT, Poisson stencil, power-law,
       Bernoulli and SVM-like feature matrices; for each, input vectors whose nnz_x grows from
       1 to n on a log scale, uniformly placed), times every candidate kernel
       with HIP events (median of several runs, the result of each run
       discarded), and appends one JSON record per (matrix, vector): the 13
       features of Table 1 and the time of every plan. An interrupted sweep
       resumes by skipping keys already in the file.
train  labels each record per factor (the pattern of the fastest kernel;
       the best distribution within that pattern; the best write-back within
       the column-major pattern and the chosen distribution; times within 2%
       go to the cheaper alternative), splits 7:3, and grid-searches a
       project-written CART decision tree (max_depth 1..10; sample weights
       balanced by class, uniform, or by regret, i.e. the relative time the
       worst alternative would lose; 3-fold cross-validation on the training
       part, scored by accuracy).
       The three trees are written as the JSON the library loads
       (spx_load_selector).

By default the trees use only features the host knows without a device
round trip (everything except nnz_s, m_sparsity and the derived s_per_x);
--all-features trains the trees for callers that know nnz_s (the graph
drivers), which the library keeps apart from run()'s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

FEATURES = ("m", "n", "nnz", "max_row", "min_row", "avg_row", "relative_range", "var_nnz_row", "gini",
            "nnz_x", "x_sparsity", "nnz_s", "m_sparsity", "s_per_x")
# s_per_x = nnz_s / max(1, nnz_x), the mean length of the selected columns,
# is derived here (not in Table 1, not stored by the sweep): the trees
# cannot form a ratio of two features, and it separates hub-heavy vectors,
# on which the direct column-major distribution serializes on long columns.
CHEAP = tuple(f for f in FEATURES if f not in ("nnz_s", "m_sparsity", "s_per_x"))


def _feature_row(rec):
    f = dict(rec["features"])
    f["s_per_x"] = f["nnz_s"] / max(1.0, f["nnz_x"])
    return [f[k] for k in FEATURES]
PATTERNS = ("spmv", "csr_spmspv", "csc_spmspv")
DISTS = ("direct", "balanced")
WBS = ("none", "atomic", "sort", "lds_atomic", "bucket", "merge")
# cheaper-first order used to break near-ties (within 2%)
COST_ORDER = {("spmv",): 0, ("csr_spmspv",): 1, ("csc_spmspv", "atomic"): 2, ("csc_spmspv", "lds_atomic"): 3,
              ("csc_spmspv", "bucket"): 4, ("csc_spmspv", "merge"): 5, ("csc_spmspv", "sort"): 6}
# features that cost run() a device count and a stream synchronization
COUNT_FEATURES = ("nnz_s", "m_sparsity", "s_per_x")
TIE = 1.02


# ----------------------------------------------------------------------------- corpus
def corpus(quick: bool = False):
    """(name, generator) pairs of the synthetic training matrices."""
    from . import synth
    mats = [
        ("uniform_4k_d16", lambda: synth.uniform_rows(4096, 4096, 16, 43)),
        ("uniform_16k_d4", lambda: synth.uniform_rows(16384, 16384, 4, 44)),
        ("uniform_64k_d8", lambda: synth.uniform_rows(65536, 65536, 8, 11)),
        ("uniform_128k_d64", lambda: synth.uniform_rows(131072, 131072, 64, 45)),
        ("uniform_256k_d32", lambda: synth.uniform_rows(262144, 262144, 32, 12)),
        ("uniform_1m_d16", lambda: synth.uniform_rows(1 << 20, 1 << 20, 16, 13)),
        ("uniform_2m_d8", lambda: synth.uniform_rows(1 << 21, 1 << 21, 8, 46)),
        ("rmat14_d16", lambda: synth.rmat(14, 16, 21)),
        ("rmat16_d4", lambda: synth.rmat(16, 4, 26)),
        ("rmat17_d8", lambda: synth.rmat(17, 8, 22)),
        ("rmat18_d32", lambda: synth.rmat(18, 32, 23)),
        ("rmat19_d16", lambda: synth.rmat(19, 16, 27)),
        ("rmat20_d4", lambda: synth.rmat(20, 4, 28)),
        ("rmat20_d16", lambda: synth.rmat(20, 16, 24)),
        ("rmat20_d16_nrl", lambda: synth.rmat(20, 16, 25, relabel=False)),
        ("rmat21_d8", lambda: synth.rmat(21, 8, 29)),
        ("poisson32", lambda: synth.poisson3d(32)),
        ("poisson64", lambda: synth.poisson3d(64)),
        ("poisson100", lambda: synth.poisson3d(100)),
        ("poisson128", lambda: synth.poisson3d(128)),
        ("powerlaw_100k_50k", lambda: synth.powerlaw_rows(100_000, 50_000, 40.0, 31)),
        ("powerlaw_500k_500k", lambda: synth.powerlaw_rows(500_000, 500_000, 12.0, 32)),
        ("powerlaw_1m_1m", lambda: synth.powerlaw_rows(1 << 20, 1 << 20, 6.0, 33)),
        ("powerlaw_50k_200k_a2", lambda: synth.powerlaw_rows(50_000, 200_000, 20.0, 34, alpha=2.0)),
        ("bernoulli_16k_4k", lambda: synth.bernoulli(16384, 4096, 0.05, 41)),
        ("bernoulli_4k_16k", lambda: synth.bernoulli(4096, 16384, 0.02, 42)),
        ("bernoulli_32k_8k", lambda: synth.bernoulli(32768, 8192, 0.01, 47)),
        ("bernoulli_8k_8k", lambda: synth.bernoulli(8192, 8192, 0.1, 48)),
        ("powerlaw_200k_1m", lambda: synth.powerlaw_rows(200_000, 1 << 20, 8.0, 35)),
        ("powerlaw_cols_1m_200k", lambda: synth.powerlaw_cols(1 << 20, 200_000, 8.0, 36)),
    ]
    if quick:
        mats = [m for m in mats if m[0] in ("uniform_4k_d16", "rmat14_d16", "poisson32")]
    return mats


def densities(n: int, count: int = 40):
    """nnz_x from 1 to n, log-spaced (the paper grows nnz_x from 1 to n)."""
    vals = np.unique(np.round(np.geomspace(1, n, count)).astype(np.int64))
    return [int(v) for v in vals]


SUPPORTS = ("uniform", "hub", "low")


def _vectors(A, kind: str):
    """(key suffix, sparse vector) pairs of one support kind: "uniform"
    places nnz_x indices uniformly (40 sizes from 1 to n); "hub" draws them
    with probability proportional to the column length and "low" to
    1 / (length + 1), as graph frontiers do (20 sizes up to n / 2), so that
    nnz_s departs from nnz_x times the average column length."""
    from . import synth
    if kind == "uniform":
        return [(f"{nx}", synth.sparse_vector(A.n, nx, 5000 + i, lo=0.0, hi=1.0))
                for i, nx in enumerate(densities(A.n))]
    clen = np.bincount(np.asarray(A.col_idx), minlength=A.n).astype(np.float64)
    w = clen if kind == "hub" else 1.0 / (clen + 1.0)
    cap = int(min(A.n // 2, (w > 0).sum()))
    sizes = [nx for nx in densities(A.n, 20) if nx <= cap]
    seed0 = 7000 if kind == "hub" else 9000
    return [(f"{kind}:{nx}", synth.weighted_sparse_vector(A.n, nx, w, seed0 + i)) for i, nx in enumerate(sizes)]


def sweep(out_path: str, reps: int = 5, quick: bool = False, plans=None, dtype: str = "f32",
          supports=("uniform",)):
    """dtype "f32": FP32 values; "bool": the pattern and index-only vectors
    in the (OR, AND) semiring. supports: the vector kinds of _vectors."""
    import torch
    from . import BOOL, Matrix, all_plans, synth

    done = set()
    if os.path.exists(out_path):
        with open(out_path) as f:
            for line in f:
                try:
                    done.add(json.loads(line)["key"])
                except Exception:
                    pass
    plans = plans or all_plans()
    with open(out_path, "a") as fout:
        for name, gen in corpus(quick):
            t0 = time.time()
            A = gen()
            M = Matrix.from_host(A, dtype=BOOL if dtype == "bool" else None)
            mf = M.features()
            print(f"[tune] {name}: m={A.m} n={A.n} nnz={A.nnz} gen {time.time() - t0:.1f}s", flush=True)
            y = M.out_tensor()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            todo = [(f"{name}:{suffix}", kind, v) for kind in supports for suffix, v in _vectors(A, kind)
                    if f"{name}:{suffix}" not in done]
            for key, kind, v in todo:
                x = (torch.as_tensor(v.idx, device="cuda"),
                     None if dtype == "bool" else torch.as_tensor(np.asarray(v.val, np.float32), device="cuda"))
                vf = M.vector_features(x)
                times = {}
                for p in plans:
                    label = repr(p)
                    try:
                        M.run_plan(x, p, y)
                    except Exception:
                        continue  # plan not available for this matrix (e.g. LDS too small)
                    ts = []
                    for _ in range(reps):
                        ev0.record()
                        M.run_plan(x, p, y)
                        ev1.record()
                        ev1.synchronize()
                        ts.append(ev0.elapsed_time(ev1))
                    times[label] = float(np.median(ts))
                rec = {"key": key, "matrix": name, "support": kind, "features": {**mf, **vf}, "times_ms": times}
                fout.write(json.dumps(rec) + "\n")
                fout.flush()
            print(f"[tune] {name}: done in {time.time() - t0:.1f}s", flush=True)
            del M


def _time_plans(M, x, y, plans, reps):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    times = {}
    for p in plans:
        try:
            M.run_plan(x, p, y)
        except Exception:
            continue  # plan not available for this matrix
        ts = []
        for _ in range(reps):
            ev0.record()
            M.run_plan(x, p, y)
            ev1.record()
            ev1.synchronize()
            ts.append(ev0.elapsed_time(ev1))
        times[repr(p)] = float(np.median(ts))
    return times


DRIVER_GRAPHS = {
    "rmat20_d16": lambda synth: synth.cfg2_matrix(),
    "rmat19_d16": lambda synth: synth.rmat(19, 16, 27),
    "rmat18_d32": lambda synth: synth.rmat(18, 32, 23),
}


def driver_sweep(out_path: str, reps: int = 5, graph: str = "rmat20_d16"):
    """Every candidate plan timed on the vectors the graph drivers produce
    on an R-MAT graph (R-MAT 2^20 by default, the setting of the paper's
    misprediction study, Section 6): the frontier of every BFS level (BOOL,
    from the lowest vertex with an out-edge) and the x of every incremental
    PageRank round (FP32, d = 0.85, eps = 1e-3 (1 - d) / n; round k's x is
    taken from the residual after k products). One record per vector, as
    the sweep writes them, with support "bfs" or "pagerank" and the plan the
    driver ran. Other graphs give driver vectors to train on that the
    R-MAT 2^20 evaluation does not contain."""
    import torch
    from . import BOOL, Matrix, all_plans, synth
    A = DRIVER_GRAPHS[graph](synth)
    plans = all_plans()
    dev = lambda a: torch.as_tensor(a, device="cuda")  # noqa: E731
    with open(out_path, "w") as fout:
        M = Matrix.from_host(A, dtype=BOOL)
        mf = M.features()
        outdeg = np.bincount(np.asarray(A.col_idx), minlength=A.n)
        src = int(np.nonzero(outdeg > 0)[0][0])
        level, used = M.bfs(src, push_only=True)
        lv = level.cpu().numpy()
        y = M.out_tensor()
        for L in range(M.bfs_levels):
            idx = np.nonzero(lv == L)[0].astype(np.int32)
            x = (dev(idx), None)
            rec = {"key": f"{graph}:bfs:{L}", "matrix": graph, "support": "bfs",
                   "features": {**mf, **M.vector_features(x)}, "times_ms": _time_plans(M, x, y, plans, reps),
                   "driver_plan": repr(used[L]) if L < len(used) else None}
            fout.write(json.dumps(rec) + "\n")
            print(f"[drivers] bfs level {L}: nnz_x {idx.size}", flush=True)
        del M
        M = Matrix.from_host(A)
        mf = M.features()
        d = 0.85
        eps = 1e-3 * (1 - d) / A.n
        _, used = M.pagerank(d, eps)
        k_total = M.pr_iters
        cols = dev(np.asarray(A.col_idx, np.int64))
        W = torch.zeros(A.n, dtype=torch.float32, device="cuda").index_add_(0, cols, M.vals)
        y = M.out_tensor()
        for k in range(k_total):
            _, r, _ = M.pagerank(d, eps, max_iters=k, want_residual=True)
            prop = (r.abs() > eps) & (W > 0)
            idx = torch.nonzero(prop).flatten().to(torch.int32)
            x = (idx, (r[idx.long()] / W[idx.long()]).contiguous())
            rec = {"key": f"{graph}:pagerank:{k}", "matrix": graph, "support": "pagerank",
                   "features": {**mf, **M.vector_features(x)}, "times_ms": _time_plans(M, x, y, plans, reps),
                   "driver_plan": repr(used[k])}
            fout.write(json.dumps(rec) + "\n")
            fout.flush()
            print(f"[drivers] pagerank round {k}: nnz_x {int(idx.numel())}", flush=True)


# ----------------------------------------------------------------------------- storage format
FORMAT_FEATURES = ("m", "n", "nnz", "max_row", "min_row", "avg_row", "relative_range", "var_nnz_row", "gini",
                   "padding", "ell_padding")
FORMATS = ("csr", "sell", "ell", "csr5")
SELL_SIGMA = 4096  # rows per sorting window of the sliced copy


def sell_padding(A) -> float:
    """Cells / nnz of the sliced ELLPACK copy of A (slices of 64 rows, rows
    sorted by descending length within windows of SELL_SIGMA rows)."""
    lens = np.diff(np.asarray(A.row_ptr, dtype=np.int64))
    m = len(lens)
    ns = (m + 63) // 64
    slot = np.zeros(ns * 64, dtype=np.int64)
    pos = 0
    for w0 in range(0, m, SELL_SIGMA):
        part = lens[w0:w0 + SELL_SIGMA]
        slot[pos:pos + len(part)] = part[np.argsort(-part, kind="stable")]
        pos += len(part)
    return float(slot.reshape(ns, 64).max(axis=1).sum() * 64) / max(1, int(lens.sum()))


def format_sweep(out_path: str, reps: int = 10, dtype: str = "f32"):
    """Training data of the storage-format pre-selector: on every corpus
    matrix, the SpMV of a dense x (FP32, or FP64 to check the tree on the
    other precision) by the fastest SpMV plan of a CSR handle against the
    sliced ELLPACK, the ELLPACK and the CSR5 copies of handles forced to
    keep them (null when the matrix is too skewed for a copy). One record
    per matrix."""
    import torch
    from . import F32, F64, Matrix, SpxError, plan
    code, tdt = (F64, torch.float64) if dtype == "f64" else (F32, torch.float32)
    csr_plans = [plan("spmv", "direct"), plan("spmv", "balanced"), plan("spmv", "balanced", tile=4096)]
    with open(out_path, "w") as fout:
        for name, gen in corpus():
            A = gen()
            x = torch.rand(A.n, device="cuda", dtype=tdt)
            y = torch.empty(A.m, device="cuda", dtype=tdt)
            Mc = Matrix.from_host(A, dtype=code, fmt="csr")
            feats = Mc.features()
            tc = _time_plans(Mc, x, y, csr_plans, reps)
            Mc.close()
            lens = np.diff(np.asarray(A.row_ptr, dtype=np.int64))
            ell = float(lens.max() * A.m) / max(1, int(lens.sum())) if A.m else 1.0
            rec = {"matrix": name, "features": dict(feats, padding=sell_padding(A), ell_padding=ell), "csr_ms": tc,
                   "sell_ms": None, "ell_ms": None, "csr5_ms": None}
            for fmt in ("sell", "ell", "csr5"):
                try:
                    Ms = Matrix.from_host(A, dtype=code, fmt=fmt)
                    rec[f"{fmt}_ms"] = _time_plans(Ms, x, y, [plan("spmv", "direct")], reps)[
                        repr(plan("spmv", "direct"))]
                    if fmt == "sell":
                        rec["features"]["padding"] = Ms.storage_format()[1]
                    Ms.close()
                except SpxError:
                    pass
            fout.write(json.dumps(rec) + "\n")
            fout.flush()
            ts = lambda v: "-" if v is None else f"{v * 1e3:.1f}"  # noqa: E731
            print(f"[format] {name}: csr {min(tc.values()) * 1e3:.1f} us, sell {ts(rec['sell_ms'])} us, "
                  f"ell {ts(rec['ell_ms'])} us, csr5 {ts(rec['csr5_ms'])} us", flush=True)


def _format_times(r):
    """(csr, sell, ell, csr5) SpMV times of a format record, inf where the
    copy was refused or not timed."""
    c = min(r["csr_ms"].values())
    f = lambda k: r.get(k) if r.get(k) is not None else float("inf")  # noqa: E731
    return [c, f("sell_ms"), f("ell_ms"), f("csr5_ms")]


def _format_row(r):
    f = dict(r["features"])
    if "ell_padding" not in f:  # records written before the ELL candidate
        f["ell_padding"] = f["max_row"] * f["m"] / max(1.0, f["nnz"])
    return [f[k] for k in FORMAT_FEATURES]


def format_train(path: str, out_path: str, max_depth: int = 3):
    """The storage-format tree from a format sweep: the class of the format
    (0 CSR, 1 sliced ELLPACK, 2 ELLPACK, 3 CSR5) that ran the SpMV fastest. Samples
    are weighted by the time the slowest available choice would lose
    (relative), and the tree is grown on all records (one per matrix, too
    few to hold some out); the report gives the time lost against always
    taking the fastest format, and the rows of the tree for the library's
    built-in table."""
    recs = [json.loads(l) for l in open(path) if l.strip()]
    X, y, w, T = [], [], [], []
    for r in recs:
        t = _format_times(r)
        best = min(t)
        worst = max(v for v in t if np.isfinite(v))
        X.append(_format_row(r))
        y.append(int(np.argmin(t)))
        w.append(abs(min(worst, 10 * best) - best) / best)
        T.append(t)
    X = np.asarray(X)
    T = np.asarray(T)
    tree = Cart(max_depth).fit(X, np.asarray(y), np.asarray(w) + 1e-3, len(FORMATS))
    pred = tree.predict(X)
    best = float(T.min(axis=1).sum())
    chosen = float(sum(T[i, p] if np.isfinite(T[i, p]) else T[i, 0] for i, p in enumerate(pred)))
    csr_only = float(T[:, 0].sum())
    # library rows: feature, threshold, left, right, class (-1 = internal)
    rows = [[int(n[0]), float(n[1]), int(n[2]), int(n[3]), int(n[4])] for n in tree.nodes]
    rep = {"records": len(recs), "fastest": {f: int(sum(1 for v in y if v == i)) for i, f in enumerate(FORMATS)},
           "accuracy": float(np.mean(pred == np.asarray(y))), "loss_vs_best": chosen / best - 1.0,
           "csr_only_loss_vs_best": csr_only / best - 1.0, "features": list(FORMAT_FEATURES), "rows": rows}
    with open(out_path, "w") as f:
        json.dump(rep, f, indent=1)
    return rep


def format_evaluate(path: str, tree_path: str):
    """Time lost on a format sweep by a trained format tree (the rows of
    format_train's report), against always taking the fastest format and
    against CSR alone."""
    rows = json.load(open(tree_path))["rows"]
    recs = [json.loads(l) for l in open(path) if l.strip()]
    best = chosen = csr_only = 0.0
    hits = 0
    for r in recs:
        x = _format_row(r)
        i = 0
        while rows[i][4] < 0:
            i = rows[i][2] if x[rows[i][0]] <= rows[i][1] else rows[i][3]
        t = _format_times(r)
        pick = t[rows[i][4]] if np.isfinite(t[rows[i][4]]) else t[0]
        best += min(t)
        chosen += pick
        csr_only += t[0]
        hits += int(pick == min(t))
    return {"records": len(recs), "right_format": hits / len(recs), "loss_vs_best": chosen / best - 1.0,
            "csr_only_loss_vs_best": csr_only / best - 1.0}


def evaluate(paths, selector_paths, kinds=None):
    """Accuracy and time loss of saved selectors on timed records (the
    misprediction study): per selector and support kind, the share of
    vectors whose predicted plan is within 2 % of the fastest, the share
    with the right pattern, and the total and mean time over the best.
    kinds: the support kinds to keep (the BFS levels are timed in the BOOL
    semiring, the PageRank rounds in FP32)."""
    recs = []
    for p in paths:
        with open(p) as f:
            recs += [json.loads(l) for l in f if l.strip()]
    if kinds:
        recs = [r for r in recs if r.get("support", "uniform") in kinds]
    out = {}
    for sp in selector_paths:
        with open(sp) as f:
            sel = json.load(f)
        per = {}
        for r in recs:
            lab = labels(r)
            if lab is None:
                continue
            x = _feature_row(r)
            pat = _eval(sel["pattern"]["nodes"], x)
            dist = _eval(sel["distribution"][PATTERNS[pat]]["nodes"], x)
            wb = _eval(sel["writeback"]["nodes"], x) if pat == 2 else 0
            t = lab["times"].get((PATTERNS[pat], DISTS[dist], WBS[wb]), 2 * lab["best_ms"])
            o = per.setdefault(r.get("support", "uniform"), {"n": 0, "hit": 0, "pattern_hit": 0, "best": 0.0,
                                                            "chosen": 0.0, "loss": []})
            o["n"] += 1
            o["hit"] += int(t <= lab["best_ms"] * TIE)
            o["pattern_hit"] += int(pat == lab["pattern"])
            o["best"] += lab["best_ms"]
            o["chosen"] += t
            o["loss"].append(t / lab["best_ms"] - 1.0)
        out[os.path.basename(sp)] = {
            k: {"vectors": o["n"], "within_2pct_of_best": o["hit"] / o["n"], "pattern_accuracy": o["pattern_hit"] / o["n"],
                "total_best_ms": o["best"], "total_chosen_ms": o["chosen"],
                "total_loss": o["chosen"] / o["best"] - 1.0, "mean_loss": float(np.mean(o["loss"]))}
            for k, o in per.items()}
    return out


# ----------------------------------------------------------------------------- labels
def _parse_plan(label: str):
    body = label[label.index("(") + 1:label.index(")")]
    parts = [p.strip() for p in body.split(",")]
    return parts[0], parts[1], parts[2]


def _pick(cands):
    """cands: list of (time, cost, value); fastest, ties within 2% go to
    the cheaper alternative."""
    best_t = min(c[0] for c in cands)
    close = [c for c in cands if c[0] <= best_t * TIE]
    return min(close, key=lambda c: (c[1], c[0]))[2]


def labels(rec):
    """Per-factor labels of one record (the other factors at their best)."""
    t = {}
    for label, ms in rec["times_ms"].items():
        t[_parse_plan(label)] = ms
    if not t:
        return None

    def cost(pat, wb):
        return COST_ORDER.get((pat,) if pat != "csc_spmspv" else (pat, wb), 9)

    # pattern: pattern of the fastest kernel
    per_pat = {}
    for (pat, dist, wb), ms in t.items():
        per_pat.setdefault(pat, []).append(ms)
    pat = _pick([(min(v), cost(p, "atomic" if p == "csc_spmspv" else "none"), p) for p, v in per_pat.items()])
    # distribution: best within the pattern
    per_dist = {}
    for (p, dist, wb), ms in t.items():
        if p == pat:
            per_dist.setdefault(dist, []).append(ms)
    dist = _pick([(min(v), 0 if d == "direct" else 1, d) for d, v in per_dist.items()])
    # write-back: best within the column-major pattern and the chosen distribution
    cands = [(ms, cost("csc_spmspv", wb), wb) for (p, d, wb), ms in t.items() if p == "csc_spmspv" and d == dist]
    if not cands:
        cands = [(ms, cost("csc_spmspv", wb), wb) for (p, d, wb), ms in t.items() if p == "csc_spmspv"]
    wb = _pick(cands) if cands else "atomic"
    return {"pattern": PATTERNS.index(pat), "distribution": DISTS.index(dist), "writeback": WBS.index(wb),
            "best_ms": min(t.values()), "times": t}


# ----------------------------------------------------------------------------- CART
class Cart:
    """Binary decision tree with Gini impurity (CART), weighted samples."""

    def __init__(self, max_depth: int, min_leaf: int = 1):
        self.max_depth = max_depth
        self.min_leaf = min_leaf
        self.nodes = []  # [feature, threshold, left, right, class]

    def fit(self, X, y, w=None, n_classes=None):
        X = np.asarray(X, np.float64)
        y = np.asarray(y, np.int64)
        w = np.ones(len(y)) if w is None else np.asarray(w, np.float64)
        self.k = int(n_classes or (y.max() + 1))
        self.nodes = []
        self._grow(X, y, w, 0)
        return self

    def _leaf(self, y, w):
        cnt = np.bincount(y, weights=w, minlength=self.k)
        self.nodes.append([0, 0.0, 0, 0, int(np.argmax(cnt))])
        return len(self.nodes) - 1

    def _grow(self, X, y, w, depth):
        cnt = np.bincount(y, weights=w, minlength=self.k)
        if depth >= self.max_depth or (cnt > 0).sum() <= 1 or len(y) < 2 * self.min_leaf:
            return self._leaf(y, w)
        best = None
        tot = w.sum()
        parent = 1.0 - ((cnt / tot) ** 2).sum()
        for f in range(X.shape[1]):
            order = np.argsort(X[:, f], kind="stable")
            xs = X[order, f]
            ys = y[order]
            ws = w[order]
            onehot = np.zeros((len(ys), self.k))
            onehot[np.arange(len(ys)), ys] = ws
            left = np.cumsum(onehot, axis=0)[:-1]
            right = cnt[None, :] - left
            wl = left.sum(1)
            wr = right.sum(1)
            valid = (xs[1:] > xs[:-1]) & (np.arange(1, len(ys)) >= self.min_leaf) & \
                    (np.arange(len(ys) - 1, 0, -1) >= self.min_leaf) & (wl > 0) & (wr > 0)
            if not valid.any():
                continue
            with np.errstate(invalid="ignore", divide="ignore"):
                gl = 1.0 - ((left / wl[:, None]) ** 2).sum(1)
                gr = 1.0 - ((right / wr[:, None]) ** 2).sum(1)
                imp = (wl * gl + wr * gr) / tot
            imp[~valid] = np.inf
            i = int(np.argmin(imp))
            if best is None or imp[i] < best[0]:
                best = (imp[i], f, 0.5 * (xs[i] + xs[i + 1]))
        if best is None or best[0] >= parent - 1e-12:
            return self._leaf(y, w)
        _, f, thr = best
        me = len(self.nodes)
        self.nodes.append([f, float(thr), -1, -1, -1])
        mask = X[:, f] <= thr
        l = self._grow(X[mask], y[mask], w[mask], depth + 1)
        r = self._grow(X[~mask], y[~mask], w[~mask], depth + 1)
        self.nodes[me][2] = l
        self.nodes[me][3] = r
        return me

    def predict(self, X):
        X = np.asarray(X, np.float64)
        out = np.empty(len(X), np.int64)
        for i, row in enumerate(X):
            j = 0
            while self.nodes[j][4] < 0:
                f, thr, l, r, _ = self.nodes[j]
                j = l if row[f] <= thr else r
            out[i] = self.nodes[j][4]
        return out


def _weights(y, mode, T=None):
    """Sample weights: uniform, balanced classes, or regret (how much time
    choosing the worst alternative would cost, relative to the best, from
    the per-class times T; clipped to [0.02, 2])."""
    if mode == "uniform":
        return np.ones(len(y))
    if mode == "regret":
        fin = np.where(np.isfinite(T), T, np.nan)
        best = np.nanmin(fin, axis=1)
        worst = np.nanmax(fin, axis=1)
        return np.clip((worst - best) / best, 0.02, 2.0)
    cls, cnt = np.unique(y, return_counts=True)
    wmap = {c: len(y) / (len(cls) * n) for c, n in zip(cls, cnt)}
    return np.array([wmap[c] for c in y])


def _time_loss(T, pred):
    """Mean relative time lost by choosing class pred[i] instead of the
    fastest (an alternative with no timing counts as a loss of 1)."""
    best = np.min(np.where(np.isfinite(T), T, np.inf), axis=1)
    chosen = T[np.arange(len(pred)), pred]
    loss = np.where(np.isfinite(chosen), chosen / best - 1.0, 1.0)
    return float(np.mean(loss))


def grid_search(X, y, n_classes, seed=0, T=None, score_time=False):
    """max_depth 1..10 x sample weighting {balanced, uniform, and regret when
    per-class times T are given}, 3-fold CV. The score is accuracy, or with
    score_time 1 - the mean relative time lost against the fastest class."""
    rng = np.random.default_rng(seed)
    idx = rng.permutation(len(y))
    folds = np.array_split(idx, 3)
    best = None
    modes = ("balanced", "uniform") + (("regret",) if T is not None else ())
    for depth in range(1, 11):
        for cw in modes:
            scores = []
            for k in range(3):
                te = folds[k]
                tr = np.concatenate([folds[j] for j in range(3) if j != k])
                if len(tr) == 0 or len(te) == 0:
                    continue
                w = _weights(y[tr], cw, None if T is None else T[tr])
                t = Cart(depth).fit(X[tr], y[tr], w, n_classes)
                pred = t.predict(X[te])
                scores.append((pred == y[te]).mean() if not score_time else 1.0 - _time_loss(T[te], pred))
            sc = float(np.mean(scores)) if scores else 0.0
            if best is None or sc > best[0] + 1e-9:
                best = (sc, depth, cw)
    return best


def train(paths, out_path, all_features=False, seed=0):
    recs = []
    for p in paths:
        with open(p) as f:
            recs += [json.loads(l) for l in f if l.strip()]
    rows = []
    for r in recs:
        lab = labels(r)
        if lab is None:
            continue
        rows.append((r, lab))
    feats = FEATURES if all_features else CHEAP
    fidx = [FEATURES.index(f) for f in feats]
    X = np.array([_feature_row(r) for r, _ in rows], np.float64)
    Xs = X[:, fidx]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(rows))
    ntr = int(round(0.7 * len(rows)))
    tr, te = perm[:ntr], perm[ntr:]
    report = {"records": len(rows), "train": len(tr), "test": len(te), "features": list(feats)}
    trees = {}

    def fit_tree(name, ysel, mask, n_classes, tsel=None):
        y = np.array([ysel(lab) for _, lab in rows])
        T = None if tsel is None else np.array([tsel(lab) for _, lab in rows], np.float64)
        trm = tr[mask[tr]]
        tem = te[mask[te]]
        if len(trm) == 0:
            return None
        acc, depth, cw = grid_search(Xs[trm], y[trm], n_classes, seed, None if T is None else T[trm])
        t = Cart(depth).fit(Xs[trm], y[trm], _weights(y[trm], cw, None if T is None else T[trm]), n_classes)
        test_acc = float((t.predict(Xs[tem]) == y[tem]).mean()) if len(tem) else float("nan")
        report[name] = {"cv_score": acc, "max_depth": depth, "class_weight": cw, "test_acc": test_acc,
                        "n_train": int(len(trm)), "n_test": int(len(tem)),
                        "classes": np.bincount(y[trm], minlength=n_classes).tolist()}
        # map feature columns back to Table 1 ids for the library
        nodes = [[fidx[n[0]] if n[4] < 0 else 0, n[1], n[2], n[3], n[4]] for n in t.nodes]
        return {"nodes": nodes, "max_depth": depth, "class_weight": cw}

    def class_times(l, factor, pat=None):
        """Per-class times of one factor, the others at their best (inf
        where a class has no timing)."""
        t = l["times"]
        if factor == "pattern":
            return [min((ms for (p, d, w), ms in t.items() if p == c), default=np.inf) for c in PATTERNS]
        if factor == "distribution":
            return [min((ms for (p, d, w), ms in t.items() if p == pat and d == c), default=np.inf) for c in DISTS]
        dist = DISTS[l["distribution"]]
        return [min((ms for (p, d, w), ms in t.items() if p == "csc_spmspv" and d == dist and w == c),
                    default=np.inf) for c in WBS]

    allm = np.ones(len(rows), bool)
    trees["pattern"] = fit_tree("pattern", lambda l: l["pattern"], allm, 3, lambda l: class_times(l, "pattern"))
    trees["distribution"] = {}
    for pi, pn in enumerate(PATTERNS):
        # distribution labels of records whose best pattern is this one; fall
        # back to all records if the pattern never wins
        def dsel(l, pi=pi):
            ts = {k: v for k, v in l["times"].items() if k[0] == PATTERNS[pi]}
            if not ts:
                return 0
            per = {}
            for (p, d, w), ms in ts.items():
                per.setdefault(d, []).append(ms)
            return DISTS.index(_pick([(min(v), 0 if d == "direct" else 1, d) for d, v in per.items()]))
        mask = np.array([l["pattern"] == pi for _, l in rows])
        if mask.sum() < 10:
            mask = allm
        t = fit_tree(f"distribution_{pn}", dsel, mask, 2, lambda l, pn=pn: class_times(l, "distribution", pn))
        trees["distribution"][pn] = t or {"nodes": [[0, 0, 0, 0, 0]]}
    mask = np.array([l["pattern"] == 2 for _, l in rows])
    if mask.sum() < 10:
        mask = allm
    trees["writeback"] = fit_tree("writeback", lambda l: l["writeback"], mask, len(WBS),
                                  lambda l: class_times(l, "writeback"))
    # selection quality against exhaustive search on the held-out part:
    # time of the predicted kernel vs the fastest kernel
    out = {"format": "spx-selector-v1", "source": "tuned on MI355X timings", "report": report, **trees}
    loss = []
    hits = 0
    for i in te:
        r, lab = rows[i]
        x = Xs[i]
        pat = _eval(trees["pattern"]["nodes"], X[i])
        dist = _eval(trees["distribution"][PATTERNS[pat]]["nodes"], X[i])
        wb = _eval(trees["writeback"]["nodes"], X[i]) if pat == 2 else 0
        key = (PATTERNS[pat], DISTS[dist], WBS[wb])
        t_pred = lab["times"].get(key)
        if t_pred is None:
            continue
        loss.append(t_pred / lab["best_ms"] - 1.0)
        hits += int(t_pred <= lab["best_ms"] * TIE)
    report["held_out_mean_loss_vs_exhaustive"] = float(np.mean(loss)) if loss else None
    report["held_out_within_2pct_of_best"] = hits / max(1, len(loss))
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    return report


# ----------------------------------------------------------------------------- lazy trees
def _tree_leaves(nodes):
    return [i for i, n in enumerate(nodes) if int(n[4]) >= 0]


def _splice(host_nodes, count_nodes, ask):
    """host_nodes with every leaf in `ask` replaced by a copy of count_nodes
    (rows: feature, threshold, left, right, class; node 0 is the root)."""
    out = [list(n) for n in host_nodes]
    for leaf in sorted(ask):
        base = len(out)
        for n in count_nodes:
            n = list(n)
            if int(n[4]) < 0:
                n[2] = int(n[2]) + base
                n[3] = int(n[3]) + base
            out.append(n)
        # the leaf becomes the copy's root
        out[leaf] = list(out[base])
        out[base] = [0, 0.0, 0, 0, 0]  # unreachable placeholder (keeps indices)
    return out


def _gate(host_nodes, count_nodes, ask):
    """Tree that reads the counts for free once an earlier tree asked for
    them: counted > 0.5 -> count_nodes, else host_nodes with the ask leaves
    spliced."""
    h = _splice(host_nodes, count_nodes, ask)
    out = [["counted", 0.5, 1, 1 + len(h), -1]]
    for n in h:
        n = list(n)
        if int(n[4]) < 0:
            n[2] = int(n[2]) + 1
            n[3] = int(n[3]) + 1
        out.append(n)
    base = len(out)
    for n in count_nodes:
        n = list(n)
        if int(n[4]) < 0:
            n[2] = int(n[2]) + base
            n[3] = int(n[3]) + base
        out.append(n)
    return out


def lazy_selector(host_sel, count_sel, ask):
    """ask: {"pattern": leaves, "spmv"/"csr_spmspv"/"csc_spmspv": leaves of that
    distribution tree, "writeback": leaves} of the host trees at which the
    walk asks for the counts and continues on the count trees."""
    return {"format": "spx-selector-v1", "lazy": True,
            "pattern": {"nodes": _splice(host_sel["pattern"]["nodes"], count_sel["pattern"]["nodes"],
                                         ask.get("pattern", ()))},
            "distribution": {p: {"nodes": _gate(host_sel["distribution"][p]["nodes"],
                                                count_sel["distribution"][p]["nodes"], ask.get(p, ()))}
                             for p in PATTERNS},
            "writeback": {"nodes": _gate(host_sel["writeback"]["nodes"], count_sel["writeback"]["nodes"],
                                         ask.get("writeback", ()))}}


def _lazy_leaves(sel):
    """(tree, leaf index, number of classes) of every leaf of a selector."""
    out = [("pattern", i, len(PATTERNS)) for i in _tree_leaves(sel["pattern"]["nodes"])]
    for p in PATTERNS:
        out += [(p, i, len(DISTS)) for i in _tree_leaves(sel["distribution"][p]["nodes"])]
    out += [("writeback", i, len(WBS)) for i in _tree_leaves(sel["writeback"]["nodes"])]
    return out


def _tree_nodes(sel, tree):
    if tree == "pattern" or tree == "writeback":
        return sel[tree]["nodes"]
    return sel["distribution"][tree]["nodes"]


def train_lazy(paths, out_path, host_path, count_path, sync_us: float, seed=0, give_back=0.02, kinds=None):
    """Trees for run() that ask for nnz_s only where that pays (Section 6.3:
    features evaluated lazily, cheap rules first). Starting from the
    host-feature trees, leaves of the cascade are switched one at a time to
    "ask for the counts and continue on the trees that read them" while
    that lowers the training time; then every leaf of the resulting
    cascade takes the class that lowers it most (cost-sensitive leaf
    labels: the host trees were grown for accuracy, and a leaf that holds
    vectors the host features cannot tell apart, such as hub and uniform
    supports of one size, should hold the plan that is fastest over all of
    them). sync_us (the measured cost of the device count in a pipelined
    run() loop) is charged to every vector whose walk asks; once a vector
    has asked, the later trees of its cascade read the counts for free (the
    "counted" feature). The training time is the mean over support kinds of
    (total time / total of the fastest plans), so that no kind outweighs
    the others by its number of vectors, and a change is taken only while
    the uniform supports lose at most give_back more than under the host
    trees. kinds: the support kinds to keep (the driver files hold BFS
    levels timed in the BOOL semiring and PageRank rounds in FP32). 7:3
    split; the report gives the held-out loss of the host trees, of the
    count trees with the count charged on every vector, and of the lazy
    trees."""
    recs = []
    for p in paths:
        with open(p) as f:
            recs += [json.loads(l) for l in f if l.strip()]
    if kinds:
        recs = [r for r in recs if r.get("support", "uniform") in kinds]
    rows = [(r, lab) for r in recs for lab in [labels(r)] if lab is not None]
    host = json.load(open(host_path))
    cnt = json.load(open(count_path))
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(rows))
    ntr = int(round(0.7 * len(rows)))
    tr, te = perm[:ntr], perm[ntr:]
    X = [_feature_row(r) for r, _ in rows]
    kind = [r.get("support", "uniform") for r, _ in rows]

    def per_kind(sel, idx):
        tot, best = {}, {}
        for i in idx:
            _, lab = rows[i]
            pat, dist, wb, asked = _walk_cascade(sel, X[i])
            t = lab["times"].get((PATTERNS[pat], DISTS[dist], WBS[wb]), 2 * lab["best_ms"])
            k = kind[i]
            tot[k] = tot.get(k, 0.0) + t + (sync_us * 1e-3 if asked else 0.0)
            best[k] = best.get(k, 0.0) + lab["best_ms"]
        return {k: tot[k] / max(best[k], 1e-30) for k in tot}

    base = per_kind(host, tr)
    cap = base.get("uniform", np.inf) + give_back

    def cost(sel):
        r = per_kind(sel, tr)
        if r.get("uniform", 0.0) > cap:
            return np.inf
        return float(np.mean(list(r.values())))

    cands = [(t, l) for t, l, _ in _lazy_leaves(host)]
    ask = {}
    cur = cost(lazy_selector(host, cnt, ask))
    start = cur
    while True:
        best = None
        for tree, leaf in cands:
            if leaf in ask.get(tree, ()):
                continue
            trial = {k: set(v) for k, v in ask.items()}
            trial.setdefault(tree, set()).add(leaf)
            c = cost(lazy_selector(host, cnt, trial))
            if c < cur - 1e-6 and (best is None or c < best[0]):
                best = (c, tree, leaf)
        if best is None:
            break
        cur = best[0]
        ask.setdefault(best[1], set()).add(best[2])
        print(f"[lazy] ask at {best[1]} leaf {best[2]}: train time over the best {cur:.4f}", flush=True)
    sel = lazy_selector(host, cnt, ask)
    after_ask = cur
    relabeled = 0
    for _ in range(3):
        changed = False
        for tree, leaf, k in _lazy_leaves(sel):
            nodes = _tree_nodes(sel, tree)
            keep = int(nodes[leaf][4])
            for c in range(k):
                if c == keep:
                    continue
                nodes[leaf][4] = c
                v = cost(sel)
                if v < cur - 1e-6:
                    cur, keep, changed = v, c, True
                    relabeled += 1
            nodes[leaf][4] = keep
        if not changed:
            break
    print(f"[lazy] {relabeled} leaf labels changed: train time over the best {cur:.4f}", flush=True)
    sel["source"] = f"lazy counts over {os.path.basename(host_path)} and {os.path.basename(count_path)}"
    sel["sync_us"] = sync_us
    sel["ask"] = {k: sorted(v) for k, v in ask.items()}
    report = {"records": len(rows), "train": int(len(tr)), "test": int(len(te)), "sync_us": sync_us,
              "give_back": give_back,
              "train_time_over_best": {"host": start, "asks": after_ask, "lazy": cur,
                                       "per_kind": per_kind(sel, tr), "per_kind_host": base},
              "leaf_labels_changed": relabeled,
              "held_out": {"host": evaluate_lazy(rows, host, sync_us, te),
                           "counts_always": evaluate_lazy(rows, cnt, sync_us, te),
                           "lazy": evaluate_lazy(rows, sel, sync_us, te)}}
    sel["report"] = report
    with open(out_path, "w") as f:
        json.dump(sel, f, indent=1)
    return report


def _walk_cascade(sel, x):
    """(pattern, distribution, write-back, whether a count was asked for)."""
    asked = False

    def ev(nodes):
        nonlocal asked
        j = 0
        while int(nodes[j][4]) < 0:
            f = nodes[j][0]
            if f == "counted" or f == len(FEATURES):  # whether an earlier tree asked
                v = 1.0 if asked else 0.0
            else:
                f = FEATURES.index(f) if isinstance(f, str) else int(f)
                asked |= FEATURES[f] in COUNT_FEATURES
                v = x[f]
            j = int(nodes[j][2]) if v <= nodes[j][1] else int(nodes[j][3])
        return int(nodes[j][4])

    pat = ev(sel["pattern"]["nodes"])
    dist = ev(sel["distribution"][PATTERNS[pat]]["nodes"])
    wb = ev(sel["writeback"]["nodes"]) if pat == 2 else 0
    return pat, dist, wb, asked


def evaluate_lazy(rows, sel, sync_us, subset=None):
    """Per support kind: total and mean time over exhaustive search of a
    selector's plans, with sync_us added to every vector whose walk asked
    for a count, and the share of vectors that asked."""
    per = {}
    idx = range(len(rows)) if subset is None else subset
    for i in idx:
        r, lab = rows[i]
        x = _feature_row(r)
        pat, dist, wb, asked = _walk_cascade(sel, x)
        t = lab["times"].get((PATTERNS[pat], DISTS[dist], WBS[wb]), 2 * lab["best_ms"])
        t += sync_us * 1e-3 if asked else 0.0
        o = per.setdefault(r.get("support", "uniform"), {"n": 0, "asked": 0, "best": 0.0, "chosen": 0.0,
                                                        "loss": [], "hit": 0})
        o["n"] += 1
        o["asked"] += int(asked)
        o["best"] += lab["best_ms"]
        o["chosen"] += t
        o["loss"].append(t / lab["best_ms"] - 1.0)
        o["hit"] += int(t <= lab["best_ms"] * TIE)
    return {k: {"vectors": o["n"], "asked_for_counts": o["asked"] / o["n"], "total_loss": o["chosen"] / o["best"] - 1.0,
                "mean_loss": float(np.mean(o["loss"])), "within_2pct_of_best": o["hit"] / o["n"]}
            for k, o in per.items()}


# ----------------------------------------------------------------------------- model study
def study(paths, out_path, all_features=False, seed=0, jobs=8):
    """The model comparison of Section 5.2 on this GPU's timings: decision
    tree, SVM (RBF kernel), random forest and gradient tree boosting, each
    tuned by grid search with 3-fold cross-validation on the 70 % split
    (the paper's parameter ranges; the forest and boosting depth grids are
    thinned to even depths), scored on the held-out 30 %. Per factor:
    accuracy, and prediction cost per sample (scikit-learn, one batch
    over the test set, and one call per sample as a runtime would make),
    each relative to the decision tree. Per model family: the held-out time
    loss of its three-model cascade against exhaustive search. The SVM
    sees log1p-scaled, standardized features; the trees see them raw."""
    from sklearn.ensemble import GradientBoostingClassifier, RandomForestClassifier
    from sklearn.model_selection import GridSearchCV
    from sklearn.pipeline import make_pipeline
    from sklearn.preprocessing import FunctionTransformer, StandardScaler
    from sklearn.svm import SVC
    from sklearn.tree import DecisionTreeClassifier

    recs = []
    for p in paths:
        with open(p) as f:
            recs += [json.loads(l) for l in f if l.strip()]
    rows = [(r, lab) for r in recs for lab in [labels(r)] if lab is not None]
    feats = FEATURES if all_features else CHEAP
    fidx = [FEATURES.index(f) for f in feats]
    X = np.array([_feature_row(r) for r, _ in rows], np.float64)[:, fidx]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(rows))
    ntr = int(round(0.7 * len(rows)))
    tr, te = perm[:ntr], perm[ntr:]
    families = {
        "decision_tree": (DecisionTreeClassifier(random_state=seed),
                          {"max_depth": list(range(1, 11)), "class_weight": ["balanced", None]}),
        "svm": (make_pipeline(FunctionTransformer(np.log1p), StandardScaler(), SVC(kernel="rbf")),
                {"svc__C": [1, 10, 100, 1000], "svc__gamma": ["auto", "scale"]}),
        "random_forest": (RandomForestClassifier(random_state=seed),
                          {"n_estimators": [50, 100, 200, 500], "max_depth": [2, 4, 6, 8, 10]}),
        "gbdt": (GradientBoostingClassifier(random_state=seed),
                 {"learning_rate": [0.1, 0.01], "n_estimators": [50, 100, 200, 500], "max_depth": [2, 4, 6, 8]}),
    }
    factors = {
        "pattern": (np.array([lab["pattern"] for _, lab in rows]), np.ones(len(rows), bool)),
        "distribution": (np.array([lab["distribution"] for _, lab in rows]), np.ones(len(rows), bool)),
        "writeback": (np.array([lab["writeback"] for _, lab in rows]),
                      np.array([lab["pattern"] == 2 for _, lab in rows])),
    }
    report = {"records": len(rows), "train": int(len(tr)), "test": int(len(te)), "features": list(feats),
              "factors": {}, "cascade": {}}
    fitted = {}
    for fname, (y, mask) in factors.items():
        trm, tem = tr[mask[tr]], te[mask[te]]
        out = {}
        for mname, (est, grid) in families.items():
            t0 = time.time()
            g = GridSearchCV(est, grid, cv=3, n_jobs=jobs).fit(X[trm], y[trm])
            best = g.best_estimator_
            fitted[(fname, mname)] = best
            acc = float((best.predict(X[tem]) == y[tem]).mean())
            reps = 20
            t1 = time.perf_counter()
            for _ in range(reps):
                best.predict(X[tem])
            batch_us = (time.perf_counter() - t1) / (reps * max(1, len(tem))) * 1e6
            one = X[tem][:1]
            t1 = time.perf_counter()
            for _ in range(200):
                best.predict(one)
            call_us = (time.perf_counter() - t1) / 200 * 1e6
            out[mname] = {"params": {k: (v if isinstance(v, (int, float, str)) or v is None else str(v))
                                     for k, v in g.best_params_.items()},
                          "cv_score": float(g.best_score_), "test_acc": acc, "us_per_sample_batch": batch_us,
                          "us_per_call": call_us, "fit_s": time.time() - t0, "n_test": int(len(tem))}
            print(f"[study] {fname:12s} {mname:14s} acc {acc:.3f}  {batch_us:8.2f} us/sample  "
                  f"{call_us:8.1f} us/call  {g.best_params_}", flush=True)
        dt = out["decision_tree"]
        for m in out.values():
            m["acc_vs_tree"] = m["test_acc"] - dt["test_acc"]
            m["overhead_batch_vs_tree"] = m["us_per_sample_batch"] / dt["us_per_sample_batch"]
            m["overhead_call_vs_tree"] = m["us_per_call"] / dt["us_per_call"]
        report["factors"][fname] = out
    for mname in families:
        loss, hits = [], 0
        for i in te:
            _, lab = rows[i]
            x = X[i:i + 1]
            pat = int(fitted[("pattern", mname)].predict(x)[0])
            dist = int(fitted[("distribution", mname)].predict(x)[0])
            wb = int(fitted[("writeback", mname)].predict(x)[0]) if pat == 2 else 0
            t = lab["times"].get((PATTERNS[pat], DISTS[dist], WBS[wb]))
            if t is None:
                continue
            loss.append(t / lab["best_ms"] - 1.0)
            hits += int(t <= lab["best_ms"] * TIE)
        report["cascade"][mname] = {"held_out_mean_loss_vs_exhaustive": float(np.mean(loss)) if loss else None,
                                    "held_out_within_2pct_of_best": hits / max(1, len(loss))}
    with open(out_path, "w") as f:
        json.dump(report, f, indent=1)
    return report


def _eval(nodes, xrow):
    j = 0
    while nodes[j][4] < 0:
        f, thr, l, r, _ = nodes[j]
        j = l if xrow[int(f)] <= thr else r
    return int(nodes[j][4])


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--out", required=True)
    s.add_argument("--reps", type=int, default=5)
    s.add_argument("--quick", action="store_true")
    s.add_argument("--dtype", choices=("f32", "bool"), default="f32")
    s.add_argument("--supports", default="uniform",
                   help="comma-separated vector kinds: " + ", ".join(SUPPORTS))
    dr = sub.add_parser("drivers")
    dr.add_argument("--out", required=True)
    dr.add_argument("--reps", type=int, default=5)
    dr.add_argument("--graph", choices=sorted(DRIVER_GRAPHS), default="rmat20_d16")
    ev = sub.add_parser("evaluate")
    ev.add_argument("data", nargs="+")
    ev.add_argument("--selectors", nargs="+", required=True)
    ev.add_argument("--out")
    ev.add_argument("--kinds", default="", help="support kinds to keep, comma-separated (default: all)")
    st = sub.add_parser("study")
    st.add_argument("data", nargs="+")
    st.add_argument("--out", required=True)
    st.add_argument("--all-features", action="store_true")
    st.add_argument("--jobs", type=int, default=8)
    fs = sub.add_parser("formats")
    fs.add_argument("--out", required=True)
    fs.add_argument("--reps", type=int, default=10)
    fs.add_argument("--dtype", choices=("f32", "f64"), default="f32")
    fe = sub.add_parser("formats-evaluate")
    fe.add_argument("data")
    fe.add_argument("--tree", required=True)
    ft = sub.add_parser("formats-train")
    ft.add_argument("data")
    ft.add_argument("--out", required=True)
    ft.add_argument("--max-depth", type=int, default=3)
    tl = sub.add_parser("train-lazy")
    tl.add_argument("data", nargs="+")
    tl.add_argument("--out", required=True)
    tl.add_argument("--sync-us", type=float, required=True,
                    help="measured cost of run()'s device count and stream synchronization")
    tl.add_argument("--host", required=True, help="host-feature trees (JSON)")
    tl.add_argument("--counts", required=True, help="trees that read nnz_s (JSON)")
    tl.add_argument("--give-back", type=float, default=0.02,
                    help="largest loss over the host trees allowed on uniform supports")
    tl.add_argument("--kinds", default="", help="support kinds to keep, comma-separated (default: all)")
    el = sub.add_parser("evaluate-lazy")
    el.add_argument("data", nargs="+")
    el.add_argument("--selectors", nargs="+", required=True)
    el.add_argument("--sync-us", type=float, required=True)
    el.add_argument("--out")
    t = sub.add_parser("train")
    t.add_argument("data", nargs="+")
    t.add_argument("--out", required=True)
    t.add_argument("--all-features", action="store_true")
    a = ap.parse_args(argv)
    if a.cmd == "train-lazy":
        kinds = tuple(k for k in a.kinds.split(",") if k) or None
        print(json.dumps(train_lazy(a.data, a.out, a.host, a.counts, a.sync_us, give_back=a.give_back, kinds=kinds),
                         indent=1))
        return
    if a.cmd == "evaluate-lazy":
        recs = []
        for p in a.data:
            with open(p) as f:
                recs += [json.loads(l) for l in f if l.strip()]
        rows = [(r, lab) for r in recs for lab in [labels(r)] if lab is not None]
        rep = {os.path.basename(sp): evaluate_lazy(rows, json.load(open(sp)), a.sync_us) for sp in a.selectors}
        if a.out:
            with open(a.out, "w") as f:
                json.dump(rep, f, indent=1)
        print(json.dumps(rep, indent=1))
        return
    if a.cmd == "drivers":
        driver_sweep(a.out, a.reps, a.graph)
        return
    if a.cmd == "formats":
        format_sweep(a.out, a.reps, a.dtype)
        return
    if a.cmd == "formats-evaluate":
        print(json.dumps(format_evaluate(a.data, a.tree), indent=1))
        return
    if a.cmd == "formats-train":
        print(json.dumps(format_train(a.data, a.out, a.max_depth), indent=1))
        return
    if a.cmd == "evaluate":
        rep = evaluate(a.data, a.selectors, tuple(k for k in a.kinds.split(",") if k) or None)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(rep, f, indent=1)
        print(json.dumps(rep, indent=1))
        return
    if a.cmd == "study":
        rep = study(a.data, a.out, a.all_features, jobs=a.jobs)
        print(json.dumps(rep["cascade"], indent=1))
        return
    if a.cmd == "sweep":
        kinds = tuple(k for k in a.supports.split(",") if k)
        if any(k not in SUPPORTS for k in kinds):
            ap.error(f"--supports: kinds are {', '.join(SUPPORTS)}")
        sweep(a.out, a.reps, a.quick, dtype=a.dtype, supports=kinds)
    else:
        rep = train(a.data, a.out, a.all_features)
        print(json.dumps(rep, indent=1))


if __name__ == "__main__":
    main()
