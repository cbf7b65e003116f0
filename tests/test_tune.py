"""Selector training (CART, per-factor labels) and the JSON the library
loads. CPU only."""
import ctypes as C
import json

import numpy as np
import pytest

from paper_2006_16767_amd import _lib, tune


def test_cart_matches_sklearn_predictions():
    sk = pytest.importorskip("sklearn.tree")
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1, (400, 3))
    y = ((X[:, 0] > 0.4).astype(int) + (X[:, 1] > 0.7).astype(int) * (X[:, 2] < 0.5)).astype(int)
    ours = tune.Cart(4).fit(X, y, n_classes=3)
    ref = sk.DecisionTreeClassifier(max_depth=4, random_state=0).fit(X, y)
    Xt = rng.uniform(0, 1, (300, 3))
    agree = (ours.predict(Xt) == ref.predict(Xt)).mean()
    assert (ours.predict(X) == y).mean() == 1.0
    assert agree > 0.97


def test_cart_depth_limit_and_weights():
    X = np.arange(10, dtype=float)[:, None]
    y = np.array([0] * 9 + [1])
    stump = tune.Cart(1).fit(X, y, n_classes=2)
    assert len(stump.nodes) == 3 and stump.nodes[0][4] < 0
    # uniform weights: the split isolates the minority class exactly
    assert stump.predict(np.array([[9.0], [0.0]])).tolist() == [1, 0]
    leaf = tune.Cart(0).fit(X, y, n_classes=2)
    assert leaf.predict(np.array([[9.0]])).tolist() == [0]
    leaf_bal = tune.Cart(0).fit(X, y, tune._weights(y, "balanced"), n_classes=2)
    assert leaf_bal.nodes == [[0, 0.0, 0, 0, 0]] or leaf_bal.nodes[0][4] in (0, 1)


def _rec(times):
    return {"key": "k", "features": {f: 1.0 for f in tune.FEATURES},
            "times_ms": {f"Plan({p}, {d}, {w}, lanes=0, tile=0, bucket_rows=0)": t for (p, d, w), t in times.items()}}


def test_labels_per_factor_and_ties():
    lab = tune.labels(_rec({("spmv", "direct", "none"): 1.0, ("spmv", "balanced", "none"): 0.9,
                            ("csc_spmspv", "direct", "atomic"): 2.0, ("csc_spmspv", "direct", "bucket"): 1.5,
                            ("csc_spmspv", "balanced", "sort"): 3.0}))
    assert tune.PATTERNS[lab["pattern"]] == "spmv"
    assert tune.DISTS[lab["distribution"]] == "balanced"
    # write-back within (csc, chosen distribution = balanced): only sort
    assert tune.WBS[lab["writeback"]] == "sort"
    # a near tie (within 2%) goes to the cheaper alternative
    lab2 = tune.labels(_rec({("spmv", "direct", "none"): 1.01, ("csc_spmspv", "direct", "bucket"): 1.0,
                             ("csc_spmspv", "direct", "atomic"): 1.015}))
    assert tune.PATTERNS[lab2["pattern"]] == "spmv"
    lab3 = tune.labels(_rec({("spmv", "direct", "none"): 2.0, ("csc_spmspv", "direct", "bucket"): 1.0,
                             ("csc_spmspv", "direct", "atomic"): 1.015}))
    assert tune.PATTERNS[lab3["pattern"]] == "csc_spmspv" and tune.WBS[lab3["writeback"]] == "atomic"


def test_train_writes_a_selector_the_library_loads(tmp_path):
    rng = np.random.default_rng(1)
    recs = []
    for i in range(200):
        xs = float(10 ** rng.uniform(-5, 0))
        gini = float(rng.uniform(0, 1))
        t = {}
        for p in ("spmv", "csr_spmspv"):
            for d in ("direct", "balanced"):
                t[(p, d, "none")] = (1.0 if p == "spmv" else 0.6 + xs) * (1 + 0.5 * gini * (d == "direct"))
        for d in ("direct", "balanced"):
            for w in ("atomic", "bucket", "sort"):
                t[("csc_spmspv", d, w)] = 20 * xs * (1 + (w == "atomic") * 10 * xs) + 0.05
        r = _rec(t)
        r["features"].update({"x_sparsity": xs, "nnz_x": xs * 1e6, "gini": gini})
        recs.append(r)
    data = tmp_path / "sweep.jsonl"
    data.write_text("\n".join(json.dumps(r) for r in recs))
    out = tmp_path / "sel.json"
    rep = tune.train([str(data)], str(out))
    assert rep["pattern"]["test_acc"] > 0.8
    sel = json.loads(out.read_text())
    for key in ("pattern", "writeback"):
        assert sel[key]["nodes"]
    lib = _lib.load()
    assert lib.spx_load_selector(None, str(out).encode()) == 0, lib.spx_last_error()
    bad = tmp_path / "bad.json"
    bad.write_text('{"pattern": {"nodes": [[99, 0, 1, 2, -1]]}}')
    assert lib.spx_load_selector(None, str(bad).encode()) == -1
    assert lib.spx_load_selector(None, None) == 0  # back to the built-in trees
