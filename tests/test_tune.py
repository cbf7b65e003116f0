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
    _restore_shipped(lib)


def _restore_shipped(lib):
    """The package's default trees, as the binding loads them, so that
    later tests in the process see the usual defaults."""
    import os
    pkg = os.path.dirname(tune.__file__)
    for name in ("selector_mi355x.json", "selector_mi355x_nnz_s.json"):
        path = os.path.join(pkg, name)
        if os.path.exists(path):
            assert lib.spx_load_selector(None, path.encode()) == 0, lib.spx_last_error()


def _csr_rows(lens):
    rp = np.zeros(len(lens) + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    return type("A", (), {"row_ptr": rp})()


def test_sell_padding_by_hand():
    """Slices of 64 rows padded to their longest row, rows sorted by length
    (descending) within windows of 4096 rows before slicing."""
    # one slice: 64 rows, longest 5, 10 entries in all -> 64 * 5 cells
    lens = [5, 1, 1, 3] + [0] * 60
    assert tune.sell_padding(_csr_rows(lens)) == pytest.approx(64 * 5 / 10)
    # 128 rows, even length 2: no padding
    assert tune.sell_padding(_csr_rows([2] * 128)) == 1.0
    # 128 rows, 64 of length 4 interleaved with 64 of length 1: the sort
    # inside the window groups them, so the slices are 4 wide and 1 wide
    lens = [4, 1] * 64
    assert tune.sell_padding(_csr_rows(lens)) == pytest.approx((64 * 4 + 64 * 1) / (64 * 5))
    # the same rows split by the window: 4096 one-entry rows first, then the
    # pattern, which the sort cannot reach across the window boundary
    lens = [1] * 4096 + [4, 1] * 64
    cells = 4096 + 64 * 4 + 64 * 1
    assert tune.sell_padding(_csr_rows(lens)) == pytest.approx(cells / (4096 + 64 * 5))
    # 3 rows: one partly filled slice
    assert tune.sell_padding(_csr_rows([2, 0, 1])) == pytest.approx(64 * 2 / 3)


def test_format_train_separates_the_formats(tmp_path):
    """Sliced copy faster exactly on the even-row, many-row records: the
    tree learns it, loses nothing on its training set, and its rows are in
    the library's table form (the project CART, no scikit-learn)."""
    path = tmp_path / "formats.jsonl"
    rng = np.random.default_rng(1)
    with open(path, "w") as f:
        for i in range(40):
            m = float(rng.choice([4096, 65536, 1 << 20]))
            var = float(rng.choice([0.0, 0.3, 5.0]))
            sell_wins = m > 40000 and var < 1.0
            feats = {k: 1.0 for k in tune.FORMAT_FEATURES}
            feats.update(m=m, n=m, var_nnz_row=var, padding=1.0 + var)
            csr = 10.0
            rec = {"matrix": f"m{i}", "features": feats, "csr_ms": {"Plan(spmv)": csr},
                   "sell_ms": 8.0 if sell_wins else (None if var > 1 else 12.0)}
            f.write(json.dumps(rec) + "\n")
    rep = tune.format_train(str(path), str(tmp_path / "tree.json"))
    assert rep["accuracy"] == 1.0 and rep["loss_vs_best"] == pytest.approx(0.0)
    assert rep["csr_only_loss_vs_best"] > 0
    for row in rep["rows"]:
        assert len(row) == 5 and (row[4] in (0, 1) or (row[4] == -1 and 0 <= row[0] < len(tune.FORMAT_FEATURES)))


def test_lazy_splice_asks_only_at_chosen_leaves():
    """Leaf splicing: a vector reaching an 'ask' leaf of the host pattern
    tree continues on the count tree (and is charged the count); the later
    trees read the counts for free through the 'counted' gate; vectors on
    other leaves never ask."""
    F = tune.FEATURES
    nx, ns = F.index("nnz_x"), F.index("nnz_s")
    leaf = lambda c: [0, 0.0, 0, 0, c]  # noqa: E731
    host = {"pattern": {"nodes": [[nx, 100.0, 1, 2, -1], leaf(2), leaf(0)]},
            "distribution": {p: {"nodes": [leaf(0)]} for p in tune.PATTERNS},
            "writeback": {"nodes": [leaf(1)]}}
    cnt = {"pattern": {"nodes": [[ns, 1000.0, 1, 2, -1], leaf(2), leaf(1)]},
           "distribution": {p: {"nodes": [leaf(1)]} for p in tune.PATTERNS},
           "writeback": {"nodes": [[ns, 5.0, 1, 2, -1], leaf(4), leaf(2)]}}
    sel = tune.lazy_selector(host, cnt, {"pattern": {1}})
    row = lambda a, b: [1.0] * 9 + [a, a / 1e4, b, b / 1e6, b / max(1.0, a)]  # noqa: E731
    # nnz_x <= 100 -> asks; nnz_s decides pattern; dist/wb from the count trees (counted)
    assert tune._walk_cascade(sel, row(50, 500)) == (2, 1, 2, True)
    assert tune._walk_cascade(sel, row(50, 3)) == (2, 1, 4, True)
    assert tune._walk_cascade(sel, row(50, 5000)) == (1, 1, 0, True)
    # nnz_x > 100 -> host leaf, no count, host distribution (and no write-back for SpMV)
    assert tune._walk_cascade(sel, row(500, 5000)) == (0, 0, 0, False)
    # asking at a write-back leaf only: the host pattern, then the count tree at the leaf
    sel2 = tune.lazy_selector(host, cnt, {"writeback": {0}})
    assert tune._walk_cascade(sel2, row(50, 3)) == (2, 0, 4, True)
    assert tune._walk_cascade(sel2, row(500, 3)) == (0, 0, 0, False)


def test_shipped_selectors_load():
    """Every tree file the package ships parses in the library (host only:
    with no handle the trees become the defaults), the lazy trees with
    their "counted" gate nodes included."""
    import glob
    import os
    lib = _lib.load()
    pkg = os.path.dirname(tune.__file__)
    files = sorted(glob.glob(os.path.join(pkg, "selector_mi355x*.json")))
    assert any(f.endswith("_lazy.json") for f in files)
    try:
        for f in files:
            assert lib.spx_load_selector(None, f.encode()) == 0, (f, lib.spx_last_error())
    finally:
        assert lib.spx_load_selector(None, None) == 0
        _restore_shipped(lib)
