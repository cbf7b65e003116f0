"""Profiling drivers and rocprofv3 summaries.

The drivers run one piece of work so that a counter pass
(`rocprofv3 --pmc ...`) sees exactly the dispatches of interest; the
summaries read the rocpd databases rocprofv3 writes (`*_results.db`).

  python -m paper_2006_16767_amd.prof vector K [--reps R] [--plan P,D[,W]]
      run() (or run_plan with the given plan) on vector K of the R-MAT 2^20
      (degree 16) sweep, R times after one warm-up call; prints the plan and
      its kernel-name stems.
  python -m paper_2006_16767_amd.prof batch [--B 512] [--reps R]
      run_batch on the 512-vector R-MAT 2^18 (degree 32) batch.
  python -m paper_2006_16767_amd.prof fc [--reps R]
      the pruned FC layer 16384 x 4096: fused forward, then dX and dvals
      in one backward call.
  python -m paper_2006_16767_amd.prof poisson [--k K] [--dtype f32|f64] [--reps R]
      run() on a dense x over the 7-point Poisson matrix on K^3 (128 by
      default; the format tree keeps the ELL copy for it).
  python -m paper_2006_16767_amd.prof copy [--mib M] [--reps R]
      a plain device-to-device copy of M MiB, R times (counter calibration:
      it reads and writes exactly M MiB).
  python -m paper_2006_16767_amd.prof kernels DB --title T --command C
      kernel-trace summary (markdown) of a `--kernel-trace --stats` db.
  python -m paper_2006_16767_amd.prof traffic --fetch DB --write DB
        --copy-fetch DB --copy-write DB --mib M (--vector K | --workload W) --out JSON
      HBM bytes per launch of vector K's kernels (or of workload W's, keyed
      by its name): FETCH_SIZE and WRITE_SIZE
      (KiB per dispatch) scaled by what the same counters read for the copy
      of M MiB; written with the hash of the library sources, so the figure
      is void once a kernel changes.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SWEEP_WORKLOAD = "rmat20_deg16_f32_sweep12"


def library_source_hash() -> str:
    """sha256 over the library's kernel and host sources, in name order."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if path.endswith((".hip", ".hpp", ".cpp", ".h")):
            h.update(os.path.basename(path).encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _local_includes(path: str) -> list[str]:
    out = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith('#include "'):
                inc = os.path.normpath(os.path.join(os.path.dirname(path), line.split('"')[1]))
                if os.path.exists(inc):
                    out.append(inc)
    return out


def kernel_source_hash(stems) -> str:
    """sha256 over the sources that define the given kernels (the files with
    a __global__ definition of each stem) and every local header they
    include, transitively: the figure measured on those kernels stays valid
    while these files are unchanged."""
    import re
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    files = set()
    for stem in stems:
        pat = re.compile(r"__global__[^;{]*?\b" + re.escape(stem) + r"\s*\(", re.S)
        for path in srcs:
            with open(path) as f:
                if pat.search(f.read()):
                    files.add(path)
    todo = list(files)
    while todo:
        for inc in _local_includes(todo.pop()):
            if inc not in files:
                files.add(inc)
                todo.append(inc)
    h = hashlib.sha256()
    for path in sorted(files):
        h.update(os.path.relpath(path, HERE).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def csr5_bitvector(M) -> bool:
    """Whether M's balanced bitvector SpMSpV (tile 0) runs over CSR5 tiles
    with the bitvector in LDS: the handle's SpMV format is CSR5 and n <=
    2^20."""
    return M.n <= (1 << 20) and M.storage_format()[0] == "csr5"


def kernel_names(p, column_sorted: bool = False, csr5_bits: bool = False) -> list[str]:
    """Kernel-name stems of the launches a plan makes. column_sorted: the
    handle keeps the column-sorted tiles (renumbered, n <= 2^21), which the
    balanced row-major plans with 2048-item tiles read; csr5_bits: see
    csr5_bitvector."""
    if p.pattern in (0, 1):
        if p.distribution == 0:
            return ["k_csr_direct"]
        if p.pattern == 1 and p.tile == 0 and csr5_bits:
            return ["k_c5_spmspv_lds", "k_c5_fixup"]
        if p.pattern == 1 and p.tile == 1:
            main = "k_csr_bitlds"
        elif column_sorted and p.tile != 4096:
            main = "k_csr_merge_sorted"
        else:
            main = "k_csr_merge"
        return [main, "k_csr_merge_fixup"]
    dist = "direct" if p.distribution == 0 else "merge"
    if p.writeback == 5:
        return (["k_merge_emit_direct"] if p.distribution == 0 else []) + ["k_merge_tile_sort", "k_merge_accumulate"]
    if p.writeback == 4:
        return [f"k_bucket_scatter_{dist}", "k_bucket_accumulate"]
    if p.writeback == 2:
        return [f"k_csc_{dist}_pairs", "k_radix_hist", "k_radix_scatter", "k_reduce_by_key"]
    stem = {1: "atomic", 3: "lds"}[p.writeback]
    return [f"k_csc_{dist}_{stem}"]


def _stem(name: str) -> str:
    """'void spx::k_csr_merge<0, false, 2048>(int, ...)' -> 'k_csr_merge'."""
    n = name.replace("void ", "").replace("spx::", "")
    for c in "<(":
        i = n.find(c)
        if i > 0:
            n = n[:i]
    return n.strip()


def _db(path: str) -> str:
    if os.path.isdir(path):
        found = sorted(glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True))
        if not found:
            raise SystemExit(f"no *_results.db under {path}")
        return found[-1]
    return path


def counter_per_dispatch(db: str, counter: str) -> list[tuple[int, str, float]]:
    """(dispatch id, kernel name, counter value summed over its instances),
    in dispatch order."""
    con = sqlite3.connect(_db(db))
    rows = con.execute(
        "select dispatch_id, kernel_name, sum(value) from counters_collection where counter_name = ? "
        "group by dispatch_id, kernel_name order by dispatch_id", (counter,)).fetchall()
    con.close()
    return [(int(d), k, float(v)) for d, k, v in rows]


def _mean_by_stem(rows, stems):
    """Mean per-dispatch value of each kernel stem, and its dispatch count."""
    out = {}
    for s in stems:
        vals = [v for _, k, v in rows if _stem(k) == s]
        out[s] = (sum(vals) / len(vals) if vals else None, len(vals))
    return out


def cmd_vector(args):
    import torch
    from . import Matrix, plan
    from . import synth
    A = synth.cfg2_matrix()
    vecs = synth.cfg2_vectors(A.n)
    v = vecs[args.k]
    M = Matrix.from_host(A)
    x = (torch.as_tensor(v.idx, device="cuda"), torch.as_tensor(v.val, device="cuda"))
    y = M.out_tensor()
    if args.plan:
        p = plan(*args.plan.split(","))
        call = lambda: M.run_plan(x, p, y)  # noqa: E731
    else:
        call = lambda: M.run(x, y)  # noqa: E731
    call()
    torch.cuda.synchronize()
    p = M.last_plan()
    sorted_tiles = M.column_order() is not None and M.n <= (1 << 21)
    print(f"[prof] vector {args.k}: nnz_x={v.nnz} plan={p} kernels={kernel_names(p, sorted_tiles, csr5_bitvector(M))}",
          flush=True)
    for _ in range(args.reps):
        call()
    torch.cuda.synchronize()
    print(f"[prof] {args.reps} runs done", flush=True)


def cmd_batch(args):
    import numpy as np
    import torch
    from . import Matrix
    from . import synth
    A = synth.cfg4_rmat()
    M = Matrix.from_host(A)
    vecs = synth.cfg4_rmat_batch(A.n, args.B)
    ptr = np.zeros(len(vecs) + 1, np.int32)
    ptr[1:] = np.cumsum([v.nnz for v in vecs])
    dev = lambda a: torch.as_tensor(a, device="cuda")  # noqa: E731
    idx = dev(np.concatenate([v.idx for v in vecs]).astype(np.int32))
    val = dev(np.concatenate([np.asarray(v.val, np.float32) for v in vecs]))
    Y = M.out_tensor(len(vecs))
    M.run_batch(dev(ptr), idx, val, Y)
    torch.cuda.synchronize()
    print(f"[prof] batch of {len(vecs)} on R-MAT 2^18 (degree 32), status {M.batch_status()}", flush=True)
    for _ in range(args.reps):
        M.run_batch(dev(ptr), idx, val, Y)
    torch.cuda.synchronize()
    print(f"[prof] {args.reps} runs done", flush=True)


def cmd_fc(args):
    import numpy as np
    import torch
    from . import Matrix
    from . import synth
    A = synth.cfg5_matrix()
    M = Matrix.from_host(A)
    Xh = np.zeros((64, A.n), np.float32)
    for b, v in enumerate(synth.cfg5_activations()):
        Xh[b, v.idx] = v.val
    X = torch.as_tensor(Xh, device="cuda")
    G = torch.as_tensor(synth.cfg5_upstream(), device="cuda")
    Y = M.out_tensor(64)
    for _ in range(args.reps + 1):
        M.spmv_batch(X, Y)
        M.backward(G, X)  # dX and dvals from one B-minor copy of G
    torch.cuda.synchronize()
    print(f"[prof] FC layer 16384 x 4096: {args.reps + 1} forward + backward passes done", flush=True)


def cmd_bfs(args):
    import numpy as np
    import torch
    from . import BOOL, Matrix
    from . import synth
    A = synth.cfg2_matrix()
    M = Matrix.from_host(A, dtype=BOOL)
    outdeg = np.bincount(A.col_idx, minlength=A.n)
    src = 0 if outdeg[0] > 0 else int(np.nonzero(outdeg > 0)[0][0])
    for _ in range(args.reps + 1):
        _, plans = M.bfs(src, push_only=args.push_only)
    torch.cuda.synchronize()
    print(f"[prof] breadth-first search on R-MAT 2^20 from {src}: {M.bfs_levels} levels, "
          f"{sum(p.lanes == -1 for p in plans)} pull levels, {args.reps + 1} searches done", flush=True)


def cmd_pagerank(args):
    import torch
    from . import Matrix
    from . import synth
    A = synth.cfg2_matrix()
    M = Matrix.from_host(A)
    d = 0.85
    eps = 1e-3 * (1 - d) / A.n
    for _ in range(args.reps + 1):
        _, plans = M.pagerank(d, eps)
    torch.cuda.synchronize()
    print(f"[prof] incremental PageRank on R-MAT 2^20 (FP32): {M.pr_iters} products, "
          f"{args.reps + 1} runs done", flush=True)


def cmd_poisson(args):
    import numpy as np
    import torch
    from . import F32, F64, Matrix
    from . import synth
    dt = np.float64 if args.dtype == "f64" else np.float32
    A = synth.cfg3_matrix(dt, k=args.k)
    M = Matrix.from_host(A, dtype=F64 if args.dtype == "f64" else F32)
    x = torch.as_tensor(synth.dense_vector(A.n, 3).astype(dt), device="cuda")
    y = M.out_tensor()
    M.run(x, y)
    torch.cuda.synchronize()
    print(f"[prof] Poisson {args.k}^3 {args.dtype}: format {M.storage_format()[0]}, plan {M.last_plan()}",
          flush=True)
    for _ in range(args.reps):
        M.run(x, y)
    torch.cuda.synchronize()
    print(f"[prof] {args.reps} runs done", flush=True)


def cmd_copy(args):
    import torch
    n = args.mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"[prof] copied {args.mib} MiB {args.reps} times", flush=True)


def cmd_kernels(args):
    con = sqlite3.connect(_db(args.db))
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    con.close()
    scale = 1.0  # the top_kernels view reports microseconds
    print(f"# {args.title}\n")
    print(f"Command (run from the repository root on one MI355X):\n\n```\n{args.command}\n```\n")
    print("Durations in microseconds (rocprofv3 kernel trace, `top_kernels` view).\n")
    print("| kernel | calls | total us | avg us | % |")
    print("|---|---:|---:|---:|---:|")
    for n, c, t, a, p in rows[:args.top]:
        short = n.replace("spx::", "")
        i = short.find("(")
        short = short[:i] if i > 0 else short
        print(f"| `{short}` | {c} | {t * scale:.1f} | {a * scale:.3f} | {p:.1f} |")


def cmd_traffic(args):
    copy_bytes = args.mib * (1 << 20)
    cf = counter_per_dispatch(args.copy_fetch, "FETCH_SIZE")
    cw = counter_per_dispatch(args.copy_write, "WRITE_SIZE")
    # the copy is the largest dispatch of its run
    f_copy = max(v for _, _, v in cf) * 1024.0
    w_copy = max(v for _, _, v in cw) * 1024.0
    k_fetch = copy_bytes / f_copy
    k_write = copy_bytes / w_copy
    stems = args.kernels.split(",")
    fr = _mean_by_stem(counter_per_dispatch(args.fetch, "FETCH_SIZE"), stems)
    wr = _mean_by_stem(counter_per_dispatch(args.write, "WRITE_SIZE"), stems)
    fetch = sum((fr[s][0] or 0.0) for s in stems) * 1024.0 * k_fetch
    write = sum((wr[s][0] or 0.0) for s in stems) * 1024.0 * k_write
    rec = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            rec = json.load(f)
    key = args.workload or f"{SWEEP_WORKLOAD}:v{args.vector}"
    rec[key] = {
        "kernels": stems,
        "dispatches": {s: [fr[s][1], wr[s][1]] for s in stems},
        "fetch_bytes_per_launch": round(fetch),
        "write_bytes_per_launch": round(write),
        "bytes_per_launch": round(fetch + write),
        "calibration": {"copy_bytes": copy_bytes, "fetch_factor": round(k_fetch, 4),
                        "write_factor": round(k_write, 4)},
        "kernel_sources_sha256": kernel_source_hash(stems),
        "commands": args.command or [],
    }
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(rec[key]))


def traffic_for(path: str, vector: int):
    """Committed HBM bytes per launch of the sweep vector's kernels, or None
    if absent or taken on other sources of those kernels than the current
    ones."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(f"{SWEEP_WORKLOAD}:v{vector}")
    if not rec or rec.get("kernel_sources_sha256") != kernel_source_hash(rec["kernels"]):
        return None
    return rec["bytes_per_launch"]


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2006_16767_amd.prof")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("vector")
    a.add_argument("k", type=int)
    a.add_argument("--reps", type=int, default=5)
    a.add_argument("--plan", help="pattern,distribution[,writeback] instead of run()'s choice")
    a = sub.add_parser("batch")
    a.add_argument("--B", type=int, default=512)
    a.add_argument("--reps", type=int, default=5)
    a = sub.add_parser("fc")
    a.add_argument("--reps", type=int, default=5)
    a = sub.add_parser("bfs")
    a.add_argument("--reps", type=int, default=3)
    a.add_argument("--push-only", action="store_true")
    a = sub.add_parser("pagerank")
    a.add_argument("--reps", type=int, default=2)
    a = sub.add_parser("poisson")
    a.add_argument("--k", type=int, default=128)
    a.add_argument("--dtype", choices=("f32", "f64"), default="f32")
    a.add_argument("--reps", type=int, default=5)
    a = sub.add_parser("copy")
    a.add_argument("--mib", type=int, default=512)
    a.add_argument("--reps", type=int, default=3)
    a = sub.add_parser("kernels")
    a.add_argument("db")
    a.add_argument("--title", required=True)
    a.add_argument("--command", required=True)
    a.add_argument("--top", type=int, default=30)
    a = sub.add_parser("traffic")
    for n in ("fetch", "write", "copy_fetch", "copy_write", "out", "kernels"):
        a.add_argument("--" + n.replace("_", "-"), dest=n, required=True)
    a.add_argument("--mib", type=int, required=True)
    g = a.add_mutually_exclusive_group(required=True)
    g.add_argument("--vector", type=int)
    g.add_argument("--workload")
    a.add_argument("--command", action="append")
    args = ap.parse_args(argv)
    {"vector": cmd_vector, "batch": cmd_batch, "fc": cmd_fc, "bfs": cmd_bfs, "pagerank": cmd_pagerank,
     "poisson": cmd_poisson, "copy": cmd_copy, "kernels": cmd_kernels,
     "traffic": cmd_traffic}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
