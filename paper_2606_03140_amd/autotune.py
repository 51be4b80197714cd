"""Autotuner for the run-time options of both solver paths.

For a workload (a partition with its H and S) it times every candidate
setting of the options that change speed but not the method:

* FP64 path: the largest leaf of the tridiagonal divide and conquer
  (gdm_set_fp64_options; results agree to FP64 rounding for every value);
* mixed paths: upper-tile or whole storage of the expansion's symmetric
  matrices (gdm_set_mixed_storage), the degree of the minimax start of each
  doubling's inverse (gdm_set_mixed_inverse_start) and the Newton-Schulz
  iterations after it (gdm_set_mixed_options).  These change
  the rounding, so a candidate is kept only when its density and charges
  stay within `tol` of the FP64 path's on the same workload.

The fastest admissible candidate of each path is stored in a JSON table
keyed by a size bucket (the largest subgraph, rounded up to a power of two
from 256), and `apply_table` sets the table's choice for a subgraph set
before its gdm_plan.  Run on the GPU as

    python -m paper_2606_03140_amd.autotune --out paper_2606_03140_amd/tuning.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PATHS = ("fp64", "mixed", "mixed_bf16")
CANDIDATES = {
    "fp64": [{"leaf_rows": v} for v in (16, 24, 32, 48, 64)],
    "mixed": [{"upper_tiles": u, "inv_start": d, "ns_inv": k} for u in (1, 0) for d, k in ((4, 1), (2, 2), (4, 2))],
    "mixed_bf16": [{"upper_tiles": u, "inv_start": d, "ns_inv": k}
                   for u in (1, 0) for d, k in ((4, 1), (2, 2), (4, 2))],
}
DEFAULTS = {"fp64": {"leaf_rows": 64}, "mixed": {"upper_tiles": 1, "inv_start": 4, "ns_inv": 1},
            "mixed_bf16": {"upper_tiles": 1, "inv_start": 4, "ns_inv": 1}}
TABLE_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def bucket(max_n: int) -> str:
    """Size bucket of a subgraph set: its largest subgraph rounded up to a
    power of two, at least 256."""
    b = 256
    while b < max_n:
        b *= 2
    return f"n<={b}"


def pick(results: list[dict]) -> dict | None:
    """Fastest admissible candidate (ties: the earlier one)."""
    best = None
    for r in results:
        if r.get("ok", True) and (best is None or r["ms"] < best["ms"]):
            best = r
    return best


def apply(ctx, path: str, opts: dict) -> None:
    if path == "fp64":
        ctx.set_fp64_options(int(opts.get("leaf_rows", 64)))
    else:
        # a table entry without "inv_start" was tuned with the quadratic start
        ctx.set_mixed_storage(bool(opts.get("upper_tiles", 1)))
        ctx.set_mixed_inverse_start(int(opts.get("inv_start", 2)))
        ctx.set_mixed_options(ns_inv=int(opts.get("ns_inv", 2)))


def apply_table(ctx, table: dict, max_n: int, paths=PATHS) -> dict:
    """Set the tuned options of every path for a subgraph set whose largest
    subgraph has max_n orbitals (library defaults where the table has no
    entry); returns the options set."""
    entry = table.get(bucket(max_n), {})
    used = {}
    for p in paths:
        opts = entry.get(p, {}).get("choice", DEFAULTS[p])
        apply(ctx, p, opts)
        used[p] = opts
    return used


def load_table(path: str = TABLE_FILE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_table(table: dict, path: str = TABLE_FILE) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")


def _time(ctx, system, part, H, S, kT, precision, steps, warmup, mu_guess):
    import torch
    from . import pipeline
    ctx.plan(part.sg, precision)
    sol = None
    for _ in range(warmup):
        sol = pipeline.solve(ctx, system, part, H, S, kT, precision, mu_guess=mu_guess, plan=False)
        mu_guess = sol.mu
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sol = pipeline.solve(ctx, system, part, H, S, kT, precision, mu_guess=mu_guess, plan=False)
        mu_guess = sol.mu
    torch.cuda.synchronize()
    return sol, (time.perf_counter() - t0) * 1e3 / steps


def tune(ctx, system, part, H, S, kT: float, paths=PATHS, steps: int = 3, warmup: int = 1,
         tol: float = 1e-4, tol_bf16: float = 1e-3, log=None) -> dict:
    """Time every candidate of each path on this workload; returns
    {path: {"choice": opts, "ms": t, "candidates": [...]}}."""
    from . import pipeline
    precs = {"fp64": pipeline.FP64_EIG, "mixed": pipeline.MIXED_F16, "mixed_bf16": pipeline.MIXED_BF16}
    apply(ctx, "fp64", DEFAULTS["fp64"])
    ref, _ = _time(ctx, system, part, H, S, kT, pipeline.FP64_EIG, 1, 0, 0.0)
    q_ref = ref.q.cpu().numpy()
    out = {}
    try:
        for p in paths:
            res = []
            for opts in CANDIDATES[p]:
                apply(ctx, p, opts)
                sol, ms = _time(ctx, system, part, H, S, kT, precs[p], steps, warmup, ref.mu)
                r = {"opts": opts, "ms": ms}
                if p != "fp64":
                    t = tol_bf16 if p == "mixed_bf16" else tol
                    r["max_abs_dD"] = (sol.D_core - ref.D_core).abs().max().item()
                    r["max_abs_dq"] = float(np.abs(sol.q.cpu().numpy() - q_ref).max())
                    r["ok"] = r["max_abs_dD"] <= t and r["max_abs_dq"] <= t
                if log:
                    log(f"[autotune] {p} {opts}: {ms:.2f} ms" +
                        (f", dD {r['max_abs_dD']:.1e} dq {r['max_abs_dq']:.1e}" if p != "fp64" else ""))
                res.append(r)
            best = pick(res)
            out[p] = {"choice": best["opts"] if best else DEFAULTS[p], "ms": best["ms"] if best else None,
                      "candidates": res}
    finally:
        for p in paths:
            apply(ctx, p, DEFAULTS[p])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_FILE)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--workloads", default="water10000,water3000")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import waterbox
    from . import pipeline
    from ._lib import Context, System, TBParams

    def log(m):
        print(m, file=sys.stderr, flush=True)

    table = load_table(args.out)
    ctx = Context(0)
    for name in args.workloads.split(","):
        if name == "water10000":
            nw, seed, grid, tau, mode = 10000, 3, (10, 10, 10), 1e-3, pipeline.GRAPH_DM
        elif name == "water3000":
            nw, seed, grid, tau, mode = 3000, 7, (5, 5, 6), 1e-5, pipeline.GRAPH_ADAPTIVE
        else:
            raise SystemExit(f"unknown workload {name}")
        box = waterbox.water_box(nw, seed)
        system = System(box.pos, box.species, box.anchor, box.box)
        tb = TBParams(orthogonal=False)
        part = pipeline.cutoff_partition(ctx, system, tb, grid)
        H, S = ctx.build_hs(system, tb, part.nbr)
        sol = pipeline.solve(ctx, system, part, H, S, 0.1, pipeline.FP64_EIG)
        if mode == pipeline.GRAPH_DM:
            g = ctx.build_graph_dm(system, mode, part.sg, sol.D_core, tau, union=part.graph)
        else:
            g = ctx.build_graph_dm(system, mode, part.sg, sol.D_core, tau, alpha=0.7, nbr=part.nbr)
        part = pipeline.repartition(ctx, system, tb, part, g)
        max_n = int(part.sg.norb.max())
        log(f"[autotune] {name}: {part.sg.n_sub} subgraphs, n up to {max_n} -> bucket {bucket(max_n)}")
        paths = PATHS if name == "water10000" else ("fp64",)
        res = tune(ctx, system, part, H, S, 0.1, paths=paths, steps=args.steps, log=log)
        entry = table.setdefault(bucket(max_n), {})
        for p, r in res.items():
            entry[p] = {"choice": r["choice"], "ms": r["ms"], "workload": name,
                        "candidates": [{k: v for k, v in c.items()} for c in r["candidates"]]}
    ctx.close()
    save_table(table, args.out)
    log(f"[autotune] table written to {args.out}")


if __name__ == "__main__":
    main()
