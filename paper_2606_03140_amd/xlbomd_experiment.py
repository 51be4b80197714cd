"""XL-BOMD on a water box: shadow molecular dynamics with graph-partitioned
density matrices (Shadow MD section; Dynamic Graph Adaption section).

    python -m paper_2606_03140_amd.xlbomd_experiment [--waters 3000] [--grid 5 5 6]
        [--steps 40] [--dt 0.25 0.5] [--graph cutoff|adaptive] [--rebuild 10]

A seeded water box with the tapered synthetic model and its repulsive pair
term, one spatial core per grid cell, Maxwell velocities at 300 K (seed
5005), the extended charges started at the SCC ground state (Anderson,
FP64 path) and driven by the low-rank Krylov kernel (or c I).  For each
time step in --dt the run integrates --steps steps (scaled so that every
run covers the same simulated time) and reports the
total free energy's fluctuation and drift, RMS(q[n] - n), the subgraph sizes
and the wall time of each stage of a step.  Prints one JSON line; progress
goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

import waterbox

from . import xlbomd
from ._lib import Context, System


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_one(ctx, box, grid, dt, steps, graph, rebuild, tau, n0, vel, c, kernel, max_rank, rank_tol, response):
    system = System(box.pos, box.species, box.anchor, box.box)
    tb = xlbomd.md_params()
    core, nco = ctx.grid_cores(system, grid)
    md = xlbomd.XLBOMD(ctx, system, tb, core, nco, dt=dt, c=c, graph=graph, tau=tau, rebuild=rebuild, timing=True,
                       kernel=kernel, max_rank=max_rank, rank_tol=rank_tol, response=response)
    md.start(n0, vel)
    md.timing.clear()
    t0 = time.perf_counter()
    for k in range(steps):
        md.step()
        if (k + 1) % 10 == 0:
            e = md.rec.e_tot
            _log(f"[xlbomd] dt {dt}: step {k + 1}/{steps}, E - E0 {e[-1] - e[0]:+.3e} eV, "
                 f"rms(q - n) {md.rec.rms_qn[-1]:.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e = np.array(md.rec.e_tot)
    n_atoms = system.n_atoms
    sizes = np.concatenate(md.rec.sizes)
    return {
        "dt_fs": dt, "steps": steps, "ms_per_step": 1e3 * wall / steps,
        "stage_ms_per_step": {k: round(1e3 * v / steps, 3) for k, v in md.timing.items()},
        "e_fluct_ev": float(e.max() - e.min()), "e_fluct_ev_per_atom": float((e.max() - e.min()) / n_atoms),
        "e_drift_ev": float(e[-1] - e[0]),
        "e_kin_ev": [float(md.rec.e_kin[0]), float(md.rec.e_kin[-1])],
        "rms_q_minus_n_max": float(max(md.rec.rms_qn)),
        "subgraph_orbitals": [int(sizes.min()), int(np.median(sizes)), int(sizes.max())],
        "n_subgraphs": int(nco),
        "kernel_rank_mean": float(np.mean(md.ranks)) if md.ranks else None,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--waters", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--grid", type=int, nargs=3, default=(5, 5, 6))
    ap.add_argument("--steps", type=int, default=16, help="steps at the largest dt")
    ap.add_argument("--dt", type=float, nargs="+", default=(0.5, 0.25))
    ap.add_argument("--graph", default="cutoff", choices=("cutoff", "adaptive"))
    ap.add_argument("--rebuild", type=int, default=10)
    ap.add_argument("--tau", type=float, default=1e-5)
    ap.add_argument("--c", type=float, default=0.3)
    ap.add_argument("--kernel", default="krylov", choices=("scaled", "krylov"))
    ap.add_argument("--max-rank", type=int, default=6)
    ap.add_argument("--rank-tol", type=float, default=0.1)
    ap.add_argument("--response", default="mixed", choices=("mixed", "fd"))
    ap.add_argument("--temperature", type=float, default=300.0)
    ap.add_argument("--scc-tol", type=float, default=1e-7)
    ap.add_argument("--scc", default="anderson", choices=("anderson", "quasi_newton"))
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    ctx = Context(0)
    box = waterbox.water_box(args.waters, args.seed)
    system = System(box.pos, box.species, box.anchor, box.box)
    tb = xlbomd.md_params()
    core, nco = ctx.grid_cores(system, tuple(args.grid))
    t0 = time.perf_counter()
    def scc_log(it, rms, rank, rel, alpha, mu):
        _log(f"[xlbomd] SCC start {it}: rms {rms:.2e}, rank {rank}, fit {rel:.2e}, step {alpha}")

    n0 = xlbomd.converged_charges(ctx, system, tb, core, nco, tol=args.scc_tol, mixer=args.scc,
                                  max_iter=200 if args.scc == "anderson" else 60, log=scc_log)
    t_scc = time.perf_counter() - t0
    _log(f"[xlbomd] {args.waters} waters, {nco} cores: SCC start in {t_scc:.1f} s")
    vel = xlbomd.maxwell_velocities(box.species, args.temperature, 5005)
    dts = sorted(args.dt, reverse=True)
    runs = []
    for dt in dts:
        steps = int(round(args.steps * dts[0] / dt))
        runs.append(run_one(ctx, box, tuple(args.grid), dt, steps, args.graph, args.rebuild, args.tau, n0, vel,
                            args.c, args.kernel, args.max_rank, args.rank_tol, args.response))
        _log(f"[xlbomd] dt {dt}: {json.dumps(runs[-1])}")
    ratios = [runs[i]["e_fluct_ev"] / runs[i + 1]["e_fluct_ev"] for i in range(len(runs) - 1)]
    out = {"experiment": "xlbomd", "waters": args.waters, "atoms": system.n_atoms, "grid": list(args.grid),
           "graph": args.graph, "rebuild": args.rebuild, "tau": args.tau, "kernel": args.kernel,
           "kernel_c": args.c, "max_rank": args.max_rank, "rank_tol": args.rank_tol, "response": args.response,
           "scc_start_s": t_scc, "scc_tol": args.scc_tol, "scc": args.scc, "runs": runs, "fluct_ratio_per_dt_doubling": ratios}
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    ctx.close()


if __name__ == "__main__":
    main()
