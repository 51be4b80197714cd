"""MD-shaped sequence: learned charges + one mixed-precision density solve per step.

    python -m paper_2606_03140_amd.md_experiment [--waters 30000] [--steps 100]

30,000 rigid waters (seed 5; 90,000 atoms, 180,000 orbitals), non-orthogonal
model, kT 0.1 eV, 14x14x15 spatial cores.  Motion is prescribed: rigid
molecules in free flight with Maxwell centre-of-mass and angular velocities
at 300 K (seed 5005), 0.25 fs steps (there is no force model, so the
free-flight trajectory is exact).  Every step on the GPU:

  4 A neighbour graph -> descriptors -> BF16 charge network -> neutral q_guess
  -> screened Ewald potential V(q_guess) -> H[V], S -> mixed-precision solve
  (mu warm-started from the previous step) -> Mulliken charges q,

and every `--rebuild` steps the partition graph is rebuilt from the previous
step's density matrix, G_tau = (G^N G^D + G^D G^N)|_tau at tau 1e-3 (Dynamic
Graph Adaption).  The descriptor (5 A) and real-space Ewald pair lists are
rebuilt with the partition, with a skin, and filtered by distance inside the
kernels; the run checks that no atom moves more than half the skin within a
rebuild window.  Every `--fp64-every`
steps the FP64 path solves the same H, S on the same partition and the
charge difference is recorded.  The charge network is trained first on
displaced 3,000-water snapshots (SCC-converged labels).  Prints one JSON
line; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

import waterbox

from . import learned, pipeline, scc
from ._lib import Context, System, TBParams


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def train_model(ctx, n_snapshots: int, epochs: int, seed: int = 4):
    base = waterbox.water_box(3000, seed)
    tb = TBParams(orthogonal=False)
    species = torch.as_tensor(base.species.astype(np.int32)).to(ctx.dev)
    model = learned.ChargeModel(ctx, waterbox.mlp_init(seed))
    feats, labels, warm, mu = [], [], None, -7.0
    for j in range(n_snapshots):
        box = waterbox.displaced(base, 4000 + j)
        sysm = System(box.pos, box.species, box.anchor, box.box)
        part = pipeline.cutoff_partition(ctx, sysm, tb, (5, 5, 6))
        r = scc.scc_loop(ctx, sysm, tb, part, 0.1, pipeline.MIXED_F16, q_start=warm, mu_guess=mu)
        if not r.converged:
            raise RuntimeError(f"label snapshot {j}: SCC did not converge")
        warm, mu = r.q, r.mu
        labels.append(r.q.clone())
        feats.append(model.descriptors(sysm))
        if j % 5 == 0:
            _log(f"[train] labels {j + 1}/{n_snapshots}: {r.iterations} SCC iterations")
    model.fit_norm(feats, species)
    hist = model.train(feats, species, labels, epochs=epochs, lr=1e-3, seed=seed)
    _log(f"[train] loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    return model, hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--waters", type=int, default=30000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--grid", type=int, nargs=3, default=(14, 14, 15))
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--dt", type=float, default=0.25)
    ap.add_argument("--rebuild", type=int, default=10)
    ap.add_argument("--fp64-every", type=int, default=10)
    ap.add_argument("--tau", type=float, default=1e-3)
    ap.add_argument("--train-snapshots", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--ewald-rcut", type=float, default=16.0)
    ap.add_argument("--skin", type=float, default=1.0)
    args = ap.parse_args(argv)
    kT = 0.1
    ctx = Context(0)
    t_all = time.time()
    model, train_hist = train_model(ctx, args.train_snapshots, args.epochs)

    _log(f"[md] {args.waters} waters, trajectory of {args.steps} steps")
    base = waterbox.water_box(args.waters, args.seed)
    frames = waterbox.rigid_trajectory(base, args.steps, args.dt, seed=5005, temperature=300.0)
    L = base.box[0]
    max_disp = 0.0                     # largest move within one rebuild window
    for t0w in range(0, args.steps, args.rebuild):
        d = frames[min(t0w + args.rebuild - 1, args.steps)] - frames[t0w]
        d -= L * np.rint(d / L)
        max_disp = max(max_disp, float(np.sqrt((d ** 2).sum(1)).max()))
    if max_disp > 0.5 * args.skin:
        raise RuntimeError(f"atoms move {max_disp:.3f} A within a rebuild window, more than half the "
                           f"{args.skin} A skin")
    tb = TBParams(orthogonal=False)
    system = System(frames[0], base.species, base.anchor, base.box)
    species = system.species
    # pair lists with a skin, rebuilt with the partition (valid within a window)
    lists = {}

    def build_lists():
        lists["desc"] = ctx.build_graph_cutoff(system, learned.DESCRIPTOR_CUTOFF + args.skin)
        lists["ewald"] = scc.ewald_setup(ctx, system, rcut_max=args.ewald_rcut, skin=args.skin)

    build_lists()
    ew = lists["ewald"]
    tau_s = scc.slater_tau(scc.HUBBARD_U)
    _log(f"[md] Ewald rcut {ew.rcut:.1f} A, eta {ew.eta:.3f}, k_max {ew.k_max}, {ew.graph.nnz} real-space pairs")

    def guess_potential():
        ew = lists["ewald"]
        feats = ctx.descriptors(system, lists["desc"])
        q_guess = model.predict(feats, species, bf16=True)
        V = ctx.ewald_potential(system, ew.graph, ew.rcut, ew.eta, ew.k_max, scc.HUBBARD_U, q_guess, tau=tau_s)
        return q_guess, V

    # initial partition: neighbour-graph halos, one solve, then G_tau from its D
    part = pipeline.cutoff_partition(ctx, system, tb, args.grid)
    q_guess, V = guess_potential()
    H, S = ctx.build_hs(system, tb, part.nbr, V)
    sol = pipeline.solve(ctx, system, part, H, S, kT, pipeline.MIXED_F16, mu_guess=-7.0)
    part = pipeline.rebuild_adaptive(ctx, system, tb, part, sol.D_core, args.tau)
    ctx.plan(part.sg, pipeline.MIXED_F16)
    mu = sol.mu
    _log(f"[md] partition: {part.sg.n_sub} subgraphs, n {part.sg.norb.min()}-{part.sg.norb.max()} "
         f"(median {int(np.median(part.sg.norb))})")

    names = ("graph", "guess", "hs", "solve", "rebuild")
    acc = {k: 0.0 for k in names}
    step_ms, drift, resid, sizes, gemm = [], [], [], [], []
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in names}
    sol = None
    for t in range(args.steps + 1):
        system.set_positions(frames[t])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev["graph"][0].record()
        nbr = ctx.build_graph_cutoff(system, tb.cutoff)
        part.nbr = nbr
        ev["graph"][1].record()
        ev["rebuild"][0].record()
        if t > 0 and t % args.rebuild == 0:
            part = pipeline.rebuild_adaptive(ctx, system, tb, part, sol.D_core, args.tau, nbr=nbr)
            ctx.plan(part.sg, pipeline.MIXED_F16)
            build_lists()
        ev["rebuild"][1].record()
        ev["guess"][0].record()
        q_guess, V = guess_potential()
        ev["guess"][1].record()
        ev["hs"][0].record()
        H, S = ctx.build_hs(system, tb, nbr, V)
        ev["hs"][1].record()
        ev["solve"][0].record()
        sol = pipeline.solve(ctx, system, part, H, S, kT, pipeline.MIXED_F16, mu_guess=mu, plan=False)
        ev["solve"][1].record()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        mu = sol.mu
        if t > 0:                      # step 0 carries the one-off warm-up
            step_ms.append(ms)
            for k in names:
                acc[k] += ev[k][0].elapsed_time(ev[k][1])
            st = ctx.mixed_stats()
            gemm.append(st)
        resid.append(float(torch.sqrt(torch.mean((sol.q - q_guess) ** 2))))
        if t % args.fp64_every == 0:
            ref = pipeline.solve(ctx, system, part, H, S, kT, pipeline.FP64_EIG)
            ctx.plan(part.sg, pipeline.MIXED_F16)
            dq = float((sol.q - ref.q).abs().max())
            dD = float((sol.D_core - ref.D_core).abs().max())
            drift.append({"step": t, "max_abs_dq_e": dq, "max_abs_dD": dD, "mu_mixed": sol.mu, "mu_fp64": ref.mu})
            _log(f"[md] step {t}: {ms:.1f} ms, mu {sol.mu:.4f} (FP64 {ref.mu:.4f}), max|dq| {dq:.2e} e, "
                 f"max|dD| {dD:.2e}, RMS(q - q_guess) {resid[-1]:.3e} e")
        sizes.append(int(part.sg.n_sub))
    n_st = len(step_ms)
    flops = sum(g["flops_per_launch"] * 3 * g["gemm_launches"] for g in gemm)
    byts = sum(g["bytes_per_launch"] * g["gemm_launches"] for g in gemm)
    out = {
        "metric": "MD-shaped step time (learned charge guess + mixed-precision density solve + charges)",
        "workload": f"{args.waters} waters, {3 * args.waters} atoms, {system.n_orb} orbitals, cores "
                    f"{args.grid[0]}x{args.grid[1]}x{args.grid[2]}, tau {args.tau}, rebuild every {args.rebuild} "
                    f"steps, {args.steps} steps of {args.dt} fs",
        "ms_per_step_mean": float(np.mean(step_ms)), "ms_per_step_median": float(np.median(step_ms)),
        "ms_per_step_components": {k: acc[k] / n_st for k in names},
        "subgraphs": {"min": int(min(sizes)), "max": int(max(sizes))},
        "split_gemm_per_step": {"tflops_executed": flops / n_st / (acc["solve"] / n_st * 1e-3) / 1e12,
                                "note": "executed FP16 MFMA flops of the split GEMMs per step / solve time"},
        "split_gemm_bytes_per_step_GB": byts / n_st / 1e9,
        "charge_drift_vs_fp64": drift,
        "max_abs_dq_vs_fp64_e": max(d["max_abs_dq_e"] for d in drift),
        "rms_q_minus_guess_e": {"mean": float(np.mean(resid)), "max": float(np.max(resid))},
        "max_displacement_A": max_disp,
        "train": {"snapshots": args.train_snapshots, "epochs": args.epochs,
                  "loss_first_last": [train_hist[0], train_hist[-1]]},
        "seconds_total": time.time() - t_all,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
