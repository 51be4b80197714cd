"""SCC iterations saved by the learned starting charges.

    python -m paper_2606_03140_amd.scc_experiment [--train 200] [--test 20]

Base box: 3,000 rigid waters (seed 4), non-orthogonal model, kT 0.1 eV,
5x5x6 spatial cores with one-hop halos over the 4 A neighbour graph.
Snapshots carry N(0, 0.05^2) A displacements per Cartesian component
(seeds 4000 + j; j < 200 train, 200..219 held out).  Labels are the
SCC-converged Mulliken charges (residual RMS < 1e-5 e, Anderson mixing
with memory 8 and mixing 0.03, screened Coulomb) of the mixed-precision
solver; training and inference run the libgdm MLP kernels.  For every
held-out snapshot the SCC loop runs from zero charges and from the BF16
network prediction with the same mixer and solver, and the kernel-
accelerated quasi-Newton SCF (low-rank Krylov kernel from charge responses
of the mixed-precision solver, K0 = -0.1 I, relative fit tolerance 1e-2,
rank <= 8, unfitted remainder added, backtracking line search) runs from
both starts as well; iterations, density solves, response solves and wall
time are reported for each.  Prints one JSON line; progress goes to stderr.
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--waters", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--grid", type=int, nargs=3, default=(5, 5, 6))
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--test", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--precision", choices=("mixed", "fp64"), default="mixed")
    ap.add_argument("--no-quasi-newton", dest="quasi_newton", action="store_false")
    args = ap.parse_args(argv)
    prec = pipeline.MIXED_F16 if args.precision == "mixed" else pipeline.FP64_EIG
    kT = 0.1
    ctx = Context(0)
    base = waterbox.water_box(args.waters, args.seed)
    tb = TBParams(orthogonal=False)
    species = torch.as_tensor(base.species.astype(np.int32)).to(ctx.dev)
    model = learned.ChargeModel(ctx, waterbox.mlp_init(args.seed))

    def setup(box):
        sysm = System(box.pos, box.species, box.anchor, box.box)
        part = pipeline.cutoff_partition(ctx, sysm, tb, args.grid)
        return sysm, part, scc.ewald_setup(ctx, sysm)

    t0 = time.time()
    feats, labels, warm, mu = [], [], None, -7.0
    label_iters = []
    for j in range(args.train):
        sysm, part, ew = setup(waterbox.displaced(base, 4000 + j))
        r = scc.scc_loop(ctx, sysm, tb, part, kT, prec, q_start=warm, ewald=ew, mu_guess=mu)
        if not r.converged:
            raise RuntimeError(f"training snapshot {j}: SCC did not converge in {r.iterations} iterations")
        warm, mu = r.q, r.mu
        labels.append(r.q.clone())
        feats.append(model.descriptors(sysm))
        label_iters.append(r.iterations)
        if j % 10 == 0 or j == args.train - 1:
            _log(f"[labels] snapshot {j}: {r.iterations} SCC iterations, {time.time() - t0:.0f} s")
    t_labels = time.time() - t0
    model.fit_norm(feats, species)
    t1 = time.time()
    hist = model.train(feats, species, labels, epochs=args.epochs, lr=args.lr, seed=args.seed,
                       log=lambda ep, l: _log(f"[train] epoch {ep}: loss {l:.3e}") if ep % 50 == 0 else None)
    torch.cuda.synchronize()
    t_train = time.time() - t1

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    rows = []
    for j in range(args.train, args.train + args.test):
        sysm, part, ew = setup(waterbox.displaced(base, 4000 + j))
        r0, t0s = timed(lambda: scc.scc_loop(ctx, sysm, tb, part, kT, prec, ewald=ew, mu_guess=mu))
        guess = model.predict(model.descriptors(sysm), species, bf16=True)
        r1, t1s = timed(lambda: scc.scc_loop(ctx, sysm, tb, part, kT, prec, q_start=guess, ewald=ew, mu_guess=mu))
        row = {"snapshot": 4000 + j, "zero_start": r0.iterations, "mlp_start": r1.iterations,
               "converged": bool(r0.converged and r1.converged),
               "seconds_zero_start": t0s, "seconds_mlp_start": t1s,
               "guess_rms_error_e": float(torch.sqrt(torch.mean((guess - r0.q) ** 2))),
               "zero_rms_error_e": float(torch.sqrt(torch.mean(r0.q ** 2))),
               "max_abs_dq_between_starts_e": float((r0.q - r1.q).abs().max())}
        if args.quasi_newton and prec == pipeline.MIXED_F16:
            n0, tq0 = timed(lambda: scc.scc_quasi_newton(ctx, sysm, tb, part, kT, ewald=ew, mu_guess=mu))
            n1, tq1 = timed(lambda: scc.scc_quasi_newton(ctx, sysm, tb, part, kT, q_start=guess, ewald=ew,
                                                         mu_guess=mu))
            row.update({"qn_zero_start": n0.iterations, "qn_mlp_start": n1.iterations,
                        "qn_responses_zero_start": n0.responses, "qn_responses_mlp_start": n1.responses,
                        "qn_solves_zero_start": n0.solves, "qn_solves_mlp_start": n1.solves,
                        "qn_seconds_zero_start": tq0, "qn_seconds_mlp_start": tq1,
                        "qn_converged": bool(n0.converged and n1.converged),
                        "qn_max_abs_dq_vs_anderson_e": float(max((n0.q - r0.q).abs().max(),
                                                                 (n1.q - r0.q).abs().max()))})
        rows.append(row)
        _log(f"[test] {row}")
    z = np.array([r["zero_start"] for r in rows])
    m = np.array([r["mlp_start"] for r in rows])
    out = {
        "metric": "SCC iterations to 1e-5 e RMS residual, learned start vs zero start",
        "workload": f"{args.waters} waters, {3 * args.waters} atoms, displaced snapshots sigma 0.05 A, "
                    f"cores {args.grid[0]}x{args.grid[1]}x{args.grid[2]}, kT {kT} eV, solver {args.precision}",
        "train_snapshots": args.train, "test_snapshots": args.test, "epochs": args.epochs,
        "mean_iterations_zero_start": float(z.mean()), "mean_iterations_mlp_start": float(m.mean()),
        "mean_iterations_saved": float((z - m).mean()), "all_converged": all(r["converged"] for r in rows),
        "mean_guess_rms_error_e": float(np.mean([r["guess_rms_error_e"] for r in rows])),
        "max_abs_dq_between_starts_e": float(max(r["max_abs_dq_between_starts_e"] for r in rows)),
        "mean_seconds_zero_start": float(np.mean([r["seconds_zero_start"] for r in rows])),
        "mean_seconds_mlp_start": float(np.mean([r["seconds_mlp_start"] for r in rows])),
        "training_loss_first_last": [hist[0], hist[-1]],
        "label_iterations_mean": float(np.mean(label_iters)),
        "seconds": {"labels": t_labels, "train": t_train},
        "per_snapshot": rows,
    }
    if rows and "qn_zero_start" in rows[0]:
        for k in ("qn_zero_start", "qn_mlp_start", "qn_responses_zero_start", "qn_responses_mlp_start",
                  "qn_solves_zero_start", "qn_solves_mlp_start", "qn_seconds_zero_start", "qn_seconds_mlp_start"):
            out["mean_" + k] = float(np.mean([r[k] for r in rows]))
        out["qn_all_converged"] = all(r["qn_converged"] for r in rows)
        out["qn_max_abs_dq_vs_anderson_e"] = float(max(r["qn_max_abs_dq_vs_anderson_e"] for r in rows))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
