"""Benchmark: subgraph density-matrix solves/s on one MI355X.

Workload: 10,000 rigid waters (30,000 atoms, 60,000 orbitals) of the seeded
synthetic water box, non-orthogonal TB model, kT = 0.1 eV, 10x10x10 spatial
cores, halos from the adaptive density-matrix graph at tau = 1e-3.  A step is
one pass of the whole density solve on all subgraphs: gather of h, s ->
per-subgraph solve -> global mu -> collected core rows of D -> Mulliken
charges (find_mu + subgraph_density + mulliken_charges).  Inputs are resident
in HBM before the timed region.  Both solver paths are timed; the headline
value is the mixed-precision path when it is built, else the FP64 path.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(name="water10000", n_waters=10000, seed=3, grid=(10, 10, 10), tau=1e-3, kT=0.1, rounds=2)
PEAK = {"fp64": 78.6e12, "fp16_mfma": 2.5e15, "hbm": 8.0e12}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def dc_block_sum(n: int, leaf: int = 64) -> int:
    """sum of k^2 over the blocks of every level of the divide-and-conquer
    tree of an n x n tridiagonal (balanced cuts, leaves of at most 64 rows)."""
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    tot = 0
    for lev in range(L + 1):
        b = [(i * n) >> lev for i in range((1 << lev) + 1)]
        tot += sum((b[i + 1] - b[i]) ** 2 for i in range(1 << lev))
    return tot


def fp64_flops(n: np.ndarray, nc: np.ndarray, leaf: int = 64) -> dict:
    """Nominal FP64 flops of the executed route, summed over subgraphs:
    Cholesky n^3/3, each triangular solve n^3, tridiagonalisation 4/3 n^3,
    reflectors and forward substitution on the 2 nc core rows 5 nc n^2, the
    divide-and-conquer products 2 R sum k^2 (R = 2 nc forward, nc reverse),
    reverse reflectors and the solve with L 3 nc n^2."""
    n = n.astype(np.float64)
    nc = nc.astype(np.float64)
    ks = np.array([dc_block_sum(int(v), leaf) for v in n], dtype=np.float64)
    return {
        "potrf": float(np.sum(n ** 3 / 3)),
        "trsm": float(np.sum(n ** 3)),          # per launch (two launches)
        "sytrd": float(np.sum(4.0 * n ** 3 / 3)),
        "core_rows": float(np.sum(5 * nc * n * n)),
        "dc_apply": float(np.sum(2 * 2 * nc * ks)),
        "dc_apply_rev": float(np.sum(2 * nc * ks)),
        "dcore": float(np.sum(3 * nc * n * n)),
    }


def time_path(ctx, system, part, H, S, kT, precision, steps, warmup, mu_guess=0.0):
    import torch
    from paper_2606_03140_amd import pipeline
    ctx.plan(part.sg, precision)
    stream = torch.cuda.current_stream()
    sol = None
    for _ in range(warmup):
        sol = pipeline.solve(ctx, system, part, H, S, kT, precision, mu_guess=mu_guess, plan=False)
        mu_guess = sol.mu
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    w0 = time.perf_counter()
    for _ in range(steps):
        sol = pipeline.solve(ctx, system, part, H, S, kT, precision, mu_guess=mu_guess, plan=False)
        mu_guess = sol.mu
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = t0.elapsed_time(t1) / steps
    prof = {}
    for name in ("gather", "potrf", "trsm", "symmetrize", "sytrd", "dc_leaf", "dc_merge", "core_rows", "dc_apply",
                 "core_weights", "dc_apply_rev", "dcore", "mu",
                 "mulliken", "foe_gemm", "ns_gemm", "mixed_misc", "refine64", "last64", "traces"):
        tot, n = ctx.profile_query(name)
        if n:
            prof[name] = {"ms_total": tot, "launches": n, "ms_per_step": tot / steps}
    ctx.profile(False)
    return sol, ms, wall / steps, prof


def time_response(ctx, system, part, H, S, kT, steps, warmup, mu_guess):
    """Charge response on the mixed path (the directional derivative of the
    kernel-accelerated SCF): one recorded solve, then `steps` responses to a
    seeded potential change, timed with HIP events on the library's stream."""
    import torch
    from paper_2606_03140_amd import pipeline
    ctx.set_response(16)
    try:
        ctx.plan(part.sg, pipeline.MIXED_F16)
        pipeline.solve(ctx, system, part, H, S, kT, pipeline.MIXED_F16, mu_guess=mu_guess, plan=False)
        g = torch.Generator(device="cpu").manual_seed(7)
        dV = (0.1 * torch.randn(system.n_atoms, generator=g, dtype=torch.float64)).to(ctx.dev)
        dq = torch.empty_like(dV)
        for _ in range(warmup):
            ctx.density_response(system, part.sg, part.nbr, S, dV, out=dq)
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            ctx.density_response(system, part.sg, part.nbr, S, dV, out=dq)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        tot, n = ctx.profile_query("response")
        ctx.profile(False)
        return {"ms_per_response": ms, "kernel_launches_per_response": n / steps,
                "max_abs_dq_e": float(dq.abs().max()),
                "note": "canonical charge response to a seeded 0.1 eV potential change: derivative of the recorded "
                        "expansion (3 split GEMMs per doubling + 2 for the perturbation), FP64 core rows, "
                        "Mulliken"}
    finally:
        ctx.set_response(0)


def time_cold(ctx, system, part, H, S, kT, mu_guess):
    """One mixed step whose chemical-potential search starts from a cold guess
    (the middle of the spectral bounds when mu_guess lies outside them)."""
    import torch
    from paper_2606_03140_amd import pipeline
    ctx.plan(part.sg, pipeline.MIXED_F16)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    sol = pipeline.solve(ctx, system, part, H, S, kT, pipeline.MIXED_F16, mu_guess=mu_guess, plan=False)
    t1.record(stream)
    torch.cuda.synchronize()
    st = ctx.mixed_stats()
    return {"ms": t0.elapsed_time(t1), "passes": st["passes"], "mu_guess": mu_guess, "mu": sol.mu,
            "note": "mixed step from a cold chemical-potential guess (one full expansion per pass)"}


def time_graph(system, part, H, S, kT, steps, warmup, mu_start):
    """The whole mixed step with the device-side chemical-potential search
    (gather, inverse overlap, expansion passes, mu, density at the device mu,
    charges) captured once into a hipGraph and replayed; each replay starts
    from the mu the previous one found (as an MD step would)."""
    import torch
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import Context
    from paper_2606_03140_amd.hipgraph import StreamGraph
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = Context(0)
        try:
            from paper_2606_03140_amd import autotune
            autotune.apply_table(c, autotune.load_table(), int(part.sg.norb.max()), paths=("mixed",))
            c.plan(part.sg, pipeline.MIXED_F16)
            c.set_mu_outputs(True)
            c.set_mixed_capture(3, 10)
            mu_t = torch.full((1,), mu_start, dtype=torch.float64, device=c.dev)
            n_t = torch.zeros_like(mu_t)
            D = torch.empty(int(part.sg.dcore_off[-1]), dtype=torch.float64, device=c.dev)
            q = torch.empty(system.n_atoms, dtype=torch.float64, device=c.dev)

            def step():
                c.find_mu_device(system, part.sg, part.nbr, H, S, kT, pipeline.MIXED_F16, mu_t, n_t,
                                 mu_guess=mu_start, tol_N=1e-6)
                c.subgraph_density_dmu(part.sg, mu_t, kT, pipeline.MIXED_F16, D)
                c.mulliken_charges(system, part.sg, part.nbr, S, D, out=q)

            step()
            c.check()
            g = StreamGraph(side)
            g.capture(step)
            try:
                for _ in range(warmup):
                    g.replay()
                g.synchronize()
                t0 = torch.cuda.Event(enable_timing=True)
                t1 = torch.cuda.Event(enable_timing=True)
                t0.record(side)
                for _ in range(steps):
                    g.replay()
                t1.record(side)
                g.synchronize()
                c.check()
                ms = t0.elapsed_time(t1) / steps
            finally:
                g.close()
            st = c.mixed_stats()
            return {"ms_per_step": ms, "solves_per_s": part.sg.n_sub / (ms * 1e-3), "mu": float(mu_t),
                    "electron_count": float(n_t), "passes": st["passes"], "n_doublings": st["n_doublings"],
                    "launch_budget": {"passes": 3, "doublings_per_pass": 10},
                    "note": "whole mixed step in one captured hipGraph (device-side mu search with predicated "
                            "passes and doublings), replayed"}, q.cpu().numpy()
        finally:
            c.set_mu_outputs(False)
            c.close()


BATCHED = dict(name="water3000", n_waters=3000, seed=7, grid=(5, 5, 6), tau=1e-5, kT=0.1, alpha=0.7)


def fp64_roofline(prof: dict, ms: float, n: np.ndarray, nc: np.ndarray, steps: int, leaf: int = 64) -> dict:
    """The FP64 path against the FP64 peak: nominal flops of the route it
    executes per step over the step time, and the dominant kernel."""
    fl = fp64_flops(n, nc, leaf)
    work = (fl["potrf"] + 2 * fl["trsm"] + fl["sytrd"] + fl["core_rows"] + fl["dc_apply"] + fl["dc_apply_rev"]
            + fl["dcore"])
    dom = max(prof.items(), key=lambda kv: kv[1]["ms_total"])
    return {"bound": "fp64", "achieved": work / (ms * 1e-3) / 1e12, "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
            "frac": work / (ms * 1e-3) / PEAK["fp64"], "flops_per_step": work, "dominant_kernel": dom[0],
            "dominant_kernel_ms_per_step": dom[1]["ms_per_step"],
            "note": "nominal flops of the executed route / step time"}


def time_fp64_batched(steps: int, warmup: int):
    """The batched FP64 workload: 3,000 waters, 5x5x6 cores, halos from the
    adaptive graph G_tau (tau 1e-5) grown from the neighbour partition's FP64
    solve: 150 subgraphs of about 1,200-1,700 orbitals, FP64 path only."""
    import torch
    import waterbox
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import Context, System, TBParams
    wl = BATCHED
    box = waterbox.water_box(wl["n_waters"], wl["seed"])
    c = Context(0)
    try:
        system = System(box.pos, box.species, box.anchor, box.box)
        tb = TBParams(orthogonal=False)
        part = pipeline.cutoff_partition(c, system, tb, wl["grid"])
        H, S = c.build_hs(system, tb, part.nbr)
        sol = pipeline.solve(c, system, part, H, S, wl["kT"], pipeline.FP64_EIG)
        g = c.build_graph_dm(system, pipeline.GRAPH_ADAPTIVE, part.sg, sol.D_core, wl["tau"], alpha=wl["alpha"],
                             nbr=part.nbr)
        part = pipeline.repartition(c, system, tb, part, g)
        n, nc = part.sg.norb, part.sg.ncore_orb
        from paper_2606_03140_amd import autotune
        tuned = autotune.apply_table(c, autotune.load_table(), int(n.max()), paths=("fp64",))
        log(f"[bench] batched FP64 workload: {part.sg.n_sub} subgraphs, n {n.min()}-{n.max()}; warmup {warmup}, "
            f"steps {steps}")
        sol, ms, wall, prof = time_path(c, system, part, H, S, wl["kT"], pipeline.FP64_EIG, steps, warmup)
        return {"workload": f"{wl['name']}: {wl['n_waters']} waters, {system.n_orb} orbitals, non-orthogonal, kT "
                            f"{wl['kT']} eV, {wl['grid'][0]}x{wl['grid'][1]}x{wl['grid'][2]} cores, adaptive G_tau at "
                            f"tau {wl['tau']}",
                "n_subgraphs": part.sg.n_sub, "orbitals_min": int(n.min()), "orbitals_max": int(n.max()),
                "ms_per_step": ms, "solves_per_s": part.sg.n_sub / (ms * 1e-3), "mu": sol.mu,
                "electron_count": sol.n_count, "tuning": tuned,
                "kernels_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in prof.items()},
                "roofline": fp64_roofline(prof, ms, n, nc, steps, tuned["fp64"]["leaf_rows"])}
    finally:
        c.close()


def cpu_baseline(box, wl, max_seconds: float = 20.0):
    """The oracle (untuned) on a bounded sample of the same workload: it builds
    its own partition (neighbour list, cores, the same adaptive rounds), then
    solves a sample of subgraphs with a thread pool over all host cores."""
    from oracle import graph as og
    from oracle import model as om
    from oracle import solve as osv
    m = om.TBModel(orthogonal=False, kT=wl["kT"])
    L = box.box[0]
    rp, col = om.neighbour_list_kdtree(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, wl["grid"])
    g = (rp, col)
    subs = og.extract_subgraphs(g[0], g[1], core, nco)
    for _ in range(wl["rounds"] - 1):
        res = osv.solve_system(box.pos, box.species, L, m, subs)
        gd = og.condensed_dm(subs, res.d_core, box.species, box.n_atoms)
        g = og.graph_union(box.n_atoms, g, og.graph_dm(gd, wl["tau"]))
        subs = og.extract_subgraphs(g[0], g[1], core, nco)
    workers = osv._workers()
    # sample: a stride through the subgraph list, grown until ~max_seconds of work
    rng = np.random.default_rng(0)
    order = rng.permutation(len(subs))
    done, t_used, k = 0, 0.0, 0
    batch = max(workers, 16)
    while t_used < max_seconds and k < len(order):
        chunk = [subs[i] for i in order[k:k + batch]]
        t0 = time.perf_counter()
        sols = osv.solve_subgraphs(box.pos, box.species, L, m, chunk, workers=workers)
        for s in sols:
            osv.d_core_rows(s, -7.0, m.beta)
        t_used += time.perf_counter() - t0
        done += len(chunk)
        k += batch
    n_sample = np.array([int(om.N_ORB[box.species[subs[i][0]]].sum()) for i in order[:done]])
    return {
        "value": done / t_used,
        "unit": "subgraph DM solves/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{done} of {len(subs)} subgraphs (n {n_sample.min()}-{n_sample.max()}, median "
                  f"{int(np.median(n_sample))}) of the oracle's own partition of the same box after "
                  f"{wl['rounds']} graph rounds; eigh(s), eigh(Z h Z), weights and D core rows per subgraph; "
                  f"{t_used:.1f} s",
    }


def copy_calibration():
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}), flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_gemm_split_water10000_traffic.json")


GEMM_SOURCE_END = "// ------------------------------------------------------------ FP64 GEMM"


def gemm_source_sha256():
    """SHA-256 of the split GEMM's source: mixed.hip from its start (constants,
    split helpers) to the end of k_gemm_split."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2606_03140_amd", "csrc", "mixed.hip")) as f:
        text = f.read()
    end = text.find(GEMM_SOURCE_END)
    return hashlib.sha256(text[:end if end >= 0 else len(text)].encode()).hexdigest()


def profile_mean_ms():
    """Mean split-GEMM dispatch duration of the committed rocprofv3 trace, or
    None when the kernel source has changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        sha = gemm_source_sha256()
    except (OSError, ValueError):
        return None
    return float(t["mean_duration_ms_trace"]) if t.get("source_sha256") == sha else None


def measured_traffic():
    """HBM bytes per split-GEMM dispatch from the committed rocprofv3 counter
    summary, or None when the kernel source has changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        sha = gemm_source_sha256()
    except (OSError, ValueError):
        return None
    return float(t["hbm_bytes_per_dispatch"]) if t.get("source_sha256") == sha else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--paths", default="fp64,mixed,mixed_bf16")
    ap.add_argument("--ns-z", type=int, default=0, help="coupled Newton-Schulz iterations for s^-1/2 (0: library "
                                                        "default)")
    ap.add_argument("--ns-inv", type=int, default=0, help="Newton-Schulz iterations per inverse in each doubling "
                                                          "(0: library default)")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="skip timing the whole mixed step as one captured hipGraph")
    ap.add_argument("--no-response", dest="response", action="store_false",
                    help="skip timing the charge response (the kernel-accelerated SCF's directional derivative)")
    ap.add_argument("--no-batched", dest="batched", action="store_false",
                    help="skip the batched FP64 workload (3,000 waters, adaptive graph at tau 1e-5)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the reference kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the per-subgraph "
              f"solve would shard over GPUs by subgraph, which is not built here.", file=sys.stderr)
        sys.exit(2)

    import torch
    import waterbox
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import Context, GDMError, System, TBParams

    wl = WORKLOAD
    log(f"[bench] generating {wl['n_waters']} waters (seed {wl['seed']})")
    box = waterbox.water_box(wl["n_waters"], wl["seed"])
    ctx = Context(0)
    system = System(box.pos, box.species, box.anchor, box.box)
    tb = TBParams(orthogonal=False)
    t0 = time.perf_counter()
    part = pipeline.cutoff_partition(ctx, system, tb, wl["grid"])
    H, S = ctx.build_hs(system, tb, part.nbr)
    for r in range(wl["rounds"] - 1):
        sol = pipeline.solve(ctx, system, part, H, S, wl["kT"], pipeline.FP64_EIG)
        g = ctx.build_graph_dm(system, pipeline.GRAPH_DM, part.sg, sol.D_core, wl["tau"], union=part.graph)
        part = pipeline.repartition(ctx, system, tb, part, g)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    n = part.sg.norb
    nc = part.sg.ncore_orb
    log(f"[bench] partition: {part.sg.n_sub} subgraphs, n {n.min()}-{n.max()} (median {int(np.median(n))}), "
        f"setup {setup_s:.1f} s")

    # run-time options chosen by the autotuner for this size bucket (library
    # defaults where its table has no entry); the command line overrides
    from paper_2606_03140_amd import autotune
    tuning = autotune.apply_table(ctx, autotune.load_table(), int(n.max()))
    log(f"[bench] tuned options ({autotune.bucket(int(n.max()))}): {tuning}")
    ctx.set_mixed_options(ns_z=args.ns_z, ns_inv=args.ns_inv)
    results = {}
    paths = [p for p in args.paths.split(",") if p]
    for path in paths:
        prec = {"fp64": pipeline.FP64_EIG, "mixed": pipeline.MIXED_F16, "mixed_bf16": pipeline.MIXED_BF16}[path]
        try:
            # mixed: mu is warm-started from the previous step, as in MD; the first
            # warm-up step starts from a crude guess (midpoint of the onsite energies)
            mu_guess = -15.0
            log(f"[bench] timing {path}: warmup {args.warmup}, steps {args.steps}")
            sol, ms, wall_ms, prof = time_path(ctx, system, part, H, S, wl["kT"], prec, args.steps, args.warmup,
                                               mu_guess)
            results[path] = {"ms_per_step": ms, "solves_per_s": part.sg.n_sub / (ms * 1e-3), "mu": sol.mu,
                             "n_count": sol.n_count, "kernels": prof, "q": sol.q.cpu().numpy(),
                             "D": sol.D_core}
            if path != "fp64":
                results[path]["stats"] = ctx.mixed_stats()
            log(f"[bench] {path}: {ms:.2f} ms/step, {results[path]['solves_per_s']:.1f} solves/s")
        except GDMError as e:
            log(f"[bench] {path} path unavailable: {e}")

    if "fp64" in results:
        r64 = results["fp64"]
        r64["roofline"] = fp64_roofline(r64["kernels"], r64["ms_per_step"], n, nc, args.steps,
                                        tuning["fp64"]["leaf_rows"])
    head = "mixed" if "mixed" in results else "fp64"
    R = results[head]
    fl = fp64_flops(n, nc)
    # roofline of the dominant kernel of the headline path
    kern = max(R["kernels"].items(), key=lambda kv: kv[1]["ms_total"])
    kname, kinfo = kern
    avg_ms = kinfo["ms_total"] / kinfo["launches"]
    if head == "fp64":
        work = fl.get(kname, sum(fl.values()))
        roof = {"bound": "alu", "kernel": kname, "achieved": work / (avg_ms * 1e-3) / 1e12,
                "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s", "traffic": None}
    else:
        # the split GEMM: three FP16 products per output tile (executed flops) and
        # its algorithmic HBM bytes; at ~90 flop/B it sits below the MI355X ridge
        # (2.5 PF / 8 TB/s = 312 flop/B), so the bound is HBM
        st = R["stats"]
        g = {k: v for k, v in R["kernels"].items() if k in ("foe_gemm", "ns_gemm")}
        ms_g = sum(v["ms_total"] for v in g.values())
        n_g = sum(v["launches"] for v in g.values())
        kname = "k_gemm_split (split-FP16 MFMA GEMM)"
        avg_ms = ms_g / n_g
        flops = 3.0 * st["flops_per_launch"]
        byts = st["bytes_per_launch"]
        intensity = flops / byts
        roof = {"bound": "hbm", "kernel": kname, "achieved": byts / (avg_ms * 1e-3) / 1e9,
                "peak": PEAK["hbm"] / 1e9, "unit": "GB/s", "traffic": measured_traffic(),
                "mfma_tflops": flops / (avg_ms * 1e-3) / 1e12, "mfma_peak_tflops": PEAK["fp16_mfma"] / 1e12,
                "mfma_frac": flops / (avg_ms * 1e-3) / PEAK["fp16_mfma"],
                "useful_tflops": st["flops_per_launch"] / (avg_ms * 1e-3) / 1e12,
                "flop_per_byte": intensity, "algorithmic_bytes_per_launch": byts,
                "mean_launch_ms": avg_ms, "gemm_launches_per_step": n_g / args.steps,
                "passes": st["passes"], "n_doublings": st["n_doublings"], "ns_z_used": st["ns_z_used"]}
        # the same launches counted on the method's own storage: each symmetric
        # matrix as n (n + 1) / 2 elements instead of the 64-padded upper tiles
        T = (n.astype(np.float64) + 63) // 64
        upper = float(np.sum(T * (T + 1) / 2 * 64.0 * 64.0))
        own = float(np.sum(n.astype(np.float64) * (n + 1) / 2))
        roof["algorithmic_bytes_per_launch_unpadded"] = byts * own / upper
        roof["frac_unpadded"] = byts * own / upper / (avg_ms * 1e-3) / PEAK["hbm"]
        prof = profile_mean_ms()
        if prof is not None:
            roof["mean_launch_ms_rocprof"] = prof
            roof["frac_rocprof"] = byts / (prof * 1e-3) / PEAK["hbm"]
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {
        "metric": "subgraph DM solves/s + % MFMA peak at 60k orbitals, mixed vs FP64 at 1e-4 e",
        "value": R["solves_per_s"],
        "unit": "subgraph DM solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16x3/f32acc+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl['name']}: {wl['n_waters']} waters, {system.n_atoms} atoms, {system.n_orb} "
                               f"orbitals, non-orthogonal, kT {wl['kT']} eV, {wl['grid'][0]}x{wl['grid'][1]}x"
                               f"{wl['grid'][2]} cores, tau {wl['tau']} ({wl['rounds']} graph rounds)",
                   "n_subgraphs": part.sg.n_sub, "orbitals_min": int(n.min()), "orbitals_median": int(np.median(n)),
                   "orbitals_max": int(n.max()), "path": head,
                   "mixed_options": {"ns_z": args.ns_z or 3, "ns_inv": args.ns_inv or tuning["mixed"]["ns_inv"],
                                     "inv_start": tuning["mixed"].get("inv_start", 2)},
                   "tuning": tuning},
        "paths": {k: {"ms_per_step": v["ms_per_step"], "solves_per_s": v["solves_per_s"], "mu": v["mu"],
                      "electron_count": v["n_count"],
                      "kernels_ms_per_step": {kk: round(vv["ms_per_step"], 4) for kk, vv in v["kernels"].items()},
                      **({"roofline": v["roofline"]} if "roofline" in v else {})}
                  for k, v in results.items()},
        "roofline": roof,
    }
    if "mixed" in results:
        log("[bench] mixed step from a cold mu guess")
        out["paths"]["mixed"]["cold_mu_step"] = time_cold(ctx, system, part, H, S, wl["kT"], -15.0)
        log(f"[bench] cold: {out['paths']['mixed']['cold_mu_step']['ms']:.1f} ms, "
            f"{out['paths']['mixed']['cold_mu_step']['passes']} passes")
        if args.graph:
            log(f"[bench] timing the whole mixed step as one captured hipGraph: warmup {args.warmup}, "
                f"steps {args.steps}")
            gr, q_graph = time_graph(system, part, H, S, wl["kT"], args.steps, args.warmup,
                                     results["mixed"]["mu"])
            gr["max_abs_dq_vs_eager_e"] = float(np.abs(q_graph - results["mixed"]["q"]).max())
            out["paths"]["mixed_graph"] = gr
            log(f"[bench] mixed hipGraph: {gr['ms_per_step']:.2f} ms/step")
    if args.batched and "fp64" in paths:
        out["paths"]["fp64_water3000"] = time_fp64_batched(min(args.steps, 3), min(args.warmup, 1))
        log(f"[bench] batched FP64: {out['paths']['fp64_water3000']['ms_per_step']:.1f} ms/step")
    if args.response and "mixed" in results:
        log(f"[bench] timing the charge response: warmup {args.warmup}, steps {args.steps}")
        out["response"] = time_response(ctx, system, part, H, S, wl["kT"], args.steps, args.warmup,
                                        results["mixed"]["mu"])
        log(f"[bench] response: {out['response']['ms_per_response']:.2f} ms")
    if "mixed" in results and "fp64" in results:
        # (a) self-consistent: each path with its own mu
        dq = np.abs(results["mixed"]["q"] - results["fp64"]["q"]).max()
        dD = (results["mixed"]["D"] - results["fp64"]["D"]).abs().max().item()
        # (b) at the FP64 path's mu: one expansion pass at that mu, density at that mu
        mu64 = results["fp64"]["mu"]
        ctx.plan(part.sg, pipeline.MIXED_F16)
        ctx.set_mixed_options(max_passes=1)
        ctx.find_mu(system, part.sg, part.nbr, H, S, wl["kT"], pipeline.MIXED_F16, mu64, 1e9)
        Dm = ctx.subgraph_density(part.sg, mu64, wl["kT"], pipeline.MIXED_F16)
        qm = ctx.mulliken_charges(system, part.sg, part.nbr, S, Dm).cpu().numpy()
        ctx.set_mixed_options(max_passes=16)
        out["mixed_vs_fp64"] = {
            "at_fp64_mu": {"max_abs_dD": (Dm - results["fp64"]["D"]).abs().max().item(),
                           "max_abs_dq_e": float(np.abs(qm - results["fp64"]["q"]).max()),
                           "mixed_count_error_e": float(qm.sum())},
            "self_consistent_mu": {"mu_mixed": results["mixed"]["mu"], "mu_fp64": mu64,
                                   "max_abs_dD": dD, "max_abs_dq_e": float(dq),
                                   "mixed_count_error_e": float(results["mixed"]["q"].sum())}}
    if "mixed_bf16" in results and "fp64" in results:
        rb = results["mixed_bf16"]
        out["paths"]["mixed_bf16"]["vs_fp64"] = {
            "mu_fp64": results["fp64"]["mu"],
            "max_abs_dD": (rb["D"] - results["fp64"]["D"]).abs().max().item(),
            "max_abs_dq_e": float(np.abs(rb["q"] - results["fp64"]["q"]).max()),
            "note": "split-BF16 path with its own mu against the FP64 path"}
    if not args.no_cpu:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s sample)")
        out["cpu_baseline"] = cpu_baseline(box, wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
