"""The autotuner on a small workload (300 waters, 27 cores): every timed
candidate is one of the listed settings, the admissible mixed candidates
stay within 1e-4 of the FP64 path, and with the chosen options applied both
paths still match the oracle (FP64 1e-9, mixed 1e-4)."""
import numpy as np
import pytest

import waterbox
from oracle import graph as og
from oracle import model as om
from oracle import solve as osv
from tests.gpu_common import ctx, log, oracle_model, system_of, tb_params, unpack_dcore

pytestmark = pytest.mark.gpu


def test_autotune_small_workload():
    from paper_2606_03140_amd import autotune, pipeline
    c = ctx()
    box = waterbox.water_box(300, 21)
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, (3, 3, 3))
    H, S = c.build_hs(sysm, tb, part.nbr)
    res = autotune.tune(c, sysm, part, H, S, 0.1, paths=("fp64", "mixed"), steps=1, warmup=0, log=log)
    for p in ("fp64", "mixed"):
        assert [r["opts"] for r in res[p]["candidates"]] == autotune.CANDIDATES[p]
        assert res[p]["choice"] in autotune.CANDIDATES[p]
    assert any(r["ok"] for r in res["mixed"]["candidates"])
    table = {autotune.bucket(int(part.sg.norb.max())): {p: {"choice": r["choice"]} for p, r in res.items()}}
    used = autotune.apply_table(c, table, int(part.sg.norb.max()), paths=("fp64", "mixed"))
    log(f"  chosen: {used}")
    try:
        L = box.box[0]
        rp, col = om.neighbour_list(box.pos, L)
        core, nco = og.grid_cores(box.pos, box.anchor, L, (3, 3, 3))
        ref = osv.solve_system(box.pos, box.species, L, oracle_model(False), og.extract_subgraphs(rp, col, core, nco))
        for prec, tol in ((pipeline.FP64_EIG, 1e-9), (pipeline.MIXED_F16, 1e-4)):
            sol = pipeline.solve(c, sysm, part, H, S, 0.1, prec, mu_guess=ref.mu)
            err_d = max(np.abs(a - b).max() for a, b in zip(unpack_dcore(part.sg, sol.D_core), ref.d_core))
            err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
            log(f"  precision {prec} with the chosen options: max|dD| {err_d:.2e} max|dq| {err_q:.2e}")
            assert err_d < tol and err_q < tol
    finally:
        autotune.apply(c, "fp64", autotune.DEFAULTS["fp64"])
        autotune.apply(c, "mixed", autotune.DEFAULTS["mixed"])
