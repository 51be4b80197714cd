"""Parity at the benchmark sizes.

10,000 waters (30,000 atoms, 1,000 subgraphs: the solve's launch
configuration in bench.py, every subgraph in one batch) and 3,000 waters
(9,000 atoms, 150 subgraphs of several hundred orbitals), on the
neighbour-graph partition, which GPU and oracle build bit-identically
(asserted here).  Every subgraph's D core rows and every charge are compared
with the oracle's full FP64 solve: the FP64 path within 1e-9, the mixed path
(at the oracle's mu) within 1e-4 and 1e-4 e; the electron count at the GPU's
mu within 1e-9 N_e.
"""
import numpy as np
import pytest

import waterbox
from oracle import graph as og
from oracle import model as om
from oracle import solve as osv
from tests.gpu_common import ctx, log, oracle_model, system_of, tb_params, unpack_dcore

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c():
    return ctx()


@pytest.mark.parametrize("nw,seed,grid", [(3000, 2, (5, 5, 6)), (10000, 3, (10, 10, 10))])
def test_fullsize_fp64_and_mixed(c, nw, seed, grid):
    from paper_2606_03140_amd import pipeline
    log(f"full-size parity: {nw} waters, cores {grid}")
    box = waterbox.water_box(nw, seed)
    L = box.box[0]
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, grid)
    H, S = c.build_hs(sysm, tb, part.nbr)
    rp, col = om.neighbour_list_kdtree(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, grid)
    subs = og.extract_subgraphs(rp, col, core, nco)
    # identical partitions
    ap = part.sg.atom_ptr.cpu().numpy()
    at = part.sg.atoms.cpu().numpy()
    assert len(subs) == part.sg.n_sub
    for s, (atoms, ncore) in enumerate(subs):
        assert np.array_equal(at[ap[s]:ap[s + 1]], atoms)
    log(f"  {part.sg.n_sub} subgraphs, n {part.sg.norb.min()}-{part.sg.norb.max()}; oracle solve ...")
    ref = osv.solve_system(box.pos, box.species, L, oracle_model(False), subs)
    # FP64 path
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.FP64_EIG)
    gd = unpack_dcore(part.sg, sol.D_core)
    err_d = max(np.abs(a - b).max() for a, b in zip(gd, ref.d_core))
    err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
    log(f"  FP64: mu {sol.mu:.9f} (oracle {ref.mu:.9f}) N {sol.n_count:.9f}  max|dD| {err_d:.2e} "
        f"max|dq| {err_q:.2e}")
    assert abs(sol.n_count - sysm.n_electrons) <= 1e-9 * sysm.n_electrons
    assert err_d < 1e-9 and err_q < 1e-9
    # mixed path at the oracle's mu: one expansion pass there, density there
    c.plan(part.sg, pipeline.MIXED_F16)
    c.set_mixed_options(max_passes=1)
    try:
        c.find_mu(sysm, part.sg, part.nbr, H, S, 0.1, pipeline.MIXED_F16, ref.mu, 1e9)
        Dm = c.subgraph_density(part.sg, ref.mu, 0.1, pipeline.MIXED_F16)
        qm = c.mulliken_charges(sysm, part.sg, part.nbr, S, Dm).cpu().numpy()
    finally:
        c.set_mixed_options(max_passes=16)
    md = unpack_dcore(part.sg, Dm)
    err_dm = max(np.abs(a - b).max() for a, b in zip(md, ref.d_core))
    err_qm = np.abs(qm - ref.q).max()
    log(f"  mixed at the oracle's mu: max|dD| {err_dm:.2e} max|dq| {err_qm:.2e}")
    assert err_dm < 1e-4 and err_qm < 1e-4
