"""Cost-balanced cores and re-partitioning (Determining the Subgraphs, Fig.
graph_partition f; Scalability section: subgraph cost grows as size cubed).

* An uneven box (800 waters with every molecule whose O lies in the first
  35% of the box along x removed): gdm_balanced_cores with the neighbour
  graph's degrees as weights gives the oracle's bisection bit for bit, a
  smaller spread of subgraph cost than the spatial grid with the same number
  of cores, and an FP64 solve on it matches the oracle within 1e-9.
* The re-partition trigger: cores chosen on the neighbour graph, then the
  graph grown from D at tau = 1e-5 (halos several times larger): the sum of
  n^3 passes 1.5 times its value at partitioning, new balanced cores are
  drawn from the grown graph (again identical to the oracle's), and the FP64
  solve on them matches the oracle within 1e-9.
"""
import numpy as np
import pytest
import torch

import waterbox
from oracle import graph as og
from oracle import model as om
from oracle import solve as osv
from tests.gpu_common import csr_host, ctx, log, oracle_model, system_of, tb_params, unpack_dcore

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c():
    return ctx()


def uneven_box(nw, seed, frac):
    box = waterbox.water_box(nw, seed)
    L = box.box[0]
    keep_mol = box.pos[box.anchor, 0] >= frac * L
    keep = np.nonzero(keep_mol)[0]
    new_index = -np.ones(box.n_atoms, dtype=np.int64)
    new_index[keep] = np.arange(len(keep))
    anchor = new_index[box.anchor[keep]].astype(np.int32)
    return waterbox.WaterBox(pos=np.ascontiguousarray(box.pos[keep]), species=box.species[keep].copy(),
                             anchor=anchor, box=box.box, n_waters=int((anchor == np.arange(len(keep))).sum()),
                             seed=seed)


def cost_spread(norb):
    n3 = norb.astype(np.float64) ** 3
    return n3.max() / n3.mean(), n3.sum()


def _fp64_vs_oracle(c, sysm, part, box, subs, label, pipeline):
    H, S = c.build_hs(sysm, tb_params(False), part.nbr)
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.FP64_EIG)
    ref = osv.solve_system(box.pos, box.species, box.box[0], oracle_model(False), subs)
    err_d = max(np.abs(a - b).max() for a, b in zip(unpack_dcore(part.sg, sol.D_core), ref.d_core))
    err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
    log(f"  {label}: mu {sol.mu:.6f} (oracle {ref.mu:.6f}) max|dD| {err_d:.2e} max|dq| {err_q:.2e}")
    assert err_d < 1e-9 and err_q < 1e-9
    return sol


def _same_subgraphs(part, subs):
    ap = part.sg.atom_ptr.cpu().numpy()
    at = part.sg.atoms.cpu().numpy()
    assert len(subs) == part.sg.n_sub
    for s, (atoms, ncore) in enumerate(subs):
        assert np.array_equal(at[ap[s]:ap[s + 1]], atoms), f"subgraph {s} differs"


def test_balanced_cores_on_an_uneven_box(c):
    from paper_2606_03140_amd import pipeline
    box = uneven_box(800, 5, 0.35)
    L = box.box[0]
    sysm = system_of(box)
    tb = tb_params(False)
    log(f"uneven box: {box.n_waters} waters of 800 kept, box {L:.2f} A")
    grid = pipeline.cutoff_partition(c, sysm, tb, (4, 4, 4))
    K = grid.n_cores
    bal = pipeline.balanced_partition(c, sysm, tb, K, nbr=grid.nbr)
    rp, col = csr_host(grid.nbr)
    ref_core = og.balanced_cores(box.pos, box.anchor, L, K, rp)
    assert np.array_equal(bal.core_of_atom.cpu().numpy(), ref_core)
    sg_spread, sg_cost = cost_spread(grid.sg.norb)
    bl_spread, bl_cost = cost_spread(bal.sg.norb)
    log(f"  {K} cores: grid n {grid.sg.norb.min()}-{grid.sg.norb.max()} max/mean n^3 {sg_spread:.2f} "
        f"sum n^3 {sg_cost:.3g}; balanced n {bal.sg.norb.min()}-{bal.sg.norb.max()} max/mean n^3 {bl_spread:.2f} "
        f"sum n^3 {bl_cost:.3g}")
    assert bl_spread < sg_spread
    subs = og.extract_subgraphs(rp, col, ref_core, K)
    _same_subgraphs(bal, subs)
    _fp64_vs_oracle(c, sysm, bal, box, subs, "FP64 on balanced cores", pipeline)


def test_repartition_when_halos_grow(c):
    from paper_2606_03140_amd import pipeline
    nw, seed, tau = 800, 55, 1e-5
    box = waterbox.water_box(nw, seed)
    L = box.box[0]
    n_at = box.n_atoms
    sysm = system_of(box)
    tb = tb_params(False)
    m = oracle_model(False)
    log(f"re-partition: {nw} waters, cores from the neighbour graph, graph grown at tau {tau}")
    part = pipeline.balanced_partition(c, sysm, tb, 64)
    rp0, col0 = csr_host(part.nbr)
    core0 = og.balanced_cores(box.pos, box.anchor, L, 64, rp0)
    assert np.array_equal(part.core_of_atom.cpu().numpy(), core0)
    subs0 = og.extract_subgraphs(rp0, col0, core0, 64)
    sol = _fp64_vs_oracle(c, sysm, part, box, subs0, "FP64 on the first cores", pipeline)
    r1 = osv.solve_system(box.pos, box.species, L, m, subs0)
    gd = og.condensed_dm(subs0, r1.d_core, box.species, n_at)
    orp, ocol = og.graph_union(n_at, (rp0, col0), og.graph_dm(gd, tau))
    g = c.build_graph_dm(sysm, pipeline.GRAPH_DM, part.sg, sol.D_core, tau, union=part.graph)
    rp, col = csr_host(g)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    new, changed = pipeline.maybe_repartition(c, sysm, tb, part, g, growth=1.5)
    grown = pipeline.subgraph_cost(pipeline.repartition(c, sysm, tb, part, g).sg)
    log(f"  sum n^3: at partitioning {part.cost0:.3g}, grown graph on the old cores {grown:.3g} "
        f"({grown / part.cost0:.2f}x), re-partitioned {new.cost0:.3g}; cores changed {changed}")
    assert changed and new.repartitions == 1
    core1 = og.balanced_cores(box.pos, box.anchor, L, 64, orp)
    assert np.array_equal(new.core_of_atom.cpu().numpy(), core1)
    subs1 = og.extract_subgraphs(orp, ocol, core1, 64)
    _same_subgraphs(new, subs1)
    _fp64_vs_oracle(c, sysm, new, box, subs1, "FP64 on the new cores", pipeline)
    # a step with no growth keeps the cores
    same, changed2 = pipeline.maybe_repartition(c, sysm, tb, new, g, growth=1.5)
    assert not changed2 and same.repartitions == 1
