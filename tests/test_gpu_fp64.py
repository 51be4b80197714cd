"""GPU parity of the graph, partition and FP64 subgraph solve against the oracle.

Integer outputs (CSR graph, cores, subgraph atom lists) must be bit-exact;
FP64 density-matrix core rows and Mulliken charges within 1e-9 (the FP64
target); electron count within 1e-9 of N_e.
"""
import numpy as np
import pytest
import torch

import waterbox
from oracle import graph as og
from oracle import model as om
from oracle import solve as osv
from tests.gpu_common import (csr_host, ctx, log, oracle_model, pack_dcore, system_of, tb_params,
                              unpack_dcore)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c():
    return ctx()


@pytest.mark.parametrize("nw,seed", [(16, 11), (96, 1), (3000, 2), (10000, 3)])
def test_cutoff_graph_bitexact(c, nw, seed):
    log(f"cutoff graph {nw} waters seed {seed}")
    box = waterbox.water_box(nw, seed)
    sysm = system_of(box)
    L = box.box[0]
    if L <= 8.0:
        pytest.skip("box too small for a 4 A minimum-image cutoff")
    g = c.build_graph_cutoff(sysm, 4.0)
    rp, col = csr_host(g)
    orp, ocol = om.neighbour_list(box.pos, L)
    assert np.array_equal(rp, orp)
    assert np.array_equal(col, ocol)


@pytest.mark.parametrize("nw,seed,cutoff", [(300, 21, 7.0), (300, 21, 10.0), (3000, 2, 12.0)])
def test_long_row_graph_bitexact(c, nw, seed, cutoff):
    """Wide cutoffs (Ewald real space, descriptors with a skin): rows of 140 to
    1,100 neighbours take the LDS bitonic row sort."""
    log(f"cutoff graph {nw} waters at {cutoff} A")
    box = waterbox.water_box(nw, seed)
    sysm = system_of(box)
    g = c.build_graph_cutoff(sysm, cutoff)
    rp, col = csr_host(g)
    orp, ocol = om.neighbour_list(box.pos, box.box[0], cutoff=cutoff)
    log(f"  {len(ocol)} edges, {len(ocol) / len(box.species):.0f} per atom")
    assert np.array_equal(rp, orp)
    assert np.array_equal(col, ocol)


@pytest.mark.parametrize("nw,seed,grid", [(96, 1, (2, 2, 2)), (10000, 3, (10, 10, 10)), (3000, 2, (5, 5, 6))])
def test_cores_and_subgraphs_bitexact(c, nw, seed, grid):
    log(f"cores/subgraphs {nw} waters grid {grid}")
    box = waterbox.water_box(nw, seed)
    sysm = system_of(box)
    L = box.box[0]
    g = c.build_graph_cutoff(sysm, 4.0)
    core, nco = c.grid_cores(sysm, grid)
    ocore, onco = og.grid_cores(box.pos, box.anchor, L, grid)
    assert nco == onco
    assert np.array_equal(core.cpu().numpy(), ocore)
    sg = c.extract_subgraphs(sysm, tb_params(False), g, core, nco)
    rp, col = csr_host(g)
    osubs = og.extract_subgraphs(rp, col, ocore, onco)
    gsubs = sg.host_lists()
    assert len(gsubs) == len(osubs)
    for (ga, gn), (oa, on) in zip(gsubs, osubs):
        assert gn == on and np.array_equal(ga, oa)
    norb = [int(om.N_ORB[box.species[a]].sum()) for a, _ in osubs]
    ncor = [int(om.N_ORB[box.species[a[:n]]].sum()) for a, n in osubs]
    assert list(sg.norb) == norb and list(sg.ncore_orb) == ncor


def test_hs_blocks_match_oracle(c):
    log("H/S blocks vs oracle dense H/S")
    box = waterbox.water_box(32, 11)
    sysm = system_of(box)
    L = box.box[0]
    for orth in (False, True):
        tb = tb_params(orth)
        g = c.build_graph_cutoff(sysm, 4.0)
        H, S = c.build_hs(sysm, tb, g)
        rp, col = csr_host(g)
        Hh = H.cpu().numpy().reshape(-1, 4, 4)
        Sh = None if S is None else S.cpu().numpy().reshape(-1, 4, 4)
        h_ref, s_ref = om.dense_hs(box.pos, box.species, L, oracle_model(orth))
        orb_ptr = om.orbital_layout(box.species)[0]
        nrm = np.abs(h_ref).max()
        err_h = err_s = 0.0
        n = box.n_atoms
        for i in range(n):
            ni = om.N_ORB[box.species[i]]
            oi = orb_ptr[i]
            blocks = [(i, n * 0 + len(col) + i)] + [(int(col[k]), k) for k in range(rp[i], rp[i + 1])]
            for j, k in blocks:
                nj = om.N_ORB[box.species[j]]
                oj = orb_ptr[j]
                err_h = max(err_h, np.abs(Hh[k, :ni, :nj] - h_ref[oi:oi + ni, oj:oj + nj]).max())
                if Sh is not None:
                    err_s = max(err_s, np.abs(Sh[k, :ni, :nj] - s_ref[oi:oi + ni, oj:oj + nj]).max())
        assert err_h <= 4e-16 * nrm * 8
        assert err_s <= 4e-16 * 8


def _oracle_partition(box, grid, L):
    rp, col = om.neighbour_list(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, grid)
    return og.extract_subgraphs(rp, col, core, nco)


@pytest.mark.parametrize("nw,seed,grid,orth", [(32, 11, (2, 2, 1), False), (32, 11, (2, 1, 1), True),
                                               (96, 1, (2, 2, 2), False), (96, 1, (3, 3, 3), True)])
def test_fp64_solve_cutoff_partition(c, nw, seed, grid, orth):
    log(f"fp64 solve {nw} waters grid {grid} orthogonal={orth}")
    from paper_2606_03140_amd import pipeline
    box = waterbox.water_box(nw, seed)
    sysm = system_of(box)
    L = box.box[0]
    tb = tb_params(orth)
    part = pipeline.cutoff_partition(c, sysm, tb, grid)
    H, S = c.build_hs(sysm, tb, part.nbr)
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.FP64_EIG, eig=True)
    subs = _oracle_partition(box, grid, L)
    ref = osv.solve_system(box.pos, box.species, L, oracle_model(orth), subs)
    assert abs(sol.n_count - sysm.n_electrons) < 1e-9
    gd = unpack_dcore(part.sg, sol.D_core)
    err_d = max(np.abs(a - b).max() for a, b in zip(gd, ref.d_core))
    err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
    log(f"  mu gpu {sol.mu:.10f} oracle {ref.mu:.10f}  max|dD| {err_d:.2e}  max|dq| {err_q:.2e}")
    assert err_d < 1e-9
    assert err_q < 1e-9
    assert abs(sol.q.sum().item()) < 1e-9
    # eigenvalues per subgraph (unordered on the GPU)
    E = sol.eig.cpu().numpy()
    for s, so in enumerate(ref.sols):
        e = np.sort(E[part.sg.eig_off[s]:part.sg.eig_off[s + 1]])
        assert np.abs(e - so.lam).max() < 1e-10


def test_fp64_many_small_subgraphs(c):
    """More subgraphs than compute units (the 512-thread form of the
    tridiagonalisation) and small, ragged sizes: 600 waters, 9x9x9 cores."""
    from paper_2606_03140_amd import pipeline
    box = waterbox.water_box(600, 7)
    sysm = system_of(box)
    L = box.box[0]
    grid = (9, 9, 9)
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, grid)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    log(f"fp64 solve 600 waters grid {grid}: {part.sg.n_sub} subgraphs of {part.sg.norb.min()}-"
        f"{part.sg.norb.max()} orbitals, {n_cu} CUs")
    assert part.sg.n_sub > n_cu
    H, S = c.build_hs(sysm, tb, part.nbr)
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.FP64_EIG, eig=True)
    subs = _oracle_partition(box, grid, L)
    ref = osv.solve_system(box.pos, box.species, L, oracle_model(False), subs)
    assert abs(sol.n_count - sysm.n_electrons) < 1e-9
    gd = unpack_dcore(part.sg, sol.D_core)
    err_d = max(np.abs(a - b).max() for a, b in zip(gd, ref.d_core))
    err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
    log(f"  mu gpu {sol.mu:.10f} oracle {ref.mu:.10f}  max|dD| {err_d:.2e}  max|dq| {err_q:.2e}")
    assert err_d < 1e-9
    assert err_q < 1e-9
    E = sol.eig.cpu().numpy()
    for s_, so in enumerate(ref.sols):
        e = np.sort(E[part.sg.eig_off[s_]:part.sg.eig_off[s_ + 1]])
        assert np.abs(e - so.lam).max() < 1e-10


def test_fp64_tiny_config_full_dm_graph(c):
    """96 waters, orthogonal, halos from |D_full| > 1e-5, 2x2x2 cores; parity
    with the oracle and with full-system diagonalisation."""
    log("water96 orthogonal full-DM graph")
    from paper_2606_03140_amd import pipeline
    box = waterbox.water_box(96, 1)
    sysm = system_of(box)
    L = box.box[0]
    tb = tb_params(True)
    m = oracle_model(True)
    part = pipeline.graph_from_full_dm(c, sysm, tb, (2, 2, 2), 1e-5, 0.1)
    H, S = c.build_hs(sysm, tb, part.nbr)
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.FP64_EIG)
    full = osv.full_system(box.pos, box.species, L, m)
    gd = og.condensed_dm(full.subs, full.d_core, box.species, box.n_atoms)
    orp, ocol = og.graph_dm(gd, 1e-5)
    rp, col = csr_host(part.graph)
    ties = og.near_ties(gd.data, 1e-5)
    log(f"  graph edges gpu {len(col)} oracle {len(ocol)} near-ties {ties}")
    assert ties == 0
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    core, nco = og.grid_cores(box.pos, box.anchor, L, (2, 2, 2))
    subs = og.extract_subgraphs(orp, ocol, core, nco)
    ref = osv.solve_system(box.pos, box.species, L, m, subs)
    err_d = max(np.abs(a - b).max() for a, b in zip(unpack_dcore(part.sg, sol.D_core), ref.d_core))
    err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
    err_full = np.abs(sol.q.cpu().numpy() - full.q).max()
    log(f"  max|dD| {err_d:.2e} max|dq| {err_q:.2e} vs full diag {err_full:.2e}")
    assert err_d < 1e-9 and err_q < 1e-9
    assert err_full < 1e-6


def test_dm_and_adaptive_graph_from_same_D(c):
    """Graph builders fed the oracle's D bytes: DM mode bit-exact; adaptive mode
    exact up to near ties of the summed weights (none expected)."""
    log("graph from D: same D bytes")
    box = waterbox.water_box(300, 21)
    sysm = system_of(box)
    L = box.box[0]
    tb = tb_params(False)
    m = oracle_model(False)
    grid = (3, 3, 3)
    from paper_2606_03140_amd import pipeline
    part = pipeline.cutoff_partition(c, sysm, tb, grid)
    subs = _oracle_partition(box, grid, L)
    ref = osv.solve_system(box.pos, box.species, L, m, subs)
    c.plan(part.sg, pipeline.FP64_EIG)
    D = pack_dcore(ref.d_core)
    gd = og.condensed_dm(subs, ref.d_core, box.species, box.n_atoms)
    for tau in (1e-3, 1e-5):
        g = c.build_graph_dm(sysm, pipeline.GRAPH_DM, part.sg, D, tau)
        orp, ocol = og.graph_dm(gd, tau)
        rp, col = csr_host(g)
        assert og.near_ties(gd.data, tau) == 0
        assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    rp0, col0 = om.neighbour_list(box.pos, L)
    gn = og.distance_graph(box.pos, L, rp0, col0, 0.7)
    for tau in (1e-3, 1e-4):
        g = c.build_graph_dm(sysm, pipeline.GRAPH_ADAPTIVE, part.sg, D, tau, alpha=0.7, nbr=part.nbr)
        (orp, ocol), w = og.graph_adaptive(gn, gd, tau)
        rp, col = csr_host(g)
        ties = og.near_ties(w.data, tau)
        log(f"  adaptive tau {tau}: edges gpu {len(col)} oracle {len(ocol)} near-ties {ties}")
        # every edge is compared: the two edge sets may differ only on pairs
        # whose summed weight lies within 1e-9 tau of the threshold (with no
        # near tie they are identical)
        n = box.n_atoms
        ek = lambda r_, c_: set((np.repeat(np.arange(n), np.diff(r_)) * n + c_).tolist())
        diff = ek(rp, col) ^ ek(orp, ocol)
        near = np.abs(w.data - tau) <= 1e-9 * tau
        tie_pairs = set((w.row[near].astype(np.int64) * n + w.col[near]).tolist())
        tie_pairs |= set((w.col[near].astype(np.int64) * n + w.row[near]).tolist())
        assert diff <= tie_pairs, f"{len(diff - tie_pairs)} edges differ away from the threshold"
        if ties == 0:
            assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
