"""Edge cases of the GPU path against the oracle, and the host validation.

* one water in a 30 A box: one subgraph of 6 orbitals (a single partial
  tile in both solvers), FP64 within 1e-9 and mixed within 1e-4 of the
  oracle;
* isolated cores: 5 waters more than 4 A apart on a 2x2x2 grid, so three
  grid cells are empty and every subgraph has an empty halo;
* one large subgraph: 300 waters as a single core (1,800 orbitals, 29 tiles
  of 64 per side) on the mixed path, at the oracle's mu, against full
  diagonalisation;
* host validation: an empty system, no subgraphs, a subgraph above the
  8,192-orbital limit and null outputs are rejected with GDM_E_ARG before
  anything is enqueued; a failed plan leaves no plan (GDM_E_STATE for the
  solve calls), and the context stays usable afterwards.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import waterbox
from oracle import model as om
from oracle import solve as osv
from tests.gpu_common import ctx, log, oracle_model, tb_params, unpack_dcore

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c():
    return ctx()


def waters_at(centres, L):
    """Single-water geometries translated to the given O positions."""
    pos0, sp0, _ = om.single_water_reference(om.TBModel())
    pos, sp, anchor = [], [], []
    for k, o in enumerate(centres):
        pos.append(pos0 - pos0[0] + np.asarray(o, dtype=np.float64))
        sp.append(sp0)
        anchor += [3 * k] * 3
    return np.concatenate(pos), np.concatenate(sp).astype(np.int32), np.array(anchor, dtype=np.int32), L


def solve_both(c, pos, species, anchor, L, grid, orth=False):
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import System
    sysm = System(pos, species, anchor, [L, L, L])
    tb = tb_params(orth)
    part = pipeline.cutoff_partition(c, sysm, tb, grid)
    H, S = c.build_hs(sysm, tb, part.nbr)
    subs = part.sg.host_lists()
    ref = osv.solve_system(pos, species, L, oracle_model(orth), subs, workers=1)
    out = {}
    for name, prec in (("fp64", pipeline.FP64_EIG), ("mixed", pipeline.MIXED_F16)):
        sol = pipeline.solve(c, sysm, part, H, S, 0.1, prec, mu_guess=ref.mu)
        gd = unpack_dcore(part.sg, sol.D_core)
        out[name] = (max(np.abs(a - b).max() for a, b in zip(gd, ref.d_core)),
                     np.abs(sol.q.cpu().numpy() - ref.q).max(), sol.n_count - sysm.n_electrons)
    return part, out


@pytest.mark.parametrize("orth", [False, True])
def test_single_water(c, orth):
    log(f"single water in a 30 A box, orthogonal={orth}")
    pos, sp, anchor, L = waters_at([[15.0, 15.0, 15.0]], 30.0)
    part, out = solve_both(c, pos, sp, anchor, L, (1, 1, 1), orth)
    assert part.sg.n_sub == 1 and int(part.sg.norb[0]) == 6
    log(f"  {out}")
    assert out["fp64"][0] < 1e-9 and out["fp64"][1] < 1e-9 and abs(out["fp64"][2]) < 1e-9
    assert out["mixed"][0] < 1e-4 and out["mixed"][1] < 1e-4 and abs(out["mixed"][2]) < 1e-6


def test_isolated_cores_empty_halos(c):
    log("5 isolated waters, 2x2x2 grid: empty halos and empty cells")
    centres = [[10, 10, 10], [30, 10, 10], [10, 30, 10], [10, 10, 30], [30, 30, 30]]
    pos, sp, anchor, L = waters_at(centres, 40.0)
    part, out = solve_both(c, pos, sp, anchor, L, (2, 2, 2))
    assert part.sg.n_sub == 5
    assert np.all(part.sg.norb == 6) and np.all(part.sg.ncore_orb == 6)
    log(f"  {out}")
    assert out["fp64"][0] < 1e-9 and out["fp64"][1] < 1e-9
    assert out["mixed"][0] < 1e-4 and out["mixed"][1] < 1e-4


def test_one_large_subgraph_mixed(c):
    from paper_2606_03140_amd import pipeline
    from tests.gpu_common import system_of
    log("300 waters as one subgraph (1,800 orbitals), mixed path at the oracle's mu")
    box = waterbox.water_box(300, 21)
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.full_system_partition(c, sysm, tb)
    H, S = c.build_hs(sysm, tb, part.nbr)
    ref = osv.full_system(box.pos, box.species, box.box[0], oracle_model(False))
    assert part.sg.n_sub == 1 and int(part.sg.norb[0]) == 1800
    c.plan(part.sg, pipeline.MIXED_F16)
    c.set_mixed_options(max_passes=1)
    try:
        c.find_mu(sysm, part.sg, part.nbr, H, S, 0.1, pipeline.MIXED_F16, ref.mu, 1e9)
        D = c.subgraph_density(part.sg, ref.mu, 0.1, pipeline.MIXED_F16)
        q = c.mulliken_charges(sysm, part.sg, part.nbr, S, D).cpu().numpy()
    finally:
        c.set_mixed_options(max_passes=16)
    err_d = np.abs(unpack_dcore(part.sg, D)[0] - ref.d_core[0]).max()
    err_q = np.abs(q - ref.q).max()
    st = c.mixed_stats()
    log(f"  n_d {st['n_doublings']}, ns_z {st['ns_z_used']}: max|dD| {err_d:.2e} max|dq| {err_q:.2e}")
    assert err_d < 1e-4 and err_q < 1e-4


def test_one_large_subgraph_fp64(c):
    """The largest subgraph the FP64 path takes (2,048 orbitals): 340 waters as
    one subgraph, 2,040 orbitals, every row a core row; D, charges, mu and
    eigenvalues against the oracle's full diagonalisation."""
    from paper_2606_03140_amd import pipeline
    from tests.gpu_common import system_of
    log("340 waters as one subgraph (2,040 orbitals), FP64 path")
    box = waterbox.water_box(340, 21)
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.full_system_partition(c, sysm, tb)
    assert part.sg.n_sub == 1 and int(part.sg.norb[0]) == 2040
    H, S = c.build_hs(sysm, tb, part.nbr)
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.FP64_EIG, eig=True)
    ref = osv.full_system(box.pos, box.species, box.box[0], oracle_model(False))
    err_d = np.abs(unpack_dcore(part.sg, sol.D_core)[0] - ref.d_core[0]).max()
    err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
    err_l = np.abs(np.sort(sol.eig.cpu().numpy()) - np.sort(ref.sols[0].lam)).max()
    log(f"  mu gpu {sol.mu:.10f} oracle {ref.mu:.10f}  max|dD| {err_d:.2e} max|dq| {err_q:.2e} max|dlam| {err_l:.2e}")
    # mu sits in the gap of the whole system, where the count is flat to its
    # rounding: D does not depend on where (1e-14 above), so mu is bounded
    # loosely and the count exactly
    assert abs(sol.mu - ref.mu) < 1e-6
    assert err_d < 1e-9 and err_q < 1e-9 and err_l < 1e-10
    assert abs(sol.n_count - sysm.n_electrons) < 1e-9


def test_host_validation(c):
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import GDMError, Subgraphs, System
    lib = c.lib
    # empty system
    empty = System(np.zeros((0, 3)), np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.int32), [10.0] * 3)
    with pytest.raises(GDMError) as e:
        c.build_graph_cutoff(empty, 4.0)
    assert e.value.code == -1
    # no subgraphs
    z = torch.zeros(1, dtype=torch.int32, device=c.dev)
    none_sg = Subgraphs(z, z, z, np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.int32))
    with pytest.raises(GDMError) as e:
        c.plan(none_sg, pipeline.MIXED_F16)
    assert e.value.code == -1
    # a subgraph above the 8,192-orbital limit
    ap = torch.tensor([0, 3], dtype=torch.int32, device=c.dev)
    at = torch.tensor([0, 1, 2], dtype=torch.int32, device=c.dev)
    nc = torch.tensor([3], dtype=torch.int32, device=c.dev)
    big = Subgraphs(ap, at, nc, np.array([9000], dtype=np.int32), np.array([9000], dtype=np.int32))
    for prec in (pipeline.FP64_EIG, pipeline.MIXED_F16):
        with pytest.raises(GDMError) as e:
            c.plan(big, prec)
        assert e.value.code == -1
    # a failed plan leaves no plan behind: solve calls report GDM_E_STATE
    with pytest.raises(GDMError) as e:
        c.subgraph_density(big, -7.0, 0.1, pipeline.MIXED_F16)
    assert e.value.code == -8
    # null outputs of find_mu on a valid plan
    pos, sp, anchor, L = waters_at([[15.0, 15.0, 15.0]], 30.0)
    sysm = System(pos, sp, anchor, [L, L, L])
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, (1, 1, 1))
    H, S = c.build_hs(sysm, tb, part.nbr)
    c.plan(part.sg, pipeline.MIXED_F16)
    rc = lib.gdm_find_mu(c.h, C.byref(sysm.struct()), C.byref(part.sg.struct()), C.c_void_p(part.nbr.row_ptr.data_ptr()),
                         C.c_void_p(part.nbr.col.data_ptr()), part.nbr.nnz, C.c_void_p(H.data_ptr()),
                         C.c_void_p(S.data_ptr()), sysm.n_electrons, 0.1, pipeline.MIXED_F16, -7.0, 1e-6, None, None)
    assert rc == -1
    # density before find_mu on this plan
    with pytest.raises(GDMError) as e:
        c.subgraph_density(part.sg, -7.0, 0.1, pipeline.MIXED_F16)
    assert e.value.code == -8
    # the context still works
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.MIXED_F16, mu_guess=-7.0, plan=False)
    assert abs(sol.n_count - sysm.n_electrons) < 1e-6


@pytest.mark.gpu
def test_mixed_density_outside_first_order_range_rejected():
    """The mixed path's density at another mu or kT than its expansion is a
    first-order extrapolation: a different kT, or mu more than kT away from the
    last pass, is rejected on the host (GDM_E_ARG), and a mu inside the range
    still works."""
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import GDMError, System
    c = ctx()
    log("mixed density: kT and mu range checks")
    pos, sp, anchor, L = waters_at([[15.0, 15.0, 15.0], [17.6, 15.2, 15.1]], 30.0)
    sysm = System(pos, sp, anchor, [L, L, L])
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, (1, 1, 1))
    H, S = c.build_hs(sysm, tb, part.nbr)
    c.plan(part.sg, pipeline.MIXED_F16)
    mu, n = c.find_mu(sysm, part.sg, part.nbr, H, S, 0.1, pipeline.MIXED_F16, -7.0, 1e-6)
    mu_pass = c.mixed_mu_state()["mu_pass"]
    assert abs(mu - mu_pass) <= 0.1
    for bad_mu, bad_kT in ((mu, 0.2), (mu_pass + 0.25, 0.1), (mu_pass - 0.11, 0.1)):
        with pytest.raises(GDMError) as e:
            c.subgraph_density(part.sg, bad_mu, bad_kT, pipeline.MIXED_F16)
        assert e.value.code == -1
    D = c.subgraph_density(part.sg, mu_pass + 0.09, 0.1, pipeline.MIXED_F16)
    assert torch.isfinite(D).all()
    D = c.subgraph_density(part.sg, mu, 0.1, pipeline.MIXED_F16)
    assert torch.isfinite(D).all()
