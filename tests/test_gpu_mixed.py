"""GPU parity of the mixed-precision recursive Fermi expansion (split FP16 or
split BF16 MFMA, FP32 accumulation, FP64 bounds/traces/final step) against
the FP64 oracle: D core rows within 1e-4 max-abs and Mulliken charges within
1e-4 e, electron count within the requested tolerance."""
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


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("nw,seed,grid,orth", [(96, 1, (2, 2, 2), False), (96, 1, (3, 3, 3), True),
                                               (300, 21, (3, 3, 3), False)])
def test_mixed_matches_fp64_oracle(c, nw, seed, grid, orth, bf16):
    from paper_2606_03140_amd import pipeline
    prec = pipeline.MIXED_BF16 if bf16 else pipeline.MIXED_F16
    log(f"mixed solve ({'split BF16' if bf16 else 'split FP16'}) {nw} waters grid {grid} orthogonal={orth}")
    box = waterbox.water_box(nw, seed)
    sysm = system_of(box)
    L = box.box[0]
    tb = tb_params(orth)
    part = pipeline.cutoff_partition(c, sysm, tb, grid)
    H, S = c.build_hs(sysm, tb, part.nbr)
    rp, col = om.neighbour_list(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, grid)
    subs = og.extract_subgraphs(rp, col, core, nco)
    ref = osv.solve_system(box.pos, box.species, L, oracle_model(orth), subs)
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, prec, mu_guess=ref.mu + 0.05, tol_N=1e-6)
    st = c.mixed_stats()
    gd = unpack_dcore(part.sg, sol.D_core)
    err_d = max(np.abs(a - b).max() for a, b in zip(gd, ref.d_core))
    err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
    log(f"  mu {sol.mu:.6f} (oracle {ref.mu:.6f}) N {sol.n_count:.9f} passes {st['passes']} n_d "
        f"{st['n_doublings']} gemms {st['gemm_launches']}  max|dD| {err_d:.2e} max|dq| {err_q:.2e}")
    assert abs(sol.n_count - sysm.n_electrons) <= 1e-7 * sysm.n_electrons + 1e-9
    # split BF16 carries 16 significant bits per operand (FP16: 22): bound 1e-3
    tol = 1e-3 if bf16 else 1e-4
    assert err_d < tol
    assert err_q < tol


def test_mixed_mu_search_from_far_guess(c):
    """mu found from a guess inside a band: Newton + bisection passes still
    land within tolerance, and D matches the FP64 oracle to 1e-4."""
    log("mixed mu search from a far guess")
    from paper_2606_03140_amd import pipeline
    box = waterbox.water_box(96, 1)
    sysm = system_of(box)
    L = box.box[0]
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 2))
    H, S = c.build_hs(sysm, tb, part.nbr)
    rp, col = om.neighbour_list(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, (2, 2, 2))
    subs = og.extract_subgraphs(rp, col, core, nco)
    ref = osv.solve_system(box.pos, box.species, L, oracle_model(False), subs)
    c.set_mixed_options(max_passes=16)
    sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.MIXED_F16, mu_guess=-15.0, tol_N=1e-6)
    c.set_mixed_options(max_passes=16)
    st = c.mixed_stats()
    err_q = np.abs(sol.q.cpu().numpy() - ref.q).max()
    log(f"  passes {st['passes']} mu {sol.mu:.6f} N {sol.n_count:.9f} max|dq| {err_q:.2e}")
    assert abs(sol.n_count - sysm.n_electrons) <= 1e-7 * sysm.n_electrons + 1e-9
    assert err_q < 1e-4


def test_inverse_overlap_residual_guard(c):
    """The inverse-overlap factor takes coupled Newton-Schulz iterations until
    |Z s Z - I| is small enough for one refinement step: from one iteration
    with no extra allowed gdm_find_mu reports GDM_E_NOT_CONVERGED instead of
    a silently inaccurate density; with extra iterations allowed it adds
    them and matches the default solve."""
    log("inverse-overlap residual guard (ns_z = 1 without and with extra iterations)")
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import GDMError
    box = waterbox.water_box(96, 1)
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 2))
    H, S = c.build_hs(sysm, tb, part.nbr)
    ref = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.MIXED_F16, mu_guess=-7.0)
    used_default = c.mixed_stats()["ns_z_used"]
    try:
        c.set_mixed_options(ns_z=1, ns_z_extra=0)
        with pytest.raises(GDMError) as e:
            pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.MIXED_F16, mu_guess=-7.0)
        assert e.value.code == -5
        c.set_mixed_options(ns_z=1, ns_z_extra=8)
        sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.MIXED_F16, mu_guess=-7.0)
        used = c.mixed_stats()["ns_z_used"]
    finally:
        c.set_mixed_options(ns_z=3, ns_z_extra=8)   # the library defaults
    log(f"  iterations: default {used_default}, from 1 with extras {used}; "
        f"max|dq| vs default {float((sol.q - ref.q).abs().max()):.2e}")
    assert 1 < used <= 9 and used_default >= 3
    assert float((sol.q - ref.q).abs().max()) < 1e-5


@pytest.mark.parametrize("nw,seed,grid", [(96, 1, (2, 2, 2)), (300, 21, (3, 3, 3))])
def test_upper_tile_storage_matches_whole_storage(c, nw, seed, grid):
    """The expansion with its symmetric matrices stored as upper tiles (a
    lower tile read as its stored mirror, transposed) against whole storage
    (every product also writes the mirror tiles): same doublings and
    launches, D core rows equal to FP32 rounding, fewer bytes per launch.
    They need not agree bit for bit: whole storage writes a mirror tile from
    registers with its own rounding of the epilogue (alpha AB + beta E +
    gamma I), so its lower tiles may differ from the upper ones in the last
    bit, which upper-tile storage never reads.  Subgraphs of several
    64-tiles with ragged tails; one pass at a fixed mu."""
    from paper_2606_03140_amd import pipeline
    log(f"upper-tile vs whole storage, {nw} waters, grid {grid}")
    box = waterbox.water_box(nw, seed)
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, grid)
    H, S = c.build_hs(sysm, tb, part.nbr)
    c.plan(part.sg, pipeline.MIXED_F16)
    P0 = 64 * ((int(part.sg.norb[0]) + 63) // 64)
    out = {}
    try:
        c.set_mixed_options(max_passes=1)
        for upper in (False, True):
            c.set_mixed_storage(upper)
            c.find_mu(sysm, part.sg, part.nbr, H, S, 0.1, pipeline.MIXED_F16, -6.9, 1e9)
            D = c.subgraph_density(part.sg, -6.9, 0.1, pipeline.MIXED_F16)
            X = c.debug_slot(2, 0, P0).cpu().numpy()
            out[upper] = (D.cpu().numpy(), c.mixed_stats(), float(np.abs(X - X.T).max()))
    finally:
        c.set_mixed_storage(True)
        c.set_mixed_options(max_passes=16)
    (Dw, sw, aw), (Du, su, au) = out[False], out[True]
    err = float(np.abs(Dw - Du).max())
    log(f"  n_d {su['n_doublings']}, launches {su['gemm_launches']}, bytes per launch "
        f"{sw['bytes_per_launch'] / 1e6:.1f} MB whole, {su['bytes_per_launch'] / 1e6:.1f} MB upper tiles, "
        f"max|dD| {err:.1e}, max|X - X^T| {aw:.1e} whole, {au:.1e} upper tiles")
    assert sw["n_doublings"] == su["n_doublings"] and sw["gemm_launches"] == su["gemm_launches"]
    assert err < 1e-6
    assert su["bytes_per_launch"] < 0.9 * sw["bytes_per_launch"]
