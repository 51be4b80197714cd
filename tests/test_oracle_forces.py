"""Pins of the force and XL-BOMD oracle (oracle/forces.py, oracle/xlbomd.py)
against what the mathematics and the paper fix:

* the Slater-Koster pair blocks equal those of the pinned dense H and S;
* their gradients and the taper's equal central differences, and the taper
  is continuous with its slope and curvature at both ends;
* the total force is the central difference of U(R, n) at fixed n (a
  dropped Pulay, SCC-shift, Coulomb or repulsion term, or a wrong sign,
  fails it);
* forces sum to zero; the partitioned forces with full halos equal the
  full-system forces;
* U(R, n) - E_SCC is quadratic in the charge error (Eq. UErr);
* the repulsive prefactors give an isolated water zero force at its
  reference geometry;
* the dissipation coefficients leave constant and linear histories alone,
  and the total free energy fluctuation of XL-BOMD on a water dimer grows
  by four when dt doubles (Shadow MD results: global second-order error).
"""
import numpy as np
import pytest

import waterbox
from oracle import forces as fo
from oracle import graph, model, scc, xlbomd

MD = dict(taper_on=3.5, rep_A=(500.0, 67.92, 12.79), rep_rho=0.3)
TH = np.radians(52.25)
WATER = np.array([[0.0, 0.0, 0.0], [0.96 * np.sin(TH), 0.0, 0.96 * np.cos(TH)],
                  [-0.96 * np.sin(TH), 0.0, 0.96 * np.cos(TH)]])
ROT = np.array([[0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])


def dimer(jitter=0.0, seed=3):
    pos = np.concatenate([WATER + 3.0, WATER @ ROT.T + [3.3, 3.1, 5.9]])
    if jitter:
        pos = pos + np.random.default_rng(seed).normal(scale=jitter, size=pos.shape)
    return pos, np.array([0, 1, 1, 0, 1, 1])


def converged(pos, species, L, m, ew, subs):
    q, _, _ = scc.scc(pos, species, L, m, subs, mix=0.3, tol=1e-11, max_iter=400, eta=ew.eta, n_real=ew.n_real,
                      k_max=ew.k_max)
    return q


def test_sk_blocks_equal_dense_hs():
    m = model.TBModel(taper_on=3.0)
    rng = np.random.default_rng(0)
    for si, sj in ((0, 1), (0, 0), (1, 0), (1, 1)):
        d = rng.normal(size=3)
        d *= rng.uniform(1.0, 3.8) / np.linalg.norm(d)
        pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0] + d])
        sp = np.array([si, sj])
        h, s = model.dense_hs(pos, sp, 20.0, m)
        ni = model.N_ORB[si]
        hb, sb, _, _ = fo.sk_block(d, si, sj, m)
        np.testing.assert_allclose(hb, h[:ni, ni:], rtol=0, atol=1e-14)
        np.testing.assert_allclose(sb, s[:ni, ni:], rtol=0, atol=1e-14)


@pytest.mark.parametrize("r", [1.3, 3.7])
def test_sk_gradients_central_difference(r):
    m = model.TBModel(taper_on=3.5)
    d0 = np.array([0.3, -0.5, 0.8])
    d0 *= r / np.linalg.norm(d0)
    h_ = 1e-6
    for si, sj in ((0, 0), (0, 1), (1, 0)):
        _, _, dh, ds = fo.sk_block(d0, si, sj, m)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h_
            hp, sp_, _, _ = fo.sk_block(d0 + e, si, sj, m)
            hm, sm, _, _ = fo.sk_block(d0 - e, si, sj, m)
            np.testing.assert_allclose(dh[c], (hp - hm) / (2 * h_), rtol=0, atol=1e-8)
            np.testing.assert_allclose(ds[c], (sp_ - sm) / (2 * h_), rtol=0, atol=1e-8)


def test_taper_is_c2():
    r_on, r_c = 3.5, 4.0
    t = lambda r: float(model.taper(r, r_on, r_c))
    dt = lambda r: float(fo.taper_deriv(r, r_on, r_c))
    assert t(r_on) == 1.0 and t(r_c) == 0.0 and t(3.0) == 1.0 and t(4.5) == 0.0
    for r in (3.6, 3.75, 3.9):
        assert abs(dt(r) - (t(r + 1e-7) - t(r - 1e-7)) / 2e-7) < 1e-7
    d2t = lambda r: (dt(r + 1e-7) - dt(r - 1e-7)) / 2e-7
    assert max(abs(d2t(r)) for r in np.linspace(3.55, 3.95, 9)) > 10.0
    for r in (r_on, r_c):       # slope and curvature vanish on both sides
        for s in (-1e-5, 1e-5):
            assert abs(dt(r + s)) < 1e-7 and abs(d2t(r + s)) < 1e-2


def test_forces_are_minus_gradient_of_shadow_potential():
    pos, sp = dimer(jitter=0.05)
    L = 9.0
    m = model.TBModel(**MD)
    ew = fo.Ewald(eta=0.7)
    n = np.random.default_rng(3).normal(scale=0.1, size=6)      # any n: U(R, n) is defined off the SCF point
    subs = fo.whole(6)
    F = fo.shadow_point(pos, sp, L, m, subs, n, ew).F
    h = 1e-5
    Ffd = np.zeros_like(F)
    for i in range(6):
        for c in range(3):
            p = pos.copy()
            p[i, c] += h
            ep = fo.shadow_point(p, sp, L, m, subs, n, ew, forces=False).U
            p[i, c] -= 2 * h
            em = fo.shadow_point(p, sp, L, m, subs, n, ew, forces=False).U
            Ffd[i, c] = -(ep - em) / (2 * h)
    assert np.abs(F).max() > 0.1
    np.testing.assert_allclose(F, Ffd, rtol=0, atol=1e-6)


@pytest.fixture(scope="module")
def box24():
    return waterbox.water_box(24, 21)


def test_partitioned_forces_sum_to_zero_and_full_halo_is_exact(box24):
    b = box24
    L = float(b.box[0])
    m = model.TBModel(**MD)
    ew = fo.Ewald(eta=5.6 / L)
    rp, col = model.neighbour_list(b.pos, L, m.cutoff)
    core, nco = graph.grid_cores(b.pos, b.anchor, L, (2, 2, 1))
    subs = graph.extract_subgraphs(rp, col, core, nco)
    n = np.random.default_rng(4).normal(scale=0.05, size=len(b.species))
    part = fo.shadow_point(b.pos, b.species, L, m, subs, n, ew)
    assert np.abs(part.F.sum(axis=0)).max() < 1e-9
    # every atom in every subgraph: the collected solve is the full solve
    N = len(b.species)
    full_halo = []
    for atoms, nc in subs:
        core_atoms = np.sort(atoms[:nc])
        rest = np.setdiff1d(np.arange(N), core_atoms)
        full_halo.append((np.concatenate([core_atoms, rest]), nc))
    a = fo.shadow_point(b.pos, b.species, L, m, full_halo, n, ew)
    w = fo.shadow_point(b.pos, b.species, L, m, fo.whole(N), n, ew)
    np.testing.assert_allclose(a.F, w.F, rtol=0, atol=1e-9)
    assert abs(a.U - w.U) < 1e-9


def test_shadow_error_is_quadratic_in_charge_error():
    pos, sp = dimer()
    L = 10.0
    m = model.TBModel(**MD)
    ew = fo.Ewald(eta=5.6 / L)
    subs = fo.whole(6)
    q = converged(pos, sp, L, m, ew, subs)
    e_scc = fo.shadow_point(pos, sp, L, m, subs, q, ew, forces=False).U
    delta = np.random.default_rng(7).normal(size=6)
    delta -= delta.mean()
    errs = [fo.shadow_point(pos, sp, L, m, subs, q + eps * delta, ew, forces=False).U - e_scc
            for eps in (2e-2, 1e-2, 5e-3)]
    assert abs(errs[0] / errs[1] - 4.0) < 0.1 and abs(errs[1] / errs[2] - 4.0) < 0.05


def test_repulsion_gives_water_equilibrium():
    L = 30.0
    pos = WATER + 15.0
    sp = np.array([0, 1, 1])
    m = model.TBModel(**MD)
    ew = fo.Ewald(eta=5.6 / L)
    subs = fo.whole(3)
    q = converged(pos, sp, L, m, ew, subs)
    F = fo.shadow_point(pos, sp, L, m, subs, q, ew).F
    assert np.abs(F).max() < 5e-3
    # without the repulsion the hydrogens are pulled in hard
    F0 = fo.shadow_point(pos, sp, L, model.TBModel(taper_on=3.5), subs, q, ew).F
    assert np.abs(F0).max() > 5.0


def test_dissipation_coefficients():
    k = np.arange(6)
    assert xlbomd.C_DISS.sum() == 0.0 and (k * xlbomd.C_DISS).sum() == 0.0
    # a linear history and q = n continue the line exactly
    hist = [np.array([1.0 - 0.1 * j, 2.0 + 0.3 * j]) for j in range(6)]
    nxt = xlbomd.next_charges(hist, hist[0], 0.3)
    np.testing.assert_allclose(nxt, [1.1, 1.7], rtol=0, atol=1e-14)


def test_xlbomd_energy_fluctuation_grows_fourfold_per_dt_doubling():
    pos, sp = dimer()
    L = 10.0
    m = model.TBModel(**MD)
    ew = fo.Ewald(eta=5.6 / L)
    subs = lambda R: fo.whole(6)
    q = converged(pos, sp, L, m, ew, subs(pos))
    rng = np.random.default_rng(5)
    mass = xlbomd.MASS[sp]
    v = rng.normal(size=(6, 3)) * np.sqrt(2 * 0.025852 / (mass[:, None] * xlbomd.KE_EV))
    v -= (mass[:, None] * v).sum(axis=0) / mass.sum()
    amp = []
    for dt in (0.5, 0.25, 0.125):
        tr = xlbomd.run(pos, v, sp, L, m, subs, q, ew, dt, int(round(8.0 / dt)), c=0.3)
        e = np.array(tr.e_tot)
        amp.append(e.max() - e.min())
        assert max(tr.rms_qn) < 1e-2
    assert 3.5 < amp[0] / amp[1] < 4.5 and 3.5 < amp[1] / amp[2] < 4.5
