"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible mistake in the oracle (a dropped
term, a wrong sign or index, a transposed operand) fails at least one:

* neighbour list: brute force == periodic k-d tree (library routine);
* H, S symmetric, S positive definite; one water == generalized eigensolve;
* 2x2 dimer: mu = eps by particle-hole symmetry, D in closed form;
* full-halo subgraphs == full-system diagonalisation (Eq. 1 with the
  all-to-all graph, Determining the Subgraphs: the all-to-all graph is exact);
* 2 Tr[D S] = N_e and sum q = 0 at the bisected mu (Tr[D] = N_occ);
* D Hermitian and idempotent (D S D = D) as kT -> 0;
* D independent of the choice of Z (s^-1/2 vs Cholesky);
* recursive FOE in exact arithmetic == closed form, and -> Fermi as n_d grows;
* Ewald: rock-salt Madelung constant, independence of eta;
* graph rules on hand-built matrices; cores/halos by brute force;
* charge error vs tau decreases (Accuracy Control section: power law).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.spatial import cKDTree

import waterbox
from oracle import ewald, foe, graph, model, solve


@pytest.fixture(scope="module")
def box96():
    return waterbox.water_box(96, 1)


@pytest.fixture(scope="module")
def box16():
    return waterbox.water_box(16, 11)


def test_generator_deterministic():
    a = waterbox.water_box(50, 7)
    b = waterbox.water_box(50, 7)
    assert np.array_equal(a.pos, b.pos)
    L = a.box[0]
    assert abs(L - (150 / 0.1) ** (1 / 3)) < 1e-12
    assert a.pos.min() >= 0 and a.pos.max() < L
    # rigid geometry: O-H 0.96, H-O-H 104.5 deg
    mol = a.pos.reshape(-1, 3, 3)
    d1 = mol[:, 1] - mol[:, 0]
    d2 = mol[:, 2] - mol[:, 0]
    d1 -= L * np.rint(d1 / L)
    d2 -= L * np.rint(d2 / L)
    assert np.allclose(np.linalg.norm(d1, axis=1), 0.96, atol=1e-12)
    cosang = (d1 * d2).sum(1) / (0.96 * 0.96)
    assert np.allclose(np.degrees(np.arccos(cosang)), 104.5, atol=1e-9)


def test_neighbour_list_vs_kdtree(box96):
    L = box96.box[0]
    rp, col = model.neighbour_list(box96.pos, L, chunk=37)
    tree = cKDTree(box96.pos, boxsize=L)
    pairs = tree.query_pairs(4.0, output_type="ndarray")
    ref = set(map(tuple, pairs)) | set((j, i) for i, j in pairs)
    rows = np.repeat(np.arange(box96.n_atoms), np.diff(rp))
    got = set(zip(rows.tolist(), col.tolist()))
    # the k-d tree uses <= r; the oracle uses strict <; no pair sits at 4.0 exactly here
    assert got == ref
    for i in range(box96.n_atoms):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and i not in c


def test_hs_symmetric_spd(box96):
    m = model.TBModel(orthogonal=False)
    h, s = model.dense_hs(box96.pos, box96.species, box96.box[0], m)
    assert np.array_equal(h, h.T) and np.array_equal(s, s.T)
    assert np.linalg.eigvalsh(s)[0] > 0.4


def test_hs_slater_koster_by_hand():
    # one O at origin, one H along direction u at r = 1.2 A: check every element by hand
    m = model.TBModel(orthogonal=False)
    L = 30.0
    u = np.array([0.48, 0.6, 0.64])
    u /= np.linalg.norm(u)
    pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0] + 1.2 * u])
    sp = np.array([0, 1], dtype=np.int32)
    h, s = model.dense_hs(pos, sp, L, m)
    V = -4.0 * math.exp(-(1.2 - 1.0) / 0.5)
    S = 0.3 * math.exp(-(1.2 - 1.0) / 0.6)
    # orbitals: O s, px, py, pz, H s
    assert np.allclose(np.diag(h), [-23.9, -9.0, -9.0, -9.0, -6.4])
    assert abs(h[0, 4] - V) < 1e-14                       # s_O - s_H
    for a in range(3):                                   # p_O^a - s_H : -u_a V (u from O to H)
        assert abs(h[1 + a, 4] + u[a] * V) < 1e-14
        assert abs(s[1 + a, 4] + u[a] * S) < 1e-14
        assert abs(h[4, 1 + a] - h[1 + a, 4]) == 0.0
    assert np.all(h[0, 1:4] == 0) and np.all(h[1:4, 1:4] == np.diag([-9.0] * 3))


def test_single_water_textbook():
    m = model.TBModel(orthogonal=False)
    pos, sp, L = model.single_water_reference(m)
    h, s = model.dense_hs(pos, sp, L, m)
    assert h.shape == (6, 6)
    ref_lam = sla.eigh(h, s, eigvals_only=True)               # LAPACK generalized solver
    sol = solve.solve_subgraph(h, s, 6)
    assert np.max(np.abs(sol.lam - ref_lam)) < 1e-13
    # full density matrix from the generalized eigenvectors
    lam, C = sla.eigh(h, s)
    mu = solve.find_mu([sol], 8.0, m.beta)
    Dref = (C * solve.fermi(lam - mu, m.beta)) @ C.T
    assert np.max(np.abs(solve.d_core_rows(sol, mu, m.beta) - Dref)) < 1e-13


def test_dimer_closed_form():
    eps, t, beta = -5.0, -1.3, 7.0
    h = np.array([[eps, t], [t, eps]])
    sol = solve.solve_subgraph(h, None, 2)
    mu = solve.find_mu([sol], 2.0, beta)
    assert abs(mu - eps) < 1e-11
    D = solve.d_core_rows(sol, mu, beta)
    th = math.tanh(beta * t / 2)
    Dref = 0.5 * np.array([[1.0, -th], [-th, 1.0]])
    assert np.max(np.abs(D - Dref)) < 1e-14 + abs(beta) * 1e-12


def test_fermi_stable():
    x = np.array([-1e4, -1.0, 0.0, 1.0, 1e4])
    f = solve.fermi(x, 10.0)
    assert np.all(np.isfinite(f))
    assert f[0] == 1.0 and f[-1] == 0.0 and f[2] == 0.5
    assert abs(f[1] + f[3] - 1.0) < 1e-15


@pytest.mark.parametrize("orthogonal", [True, False])
def test_full_halo_equals_full_system(box16, orthogonal):
    m = model.TBModel(orthogonal=orthogonal)
    L = box16.box[0]
    full = solve.full_system(box16.pos, box16.species, L, m)
    rp, col = graph.all_to_all(box16.n_atoms)
    core, nco = graph.grid_cores(box16.pos, box16.anchor, L, (2, 1, 2))
    subs = graph.extract_subgraphs(rp, col, core, nco)
    assert all(len(a) == box16.n_atoms for a, _ in subs)
    res = solve.solve_system(box16.pos, box16.species, L, m, subs, workers=1)
    assert np.max(np.abs(res.q - full.q)) < 1e-10
    _, aoo, _ = model.orbital_layout(box16.species)
    orb_ptr = model.orbital_layout(box16.species)[0]
    Dfull = full.d_core[0]
    for (atoms, ncore), Dc in zip(subs, res.d_core):
        orbs = graph.subgraph_orbitals(atoms, box16.species, orb_ptr)
        nco_orb = int(model.N_ORB[box16.species[atoms[:ncore]]].sum())
        assert np.max(np.abs(Dc - Dfull[np.ix_(orbs[:nco_orb], orbs)])) < 1e-10


def test_trace_and_neutrality(box96):
    m = model.TBModel(orthogonal=False)
    L = box96.box[0]
    rp, col = model.neighbour_list(box96.pos, L)
    core, nco = graph.grid_cores(box96.pos, box96.anchor, L, (2, 2, 2))
    subs = graph.extract_subgraphs(rp, col, core, nco)
    res = solve.solve_system(box96.pos, box96.species, L, m, subs)
    n_e = model.n_electrons(box96.species)
    assert n_e == 768.0
    assert abs(res.n_count - n_e) < 1e-9
    assert abs(res.q.sum()) < 1e-9
    # electron count from the collected D: 2 sum_core (D s)_aa
    tot = sum(2.0 * np.einsum("ab,ab->", d, s.s_core) for d, s in zip(res.d_core, res.sols))
    assert abs(tot - n_e) < 1e-9


def test_hermitian_idempotent_low_kT(box16):
    L = box16.box[0]
    for orthogonal in (True, False):
        m = model.TBModel(orthogonal=orthogonal, kT=1e-3)
        full = solve.full_system(box16.pos, box16.species, L, m)
        D = full.d_core[0]
        assert np.max(np.abs(D - D.T)) < 1e-13
        if orthogonal:
            err = np.max(np.abs(D @ D - D))
        else:
            _, s = model.dense_hs(box16.pos, box16.species, L, m)
            err = np.max(np.abs(D @ s @ D - D))
        assert err < 1e-8


def test_z_choice_invariance(box16):
    m = model.TBModel(orthogonal=False)
    L = box16.box[0]
    rp, col = model.neighbour_list(box16.pos, L)
    core, nco = graph.grid_cores(box16.pos, box16.anchor, L, (2, 2, 1))
    subs = graph.extract_subgraphs(rp, col, core, nco)
    a = solve.solve_system(box16.pos, box16.species, L, m, subs, workers=1, z="invsqrt")
    b = solve.solve_system(box16.pos, box16.species, L, m, subs, workers=1, z="cholesky")
    assert max(np.max(np.abs(x - y)) for x, y in zip(a.d_core, b.d_core)) < 1e-12
    assert np.max(np.abs(a.q - b.q)) < 1e-12


def test_foe_recursion_closed_form(box16):
    m = model.TBModel(orthogonal=False)
    L = box16.box[0]
    h, s = model.dense_hs(box16.pos, box16.species, L, m)
    Z = solve.inv_sqrt_spd(s)
    hp = Z @ h @ Z
    full = solve.full_system(box16.pos, box16.species, L, m)
    mu = full.mu
    lo, hi = foe.gershgorin(hp)
    nd = foe.n_doublings(m.beta, lo, hi, mu)
    assert 7 <= nd <= 10
    X = foe.foe_recursion(hp, mu, m.beta, nd)
    Xc = foe.foe_closed_form(hp, mu, m.beta, nd)
    assert np.max(np.abs(X - Xc)) < 1e-12
    # truncation error vs the true Fermi function falls ~ b^2 (x16 per 2 doublings)
    F = foe.fermi_exact(hp, mu, m.beta)
    errs = [np.max(np.abs(foe.foe_closed_form(hp, mu, m.beta, k) - F)) for k in (nd, nd + 2, nd + 4)]
    assert errs[0] < 1e-8
    assert errs[1] < errs[0] / 8 and errs[2] < errs[1] / 8


def test_ewald_madelung_and_eta():
    for eta in (1.4, 2.2):
        assert abs(ewald.madelung_nacl(eta) - 1.747565) < 1e-6
    b = waterbox.water_box(8, 3)
    rng = np.random.default_rng(0)
    q = rng.normal(size=b.n_atoms)
    q -= q.mean()
    U = np.array([13.6057, 10.8846])
    L = b.box[0]
    for screened in (False, True):
        v1 = ewald.coulomb_potential(b.pos, b.species, q, L, U, eta=4.0 / L, n_real=2, k_max=6, screened=screened)
        v2 = ewald.coulomb_potential(b.pos, b.species, q, L, U, eta=6.0 / L, n_real=2, k_max=9, screened=screened)
        assert np.max(np.abs(v1 - v2)) < 1e-8
    # isolated pair limit: two opposite point charges at 1 A in a huge box ~ k_e / r
    pos = np.array([[50.0, 50, 50], [51.0, 50, 50]])
    qq = np.array([1.0, -1.0])
    v = ewald.coulomb_potential(pos, np.array([1, 1]), qq, 100.0, np.zeros(2), eta=0.06, n_real=1, k_max=8,
                                screened=False)
    assert abs(v[0] - (-14.399645 * 1.0)) < 2e-3


def _slater_gamma_quadrature(ta, tb, R):
    """Coulomb energy of two unit densities t^3/(8 pi) exp(-t r) at distance R,
    by nested quadrature: shell averages of the second density's potential
    1/s - exp(-tb s) (1/s + tb/2) over the first density."""
    from scipy import integrate

    def phi(s):          # 1/s - exp(-tb s)/s written without cancellation
        return -np.expm1(-tb * s) / s - 0.5 * tb * np.exp(-tb * s) if s > 1e-12 else tb / 2.0

    def shell(r):
        v, _ = integrate.quad(lambda s: s * phi(s), abs(r - R), r + R, limit=200)
        return v / (2.0 * r * R)

    v, _ = integrate.quad(lambda r: r * r * ta ** 3 / 2.0 * np.exp(-ta * r) * shell(r), 0.0, 60.0 / ta, limit=400,
                          points=[R])
    return v


def test_slater_screening_closed_form():
    """gamma = 1/R - S of the screened interaction against direct quadrature,
    gamma -> U at R -> 0, S -> 0 at large R, and the species symmetry."""
    tau = ewald.slater_tau([13.6057, 10.8846])
    for ta, tb in ((tau[0], tau[0]), (tau[0], tau[1]), (tau[1], tau[1])):
        for R in (0.3, 0.96, 2.5, 6.0):
            g = 1.0 / R - ewald.slater_short(ta, tb, R)
            assert abs(g - _slater_gamma_quadrature(ta, tb, R)) < 1e-9 * max(1.0, g)
        assert abs(ewald.slater_short(ta, tb, 0.96) - ewald.slater_short(tb, ta, 0.96)) < 1e-15
        assert ewald.slater_short(ta, tb, 15.0) < 1e-12
    # on-site limit: gamma(0) = 5 tau / 16 = U (atomic units), i.e. U / k_e in 1/A
    R = 1e-6
    assert abs((1.0 / R - ewald.slater_short(tau[0], tau[0], R)) * 14.399645 - 13.6057) < 1e-4


def test_grid_cores_and_halos_bruteforce(box96):
    L = box96.box[0]
    core, nco = graph.grid_cores(box96.pos, box96.anchor, L, (2, 3, 2))
    # brute force: every atom's cell from its anchor
    for i in range(box96.n_atoms):
        assert core[i] == core[box96.anchor[i]]
    assert nco <= 12 and core.max() == nco - 1
    rp, col = model.neighbour_list(box96.pos, L)
    subs = graph.extract_subgraphs(rp, col, core, nco)
    seen = np.zeros(box96.n_atoms, int)
    for c, (atoms, ncore) in enumerate(subs):
        cs = atoms[:ncore]
        assert np.all(core[cs] == c) and np.all(np.diff(cs) > 0)
        seen[cs] += 1
        halo = atoms[ncore:]
        assert np.all(np.diff(halo) > 0) and np.all(core[halo] != c)
        ref = set()
        for i in cs:
            ref |= set(col[rp[i]:rp[i + 1]].tolist())
        assert set(halo.tolist()) == ref - set(cs.tolist())
    assert np.all(seen == 1)


def test_graph_rules_hand_built():
    import scipy.sparse as sp
    # 3 atoms (O,H,H) -> orbitals 4,1,1; one subgraph with all atoms in the core
    species = np.array([0, 1, 1])
    subs = [(np.array([0, 1, 2]), 3)]
    D = np.zeros((6, 6))
    D[0, 4] = -3e-3      # O-H1 block max 3e-3
    D[2, 5] = 2e-6       # O-H2 block max 2e-6
    D[4, 5] = 5e-4       # H1-H2
    D = D + D.T
    D[np.arange(6), np.arange(6)] = 0.5
    gd = graph.condensed_dm(subs, [D], species, 3).toarray()
    assert gd[0, 1] == 3e-3 and gd[0, 2] == 2e-6 and gd[1, 2] == 5e-4 and gd[0, 0] == 0.5
    rp, col = graph.graph_dm(sp.csr_matrix(gd), 1e-5)
    assert list(col[rp[0]:rp[1]]) == [1] and list(col[rp[1]:rp[2]]) == [0, 2]
    # adaptive: (GN GD + GD GN)_IJ with GN = I -> 2 GD
    gn = sp.identity(3, format="csr")
    (rp2, col2), w = graph.graph_adaptive(gn, sp.csr_matrix(gd), 1.5e-6)
    assert set(col2[rp2[0]:rp2[1]]) == {1, 2}
    # a two-hop path: GN_01 = 0.5, GD_12 = 5e-4 -> (GN GD)_02 gains 2.5e-4
    gn2 = sp.csr_matrix(np.array([[1, 0.5, 0], [0.5, 1, 0], [0, 0, 1.0]]))
    gd2 = np.zeros((3, 3)); gd2[1, 2] = gd2[2, 1] = 5e-4
    (rp3, col3), w3 = graph.graph_adaptive(gn2, sp.csr_matrix(gd2), 2e-4)
    assert 2 in set(col3[rp3[0]:rp3[1]])


def test_tau_error_decreases(box96):
    # error of collected charges vs full diagonalisation shrinks with tau (power law)
    m = model.TBModel(orthogonal=False)
    L = box96.box[0]
    full = solve.full_system(box96.pos, box96.species, L, m)
    gd = graph.condensed_dm(full.subs, full.d_core, box96.species, box96.n_atoms)
    core, nco = graph.grid_cores(box96.pos, box96.anchor, L, (3, 3, 3))
    errs = []
    for tau in (1e-2, 1e-3, 1e-4):
        rp, col = graph.graph_dm(gd, tau)
        subs = graph.extract_subgraphs(rp, col, core, nco)
        res = solve.solve_system(box96.pos, box96.species, L, m, subs)
        errs.append(np.max(np.abs(res.q - full.q)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_kdtree_neighbour_list_equals_bruteforce():
    b = waterbox.water_box(400, 9)
    L = b.box[0]
    a = model.neighbour_list(b.pos, L)
    k = model.neighbour_list_kdtree(b.pos, L)
    assert np.array_equal(a[0], k[0]) and np.array_equal(a[1], k[1])


def test_distance_graph_by_hand():
    # G^N_IJ = exp(-alpha R_IJ^2) over neighbour pairs plus G^N_II = 1 (Eq.
    # neigh_mat).  Three atoms in a 20 A box; the 0-2 pair is 1.5 A apart only
    # through the periodic image along z.
    L = 20.0
    pos = np.array([[1.0, 1.0, 1.0], [2.5, 1.0, 1.0], [1.0, 1.0, 19.5]])
    rp, col = model.neighbour_list(pos, L)
    assert list(np.diff(rp)) == [2, 2, 2]
    g = graph.distance_graph(pos, L, rp, col, 0.7).toarray()
    r2 = np.array([[0.0, 2.25, 2.25], [2.25, 0.0, 4.5], [2.25, 4.5, 0.0]])   # by hand
    want = np.array([[1.0, math.exp(-1.575), math.exp(-1.575)],
                     [math.exp(-1.575), 1.0, math.exp(-3.15)],
                     [math.exp(-1.575), math.exp(-3.15), 1.0]])
    assert np.abs(g - want).max() < 1e-15
    # the plausible mistakes give other numbers: exp(-alpha R), no unit
    # diagonal, alpha applied to R^2 without the minus sign
    off = ~np.eye(3, dtype=bool)
    assert np.abs(g[off] - np.exp(-0.7 * np.sqrt(r2[off]))).min() > 0.1
    assert np.all(np.diag(g) == 1.0)
    assert np.abs(g[off] - np.exp(0.7 * r2[off])).min() > 1.0


def _oo_pair(u, r=2.5):
    pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0] + r * np.asarray(u)])
    return model.dense_hs(pos, np.array([0, 0], dtype=np.int32), 30.0, model.TBModel(orthogonal=False))


def test_hs_pp_block_by_hand():
    # O-O pair at 2.5 A along u = (2, -3, 6)/7: with V_pp_pi = 0 the p-p block
    # is u_a u_b V(r) (sigma only), the s-p blocks are +-u_b V with the
    # direction taken from the row atom, and S follows the same pattern.
    u = np.array([2.0, -3.0, 6.0]) / 7.0
    h, s = _oo_pair(u)
    V = -4.0 * math.exp(-3.0)          # -4 exp(-(2.5 - 1)/0.5)
    S = 0.3 * math.exp(-2.5)           # 0.3 exp(-(2.5 - 1)/0.6)
    uu = np.array([[4.0, -6.0, 12.0], [-6.0, 9.0, -18.0], [12.0, -18.0, 36.0]]) / 49.0   # u_a u_b by hand
    ux = np.array([2.0, -3.0, 6.0]) / 7.0
    for mat, f in ((h, V), (s, S)):
        blk = mat[0:4, 4:8]            # rows: atom 0 (s, px, py, pz), columns: atom 1
        assert abs(blk[0, 0] - f) < 1e-15
        assert np.abs(blk[0, 1:] - ux * f).max() < 1e-15        # [s_I, p_J^b] = u_b f
        assert np.abs(blk[1:, 0] + ux * f).max() < 1e-15        # [p_I^a, s_J] = -u_a f
        assert np.abs(blk[1:, 1:] - uu * f).max() < 1e-15       # [p_I^a, p_J^b] = u_a u_b f
        # the other atom sees -u: its s-p signs flip, its p-p block is the same
        rev = mat[4:8, 0:4]
        assert np.abs(rev[0, 1:] + ux * f).max() < 1e-15
        assert np.abs(rev[1:, 1:] - uu * f).max() < 1e-15
        # plausible mistakes are caught: a negative p-p sign, a pi term equal to
        # the sigma one (which would give f * I on the p-p block)
        assert np.abs(blk[1:, 1:] + uu * f).max() > 0.1 * abs(f)
        assert np.abs(blk[1:, 1:] - f * np.eye(3)).max() > 0.1 * abs(f)


def test_hs_rotation_invariance():
    # the spectrum of a pair does not depend on the direction of its axis: a
    # wrong sign or index in any Slater-Koster block breaks this
    rng = np.random.default_rng(7)
    ref = None
    for k in range(4):
        u = np.array([0.0, 0.0, 1.0]) if k == 0 else rng.normal(size=3)
        u /= np.linalg.norm(u)
        h, s = _oo_pair(u, r=2.2)
        lam = sla.eigh(h, s, eigvals_only=True)
        if ref is None:
            ref = lam
        assert np.abs(lam - ref).max() < 1e-12


def test_scc_shift_by_hand():
    # SCC shift (SI section D): H_ab += 1/2 S_ab (V_I + V_J); on site S = I
    # gives H_aa += V_I.  O at the origin, H at 1.2 A along u.
    m = model.TBModel(orthogonal=False)
    u = np.array([0.48, 0.6, 0.64])
    u /= np.linalg.norm(u)
    pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0] + 1.2 * u])
    sp_ = np.array([0, 1], dtype=np.int32)
    vO, vH = 0.7, -0.3
    h0, _ = model.dense_hs(pos, sp_, 30.0, m)
    h1, _ = model.dense_hs(pos, sp_, 30.0, m, V_atom=np.array([vO, vH]))
    dh = h1 - h0
    S = 0.3 * math.exp(-(1.2 - 1.0) / 0.6)
    want = np.zeros((5, 5))
    want[np.arange(4), np.arange(4)] = vO                 # O orbitals: 1/2 * 1 * (vO + vO)
    want[4, 4] = vH
    want[0, 4] = want[4, 0] = 0.5 * S * (vO + vH)         # s_O - s_H
    for a in range(3):                                    # p_O^a - s_H: S_ab = -u_a S
        want[1 + a, 4] = want[4, 1 + a] = -0.5 * u[a] * S * (vO + vH)
    assert np.abs(dh - want).max() < 1e-14
    # a missing 1/2 or a shift by V_I alone would be caught
    assert abs(dh[0, 4] - S * (vO + vH)) > 1e-3
    assert abs(dh[0, 4] - 0.5 * S * 2 * vO) > 1e-3
    # orthogonal model: only the diagonal moves, by V of the orbital's atom
    mo = model.TBModel(orthogonal=True)
    g0, _ = model.dense_hs(pos, sp_, 30.0, mo)
    g1, _ = model.dense_hs(pos, sp_, 30.0, mo, V_atom=np.array([vO, vH]))
    assert np.abs((g1 - g0) - np.diag([vO] * 4 + [vH])).max() < 1e-15


def test_scc_uniform_potential_shifts_spectrum(box16):
    # a uniform potential c on every atom adds c S to H, so every generalized
    # eigenvalue moves by exactly c (with the factor 1/2 wrong it would move by 2c)
    box = box16
    m = model.TBModel(orthogonal=False)
    c = 0.37
    h0, s0 = model.dense_hs(box.pos, box.species, box.box[0], m)
    h1, _ = model.dense_hs(box.pos, box.species, box.box[0], m, V_atom=np.full(box.n_atoms, c))
    l0 = sla.eigh(h0, s0, eigvals_only=True)
    l1 = sla.eigh(h1, s0, eigvals_only=True)
    assert np.abs(l1 - l0 - c).max() < 1e-11
