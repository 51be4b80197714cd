"""Pins of the oracle's charge response and kernel-accelerated SCF.

* the canonical response equals central finite differences of the full
  solve (new mu found by bisection at each displaced potential), for the
  orthogonal and the non-orthogonal model;
* on one subgraph holding the whole system the static susceptibility
  dq_I / dV_J is symmetric (second derivative of the grand potential);
* the response keeps the electron count (sum dq = 0) and is linear in dV;
* on an affine charge map the full-rank low-rank kernel is the exact
  inverse Jacobian: one quasi-Newton step lands on the closed-form fixed
  point, and the rank-m step equals the GMRES-type minimiser over the
  Krylov space built from explicit powers of J; the completed step adds
  k0 (f + J dn); with a Jacobian model wrong by 4x the full steps diverge
  and the backtracking line search restores a decreasing residual;
* on a water box the quasi-Newton SCF reaches the Anderson fixed point.
"""
import math

import numpy as np
import pytest

import waterbox
from oracle import graph as og
from oracle import model as om
from oracle import response as orsp
from oracle import scc as osc
from oracle import solve as osv


def small_system(orthogonal, nw=24, seed=21, grid=(2, 2, 1)):
    box = waterbox.water_box(nw, seed)
    L = box.box[0]
    m = om.TBModel(orthogonal=orthogonal)
    rp, col = om.neighbour_list(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, grid)
    subs = og.extract_subgraphs(rp, col, core, nco)
    return box, L, m, subs


@pytest.mark.parametrize("orthogonal", [False, True])
def test_response_matches_finite_differences(orthogonal):
    box, L, m, subs = small_system(orthogonal)
    rng = np.random.default_rng(5)
    n = len(box.species)
    V = 0.5 * rng.standard_normal(n)
    dV = rng.standard_normal(n)
    dq, dmu, mu = orsp.charge_response(box.pos, box.species, L, m, subs, V, dV)
    h = 1e-4
    qp = osv.solve_system(box.pos, box.species, L, m, subs, V_atom=V + h * dV, workers=1).q
    qm = osv.solve_system(box.pos, box.species, L, m, subs, V_atom=V - h * dV, workers=1).q
    fd = (qp - qm) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 1e-2                                   # a real response, not a vanishing one
    assert np.abs(dq - fd).max() < 1e-6 * max(1.0, scale)
    assert abs(dq.sum()) < 1e-12 * n
    # linear in dV
    dq2, _, _ = orsp.charge_response(box.pos, box.species, L, m, subs, V, -3.0 * dV)
    assert np.abs(dq2 + 3.0 * dq).max() < 1e-12 * max(1.0, scale)


def test_full_system_susceptibility_symmetric():
    box, L, m, _ = small_system(False, nw=24, seed=22)
    n = len(box.species)
    subs = [(np.arange(n, dtype=np.int64), n)]
    V = np.zeros(n)
    J = [0, 1, 5, 12, 40, 71]
    chi = np.zeros((len(J), len(J)))
    res = osv.solve_system(box.pos, box.species, L, m, subs, V_atom=V, workers=1)
    for b, j in enumerate(J):
        e = np.zeros(n)
        e[j] = 1.0
        dq, _, _ = orsp.charge_response(box.pos, box.species, L, m, subs, V, e, mu=res.mu, sols=res.sols)
        chi[:, b] = dq[J]
    assert np.abs(chi).max() > 1e-2
    assert np.abs(chi - chi.T).max() < 1e-10
    # a potential raised on an atom pushes electrons off it
    assert np.all(np.diag(chi) < 0)


def test_occupation_difference_limits():
    beta = 10.0
    lam = np.array([-1.0, -1.0 + 1e-12, 0.3, 2.0])
    f = osv.fermi(lam, beta)
    F = orsp.occupation_differences(lam, f, beta)
    # coincident eigenvalues take the derivative of f
    assert abs(F[0, 1] + beta * f[0] * (1 - f[0])) < 1e-12
    # separated ones the divided difference
    assert abs(F[2, 3] - (f[2] - f[3]) / (lam[2] - lam[3])) < 1e-15
    assert np.allclose(F, F.T, rtol=0, atol=1e-15)


def affine_problem(n=30, seed=0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * -np.linspace(0.1, 30.0, n)) @ Q.T
    A += 0.05 * rng.standard_normal((n, n))              # not symmetric
    b = rng.standard_normal(n)
    return A, b


def test_full_rank_kernel_is_newton():
    A, b = affine_problem()
    n = len(b)
    x = np.linalg.solve(np.eye(n) - A, b)
    G = lambda v: A @ v + b
    Jv = lambda _n, v: A @ v - v
    q, it, hist, ranks, ok = orsp.quasi_newton(G, Jv, np.zeros(n), tol=1e-10, rank_tol=1e-13, max_rank=n)
    assert ok and it == 2 and np.abs(q - x).max() < 1e-9
    # one step is -J^-1 f
    f = G(np.zeros(n))
    dn, rank, rel = orsp.krylov_step(f, lambda v: A @ v - v, rank_tol=1e-13, max_rank=n)
    assert np.abs(dn + np.linalg.solve(A - np.eye(n), f)).max() < 1e-9


def test_low_rank_step_is_krylov_minimiser():
    A, b = affine_problem(seed=1)
    n = len(b)
    Jm = A - np.eye(n)
    f = A @ np.ones(n) + b - np.ones(n)
    for m in (1, 2, 4):
        dn, rank, rel = orsp.krylov_step(f, lambda v: Jm @ v, rank_tol=0.0, max_rank=m)
        assert rank == m
        # reference: minimise || J dn + f || over dn in span{f, J f, ..., J^(m-1) f}
        # (K0 = -I: the Krylov space of K0 J on K0 f is that of J on f)
        K = np.stack([np.linalg.matrix_power(Jm, k) @ f for k in range(m)], axis=1)
        y, *_ = np.linalg.lstsq(Jm @ K, -f, rcond=None)
        ref = K @ y
        assert np.abs(dn - ref).max() < 1e-8 * np.abs(ref).max()
        assert abs(rel - np.linalg.norm(Jm @ ref + f) / np.linalg.norm(f)) < 1e-8
        # the completed step adds the unfitted remainder -(r - F_v c), which with
        # r = -k0 f and F_v c = k0 J dn is k0 (f + J dn); it does not depend on k0's
        # Krylov space (the space of K0 J on K0 f is that of J on f for any k0)
        for k0 in (1.0, 0.1):
            dc, rank_c, rel_c = orsp.krylov_step(f, lambda v: Jm @ v, rank_tol=0.0, max_rank=m, k0=k0,
                                                 complete=True)
            assert rank_c == m and abs(rel_c - rel) < 1e-10
            assert np.abs(dc - (ref + k0 * (f + Jm @ ref))).max() < 1e-8 * np.abs(ref).max()


def test_backtracking_halves_a_bad_step():
    # a map whose Jacobian model is wrong by a factor 4 (the "response" passed
    # in is J/4): the full step overshoots, and halving recovers monotone
    # decrease of the residual
    A, b = affine_problem(n=20, seed=2)
    n = len(b)
    G = lambda v: A @ v + b
    wrong = lambda _n, v: 0.25 * (A @ v - v)
    _, _, hist0, _, ok0 = orsp.quasi_newton(G, wrong, np.zeros(n), tol=1e-10, max_iter=30, rank_tol=1e-13,
                                            max_rank=n, backtrack=0)
    _, _, hist4, _, ok4 = orsp.quasi_newton(G, wrong, np.zeros(n), tol=1e-10, max_iter=60, rank_tol=1e-13,
                                            max_rank=n, backtrack=4)
    assert not ok0 and hist0[-1] > hist0[0]
    assert ok4 and all(b_ < a_ for a_, b_ in zip(hist4, hist4[1:]))


@pytest.mark.slow
def test_quasi_newton_scc_reaches_anderson_fixed_point():
    box = waterbox.water_box(32, 11)
    L = box.box[0]
    m = om.TBModel()
    rp, col = om.neighbour_list(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, (2, 2, 1))
    subs = og.extract_subgraphs(rp, col, core, nco)
    q_a, it_a, _ = osc.scc(box.pos, box.species, L, m, subs)
    q_n, it_n, hist, ranks = orsp.scc_quasi_newton(box.pos, box.species, L, m, subs)
    assert hist[-1] < 1e-5
    assert it_n < it_a / 3
    assert math.sqrt(np.mean((q_n - q_a) ** 2)) < 1e-5 and np.abs(q_n - q_a).max() < 5e-5


def test_block_preconditioner_is_inverse_jacobian_for_one_core():
    """With one core holding every atom, every atom probed alone and the
    periodic kernel, the block-diagonal preconditioner is J^-1 itself
    (J v = dq[gamma v] - v from the canonical response)."""
    th = np.radians(52.25)
    w = np.array([[0.0, 0.0, 0.0], [0.96 * np.sin(th), 0.0, 0.96 * np.cos(th)],
                  [-0.96 * np.sin(th), 0.0, 0.96 * np.cos(th)]])
    pos = np.concatenate([w + [1.0, 1.0, 1.0], w + [4.0, 1.5, 1.2], w + [1.3, 4.2, 1.0], w + [3.8, 4.0, 3.9]])
    sp = np.array([0, 1, 1] * 4)
    L, eta = 10.0, 0.56
    m = om.TBModel()
    N = len(sp)
    subs = [(np.arange(N), N)]
    U = np.asarray(m.hubbard_U)
    V = orsp.coulomb_potential(pos, sp, np.random.default_rng(0).normal(scale=0.1, size=N), L, U, eta=eta)
    res = osv.solve_system(pos, sp, L, m, subs, V_atom=V)
    P = orsp.block_preconditioner(pos, sp, L, m, subs, V, res.mu, res.sols, gamma="ewald", eta=eta)
    J = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        dq, _, _ = orsp.charge_response(pos, sp, L, m, subs, V, orsp.coulomb_potential(pos, sp, e, L, U, eta=eta),
                                        mu=res.mu, sols=res.sols)
        J[:, j] = dq - e
    np.testing.assert_allclose(P.blocks[0] @ J, np.eye(N), rtol=0, atol=1e-10)
    x = np.random.default_rng(1).normal(size=N)
    np.testing.assert_allclose(P.apply(x), P.blocks[0] @ x, rtol=0, atol=1e-14)
