"""Pins of the oracle's learned-guess and SCC pieces.

* descriptors: a neighbour at a Gaussian centre gives exactly the cutoff
  weight there; neighbour species land in their own half; nothing at or
  beyond 5 A; invariance under rigid motion, permutation and periodic
  wrapping; the value vanishes smoothly at the cutoff;
* MLP: analytic gradients == central finite differences for every
  parameter class of both species networks; the prediction is neutral and
  blind to a uniform output shift;
* Adam: the first step moves every parameter by lr g / (|g| + eps) (the
  bias-corrected moments are g and g^2), and training a student network on
  a teacher of the same shape drives the loss down;
* SCC: the returned charges are a fixed point of the charge map to the
  tolerance, sum to zero, and do not depend on the start; Anderson
  acceleration reaches the closed-form fixed point of an affine map on
  which linear mixing diverges, and with memory 0 it is linear mixing.
"""
import math

import numpy as np
import pytest

import waterbox
from oracle import graph as og
from oracle import learned as ol
from oracle import model as om
from oracle import scc as osc


def fc(r):
    return 0.5 * (math.cos(math.pi * r / 5.0) + 1.0)


def test_descriptor_pair_by_construction():
    L = 30.0
    k = 5
    r = 0.8 + k * 3.2 / 15.0
    pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0 + r]])
    sp = np.array([0, 1])
    G = ol.descriptors(pos, sp, L)
    # the O atom sees one H: its O half is empty, the H half peaks at k
    assert np.all(G[0, :16] == 0.0)
    assert abs(G[0, 16 + k] - fc(r)) < 1e-15
    assert np.argmax(G[0, 16:]) == k
    # the H atom sees one O: mirror image in the other half
    assert np.all(G[1, 16:] == 0.0)
    assert np.array_equal(G[1, :16], G[0, 16:])
    # neighbouring centres are symmetric about r = c_k
    assert abs(G[0, 16 + k - 1] - G[0, 16 + k + 1]) < 1e-13
    # nothing at or beyond the cutoff, and a vanishing value just inside it
    for far in (5.0, 5.3):
        pos[1, 2] = 10.0 + far
        assert np.all(ol.descriptors(pos, sp, L) == 0.0)
    pos[1, 2] = 10.0 + 5.0 - 1e-4
    assert ol.descriptors(pos, sp, L).max() < 1e-8


def test_descriptor_invariances():
    box = waterbox.water_box(16, 11)
    L = box.box[0]
    G = ol.descriptors(box.pos, box.species, L)
    rng = np.random.default_rng(5)
    # periodic translation (wrapped) leaves every descriptor unchanged
    shift = rng.uniform(-L, L, size=3)
    G2 = ol.descriptors((box.pos + shift) % L, box.species, L)
    assert np.abs(G2 - G).max() < 1e-12
    # permuting atoms permutes rows
    perm = rng.permutation(len(box.species))
    G3 = ol.descriptors(box.pos[perm], box.species[perm], L)
    assert np.abs(G3 - G[perm]).max() < 1e-12
    # rigid rotation of an isolated cluster in a large box
    pos = box.pos.copy()
    d = pos - pos[0]
    d -= L * np.rint(d / L)
    pos = d + 20.0
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Ga = ol.descriptors(pos, box.species, 60.0)
    Gb = ol.descriptors((pos - 20.0) @ Q.T + 20.0, box.species, 60.0)
    assert np.abs(Ga - Gb).max() < 1e-11


def _problem(seed=3, n=40):
    rng = np.random.default_rng(seed)
    feats = rng.uniform(0.0, 3.0, size=(n, 32))
    species = rng.integers(0, 2, size=n)
    species[:2] = (0, 1)
    nets = waterbox.mlp_init(seed)
    for net in nets:                         # non-zero biases exercise every path
        for k in ("b1", "b2", "b3"):
            net[k] = rng.uniform(-0.3, 0.3, size=net[k].shape)
    stats = ol.standardise_stats(feats, species)
    q_ref = rng.normal(0.0, 0.5, size=n)
    q_ref -= q_ref.mean()
    return nets, stats, feats, species, q_ref


def test_mlp_gradients_match_finite_differences():
    nets, stats, feats, species, q_ref = _problem()
    loss, grads = ol.loss_and_grads(nets, stats, feats, species, q_ref)
    rng = np.random.default_rng(9)
    h = 1e-6
    for s in (0, 1):
        for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
            p = nets[s][name]
            flat = p.reshape(-1)
            picks = rng.choice(flat.size, size=min(6, flat.size), replace=False)
            for e in picks:
                old = flat[e]
                flat[e] = old + h
                lp, _ = ol.loss_and_grads(nets, stats, feats, species, q_ref)
                flat[e] = old - h
                lm, _ = ol.loss_and_grads(nets, stats, feats, species, q_ref)
                flat[e] = old
                fd = (lp - lm) / (2 * h)
                an = grads[s][name].reshape(-1)[e]
                assert abs(fd - an) <= 1e-7 + 1e-6 * abs(fd), (s, name, e, fd, an)


def test_prediction_neutral_and_shift_blind():
    nets, stats, feats, species, _ = _problem()
    q = ol.predict(nets, stats, feats, species)
    assert abs(q.sum()) < 1e-12
    for net in nets:
        net["b3"] = net["b3"] + 0.7
    assert np.abs(ol.predict(nets, stats, feats, species) - q).max() < 1e-12


def test_adam_first_step_closed_form():
    nets, stats, feats, species, q_ref = _problem()
    _, grads = ol.loss_and_grads(nets, stats, feats, species, q_ref)
    before = [{k: v.copy() for k, v in n.items()} for n in nets]
    opt = ol.Adam(nets, lr=1e-3)
    opt.step(nets, grads)
    for s in (0, 1):
        for k in nets[s]:
            g = grads[s][k]
            want = before[s][k] - 1e-3 * g / (np.abs(g) + 1e-8)
            assert np.abs(nets[s][k] - want).max() < 1e-15


def test_student_learns_teacher():
    rng = np.random.default_rng(1)
    n = 256
    feats = rng.uniform(0.0, 3.0, size=(n, 32))
    species = rng.integers(0, 2, size=n)
    stats = ol.standardise_stats(feats, species)
    teacher = waterbox.mlp_init(100)
    target = ol.predict(teacher, stats, feats, species)
    student = waterbox.mlp_init(200)
    opt = ol.Adam(student, lr=3e-3)
    first, _ = ol.loss_and_grads(student, stats, feats, species, target)
    for _ in range(300):
        loss, g = ol.loss_and_grads(student, stats, feats, species, target)
        opt.step(student, g)
    assert loss < first / 20


@pytest.mark.slow
def test_scc_fixed_point_independent_of_start():
    box = waterbox.water_box(32, 11)
    L = box.box[0]
    m = om.TBModel()
    rp, col = om.neighbour_list(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, (2, 2, 1))
    subs = og.extract_subgraphs(rp, col, core, nco)
    q, it, hist = osc.scc(box.pos, box.species, L, m, subs)
    assert it < 60 and hist[-1] < 1e-5
    assert abs(q.sum()) < 1e-9
    # the screened interaction gives water-like polarity: O gains electrons, H loses them
    assert np.all(q[box.species == 0] > 0.3) and np.all(q[box.species == 1] < -0.1)
    # one more application of the charge map stays at the fixed point: q = q0[n] with
    # RMS(q0[n] - n) < 1e-5 e, so q0[q] - q ~ J (q0[n] - n), J the (strong) charge response
    from oracle.ewald import coulomb_potential
    from oracle.solve import solve_system
    V = coulomb_potential(box.pos, box.species, q, L, np.asarray(m.hubbard_U))
    q1 = solve_system(box.pos, box.species, L, m, subs, V_atom=V).q
    assert math.sqrt(np.mean((q1 - q) ** 2)) < 1e-4
    # a different start reaches the same charges
    start = q + 0.01 * np.random.default_rng(0).standard_normal(len(q))
    q2, it2, _ = osc.scc(box.pos, box.species, L, m, subs, q_start=start)
    assert it2 < it
    # both stop at an RMS residual below 1e-5 e, so they agree at that level
    assert math.sqrt(np.mean((q2 - q) ** 2)) < 1e-5 and np.abs(q2 - q).max() < 5e-5


def test_anderson_on_affine_map():
    rng = np.random.default_rng(0)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * -np.linspace(0.1, 8.0, n)) @ Q.T          # response eigenvalues down to -8
    b = rng.standard_normal(n)
    x = np.linalg.solve(np.eye(n) - A, b)
    G = lambda v: A @ v + b
    q, it, hist, ok = osc.fixed_point(G, np.zeros(n), mix=0.3, tol=1e-10, mixer="anderson", depth=5)
    assert ok and np.abs(q - x).max() < 1e-9
    # linear mixing at c = 0.3 diverges here (|1 - 0.3 (1 + 8)| > 1)
    _, _, hist_lin, ok_lin = osc.fixed_point(G, np.zeros(n), mix=0.3, tol=1e-10, max_iter=60)
    assert not ok_lin and hist_lin[-1] > hist_lin[0]
    # memory 0 is the linear update, step for step
    h0 = osc.fixed_point(G, np.zeros(n), mix=0.05, tol=1e-10, max_iter=30, mixer="anderson", depth=0)[2]
    h1 = osc.fixed_point(G, np.zeros(n), mix=0.05, tol=1e-10, max_iter=30)[2]
    assert h0 == h1
