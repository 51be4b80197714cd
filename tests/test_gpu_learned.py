"""GPU parity of the SCC shell and the learned starting charges.

* Ewald potential vs the oracle's (and the rock-salt Madelung constant);
* linear mixing step;
* the whole SCC loop on the FP64 path vs the oracle's loop: same iteration
  count, same charges;
* descriptors (FP64) vs the oracle, feature normalisation;
* MLP forward in FP32 (to rounding) and BF16 (within a first-order bound
  derived from the bfloat16 unit roundoff), loss and FP32 gradients vs the
  FP64 oracle (1e-4 relative per parameter class), Adam steps;
* the trained network saves SCC iterations over the zero start and leads
  to the same converged charges.
"""
import math

import numpy as np
import pytest
import torch

import waterbox
from oracle import ewald as oew
from oracle import graph as og
from oracle import learned as ol
from oracle import model as om
from oracle import scc as osc
from tests.gpu_common import ctx, log, system_of, tb_params

pytestmark = pytest.mark.gpu

U_EV = (0.5 * 27.211386, 0.4 * 27.211386)


@pytest.fixture(scope="module")
def c():
    return ctx()


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


# ------------------------------------------------------------------ Ewald
@pytest.mark.parametrize("nw,seed", [(32, 11), (96, 1)])
def test_ewald_matches_oracle(c, nw, seed):
    from paper_2606_03140_amd import scc
    log(f"ewald {nw} waters")
    box = waterbox.water_box(nw, seed)
    L = box.box[0]
    sysm = system_of(box)
    q = np.random.default_rng(seed).normal(0.0, 1.0, size=len(box.species))
    q -= q.mean()
    ew = scc.ewald_setup(c, sysm)
    tau = scc.slater_tau(U_EV)
    for screened in (False, True):
        ref = oew.coulomb_potential(box.pos, box.species, q, L, np.array(U_EV), screened=screened,
                                    short_cut=ew.rcut)
        V = c.ewald_potential(sysm, ew.graph, ew.rcut, ew.eta, ew.k_max, U_EV, _dev(q),
                              tau=tau if screened else None).cpu().numpy()
        err = np.abs(V - ref).max()
        log(f"  screened={screened} rcut {ew.rcut:.3f} eta {ew.eta:.4f} k_max {ew.k_max} max|dV| {err:.2e} eV "
            f"(max|V| {np.abs(ref).max():.1f})")
        assert err < 1e-8
    # a different split (smaller real-space cutoff) gives the same point-charge potential
    ref = oew.coulomb_potential(box.pos, box.species, q, L, np.array(U_EV), screened=False)
    ew2 = scc.ewald_setup(c, sysm, rcut_max=0.3 * L)
    V2 = c.ewald_potential(sysm, ew2.graph, ew2.rcut, ew2.eta, ew2.k_max, U_EV, _dev(q)).cpu().numpy()
    assert np.abs(V2 - ref).max() < 1e-8


def test_ewald_madelung_rock_salt(c):
    from paper_2606_03140_amd import scc
    from paper_2606_03140_amd._lib import System
    idx = np.array([(a, b, d) for a in range(4) for b in range(4) for d in range(4)], dtype=np.float64)
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    sysm = System(idx + 0.0, np.zeros(len(q), dtype=np.int32), np.arange(len(q), dtype=np.int32), (4.0, 4.0, 4.0))
    ew = scc.ewald_setup(c, sysm)
    V = c.ewald_potential(sysm, ew.graph, ew.rcut, ew.eta, ew.k_max, (0.0, 0.0), _dev(q)).cpu().numpy()
    M = -V * q / 14.399645          # potential at a site of charge q is -M q / r0, r0 = 1
    log(f"  Madelung {M.min():.9f} .. {M.max():.9f}")
    assert np.abs(M - 1.747565).max() < 1e-6


def test_scc_mix(c):
    rng = np.random.default_rng(2)
    n0 = rng.normal(size=1000)
    q0 = rng.normal(size=1000)
    n = _dev(n0)
    rms = c.scc_mix(n, _dev(q0), 0.3)
    assert abs(rms - math.sqrt(np.mean((q0 - n0) ** 2))) < 1e-14
    assert np.abs(n.cpu().numpy() - (n0 + 0.3 * (q0 - n0))).max() < 1e-15


def test_anderson_matches_oracle_on_affine_map(c):
    """Same iterates as the oracle's Anderson step on G(n) = A n + b."""
    rng = np.random.default_rng(0)
    n = 300
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * -np.linspace(0.1, 8.0, n)) @ Q.T
    b = rng.standard_normal(n)
    x = _dev(np.zeros(n))
    work = torch.empty((3 * 5 + 2) * n, dtype=torch.float64, device="cuda")
    nh, fh, xr = [], [], np.zeros(n)
    for k in range(25):
        xg = x.cpu().numpy()
        c.scc_anderson(x, _dev(A @ xg + b), 0.3, 5, k, work)
        f = A @ xr + b - xr
        nh, fh = (nh + [xr])[-6:], (fh + [f])[-6:]
        xr = osc.anderson_step(nh, fh, 0.3, 5)
        assert np.abs(x.cpu().numpy() - xr).max() < 1e-9 * max(1.0, np.abs(xr).max()), k
    xs = np.linalg.solve(np.eye(n) - A, b)
    log(f"  Anderson on affine map: distance to fixed point after 25 steps {np.abs(xr - xs).max():.2e}")


@pytest.mark.parametrize("mixer", ["linear", "anderson"])
def test_scc_loop_matches_oracle(c, mixer):
    from paper_2606_03140_amd import pipeline, scc
    log(f"SCC loop, 32 waters, FP64 path vs oracle, {mixer} mixing")
    box = waterbox.water_box(32, 11)
    L = box.box[0]
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 1))
    ew = scc.ewald_setup(c, sysm)
    mix = 0.1
    res = scc.scc_loop(c, sysm, tb, part, 0.1, pipeline.FP64_EIG, ewald=ew, mixer=mixer, mix=mix)
    rp, col = om.neighbour_list(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, (2, 2, 1))
    subs = og.extract_subgraphs(rp, col, core, nco)
    q_ref, it_ref, hist_ref = osc.scc(box.pos, box.species, L, om.TBModel(), subs, mixer=mixer, mix=mix,
                                      short_cut=ew.rcut)
    err = np.abs(res.q.cpu().numpy() - q_ref).max()
    log(f"  iterations GPU {res.iterations} oracle {it_ref}; max|dq| {err:.2e}")
    assert res.converged and res.iterations == it_ref
    assert np.allclose(res.history, hist_ref, rtol=1e-5, atol=1e-9)
    assert err < 1e-7


# ---------------------------------------------------------------- learned
@pytest.mark.parametrize("nw,seed", [(96, 1), (300, 21)])
def test_descriptors_match_oracle(c, nw, seed):
    from paper_2606_03140_amd import learned
    box = waterbox.water_box(nw, seed)
    sysm = system_of(box)
    g = c.build_graph_cutoff(sysm, learned.DESCRIPTOR_CUTOFF)
    F = c.descriptors(sysm, g).cpu().numpy()
    ref = ol.descriptors(box.pos, box.species, box.box[0])
    err = np.abs(F - ref).max()
    log(f"descriptors {nw} waters: max|dG| {err:.2e} (max G {ref.max():.2f})")
    assert err < 1e-12 * max(1.0, ref.max())


def test_feature_norm_matches_oracle(c):
    boxes = [waterbox.displaced(waterbox.water_box(96, 1), 70 + j) for j in range(3)]
    feats = [ol.descriptors(b.pos, b.species, b.box[0]) for b in boxes]
    species = boxes[0].species
    stats = torch.zeros(192, dtype=torch.float64, device="cuda")
    sp = _dev(species, torch.int32)
    for f in feats:
        c.feature_sums(_dev(f), sp, stats)
    norm = torch.empty(2, 64, dtype=torch.float32, device="cuda")
    c.feature_norm(stats, norm)
    ref = ol.standardise_stats(np.concatenate(feats), np.concatenate([species] * 3))
    got = norm.cpu().numpy().astype(np.float64)
    for s in (0, 1):
        assert np.allclose(got[s, :32], ref[s][0], rtol=2e-7, atol=1e-7)
        assert np.allclose(got[s, 32:], ref[s][1], rtol=1e-6, atol=1e-7)


def _mlp_problem(seed=4):
    from paper_2606_03140_amd import learned
    box = waterbox.water_box(96, 1)
    feats = ol.descriptors(box.pos, box.species, box.box[0])
    species = box.species
    rng = np.random.default_rng(seed)
    nets = waterbox.mlp_init(seed)
    for net in nets:
        for k in ("b1", "b2", "b3"):
            net[k] = rng.uniform(-0.3, 0.3, size=net[k].shape)
    flat = learned.pack(nets)                       # float32: both sides use these exact values
    nets = learned.unpack(flat)
    st = ol.standardise_stats(feats, species)
    st = [(m.astype(np.float32).astype(np.float64), s.astype(np.float32).astype(np.float64)) for m, s in st]
    norm = np.stack([np.concatenate([m, s]) for m, s in st]).astype(np.float32)
    q_ref = np.where(species == 0, -0.8, 0.4) + rng.normal(0.0, 0.05, size=len(species))
    q_ref -= q_ref.mean()
    return nets, flat, st, norm, feats, species, q_ref


def _abs_bound(nets, st, feats, species, u):
    """First-order bound on |y_rounded - y| when weights, biases, inputs and the
    hidden activations are each rounded with unit roundoff u (|silu'| <= 1.1)."""
    bound = np.zeros(len(species))
    for s in (0, 1):
        idx = np.nonzero(species == s)[0]
        m, sd = st[s]
        x = (feats[idx] - m) / sd
        n = nets[s]
        z1 = x @ n["W1"].T + n["b1"]
        a1 = ol.silu(z1)
        z2 = a1 @ n["W2"].T + n["b2"]
        a2 = ol.silu(z2)
        dz1 = 2 * u * (np.abs(x) @ np.abs(n["W1"]).T + np.abs(n["b1"]))
        da1 = 1.1 * dz1 + u * np.abs(a1)
        dz2 = da1 @ np.abs(n["W2"]).T + 2 * u * (np.abs(a1) @ np.abs(n["W2"]).T + np.abs(n["b2"]))
        da2 = 1.1 * dz2 + u * np.abs(a2)
        bound[idx] = da2 @ np.abs(n["W3"][0]) + 2 * u * (np.abs(a2) @ np.abs(n["W3"][0]) + abs(n["b3"][0]))
    return bound


def test_mlp_forward_fp32_and_bf16(c):
    nets, flat, st, norm, feats, species, _ = _mlp_problem()
    y_ref, _ = ol.forward(nets, st, feats, species)
    P, N, F, S = _dev(flat, torch.float32), _dev(norm, torch.float32), _dev(feats), _dev(species, torch.int32)
    y = torch.empty(len(species), dtype=torch.float32, device="cuda")
    c.mlp_forward(S, F, P, N, False, y)
    e32 = np.abs(y.cpu().numpy() - y_ref)
    b32 = _abs_bound(nets, st, feats, species, 2.0 ** -24) * 32 + 1e-6
    log(f"MLP forward FP32: max err {e32.max():.2e}, max err/bound {(e32 / b32).max():.3f}")
    assert np.all(e32 <= b32)
    c.mlp_forward(S, F, P, N, True, y)
    e16 = np.abs(y.cpu().numpy() - y_ref)
    b16 = _abs_bound(nets, st, feats, species, 2.0 ** -8)
    log(f"MLP forward BF16: max err {e16.max():.2e}, max err/bound {(e16 / b16).max():.3f}")
    assert np.all(e16 <= b16)
    # neutral charges from the forward
    q = torch.empty(len(species), dtype=torch.float64, device="cuda")
    c.mlp_charges(y, q)
    yv = y.cpu().numpy().astype(np.float64)
    assert np.abs(q.cpu().numpy() - (yv - yv.mean())).max() < 1e-12


def test_mlp_gradients_match_oracle(c):
    from paper_2606_03140_amd import learned
    nets, flat, st, norm, feats, species, q_ref = _mlp_problem()
    loss_ref, g_ref = ol.loss_and_grads(nets, st, feats, species, q_ref)
    P, N, F, S = _dev(flat, torch.float32), _dev(norm, torch.float32), _dev(feats), _dev(species, torch.int32)
    n = len(species)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    st3 = torch.empty(3, dtype=torch.float64, device="cuda")
    partial = torch.empty(((n + 63) // 64) * 2 * learned.N_PARAMS, dtype=torch.float32, device="cuda")
    grad = torch.empty(2, learned.N_PARAMS, dtype=torch.float32, device="cuda")
    Q = _dev(q_ref)
    c.mlp_forward(S, F, P, N, False, y)
    c.mlp_loss(y, Q, st3)
    c.mlp_backward(S, F, P, N, y, Q, st3, partial, grad)
    loss = float(st3[2])
    log(f"MLP loss GPU {loss:.8f} oracle {loss_ref:.8f}")
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    got = learned.unpack(grad.cpu().numpy())
    for s in (0, 1):
        for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
            rel = np.linalg.norm(got[s][k] - g_ref[s][k]) / np.linalg.norm(g_ref[s][k])
            log(f"  grad species {s} {k}: rel err {rel:.2e}")
            assert rel < 1e-4
    # the reduction over blocks is deterministic
    g1 = grad.clone()
    c.mlp_backward(S, F, P, N, y, Q, st3, partial, grad)
    assert torch.equal(g1, grad)


def test_adam_matches_oracle(c):
    from paper_2606_03140_amd import learned
    nets, flat, st, norm, feats, species, q_ref = _mlp_problem()
    _, g = ol.loss_and_grads(nets, st, feats, species, q_ref)
    gflat = learned.pack(g)
    grads32 = learned.unpack(gflat)
    P = _dev(flat, torch.float32)
    G = _dev(gflat, torch.float32)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    opt = ol.Adam(nets, lr=1e-3)
    for t in range(1, 4):
        c.adam_step(P, G, m, v, t)
        opt.step(nets, grads32)
    got = learned.unpack(P.cpu().numpy())
    for s in (0, 1):
        for k in nets[s]:
            assert np.abs(got[s][k] - nets[s][k]).max() < 2e-7


def test_learned_guess_saves_scc_iterations(c):
    """Train on converged charges of displaced snapshots, then start the SCC
    loop of held-out snapshots from the prediction instead of zero."""
    from paper_2606_03140_amd import learned, pipeline, scc
    base = waterbox.water_box(48, 11)          # box edge 11.3 A > twice the 5 A descriptor cutoff
    tb = tb_params(False)
    species = _dev(base.species, torch.int32)

    def setup(b):
        sysm = system_of(b)
        part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 1))
        return sysm, part, scc.ewald_setup(c, sysm)

    model = learned.ChargeModel(c, waterbox.mlp_init(0))
    feats, labels, warm = [], [], None
    for j in range(16):
        sysm, part, ew = setup(waterbox.displaced(base, 500 + j))
        r = scc.scc_loop(c, sysm, tb, part, 0.1, pipeline.FP64_EIG, q_start=warm, ewald=ew)
        assert r.converged
        warm = r.q
        labels.append(r.q.clone())
        feats.append(model.descriptors(sysm))
    model.fit_norm(feats, species)
    hist = model.train(feats, species, labels, epochs=200, lr=2e-3, seed=1)
    log(f"training loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < hist[0] / 10
    its_zero, its_mlp = [], []
    for j in range(4):
        sysm, part, ew = setup(waterbox.displaced(base, 600 + j))
        r0 = scc.scc_loop(c, sysm, tb, part, 0.1, pipeline.FP64_EIG, ewald=ew)
        guess = model.predict(model.descriptors(sysm), species, bf16=True)
        start_rms = float(torch.sqrt(torch.mean((guess - r0.q) ** 2)))
        r1 = scc.scc_loop(c, sysm, tb, part, 0.1, pipeline.FP64_EIG, q_start=guess, ewald=ew)
        assert r0.converged and r1.converged
        dq = float(torch.sqrt(torch.mean((r0.q - r1.q) ** 2)))
        log(f"  held-out {j}: zero start {r0.iterations} it, MLP start {r1.iterations} it "
            f"(guess RMS error {start_rms:.2e} e), RMS dq between the converged charges {dq:.1e}")
        assert dq < 5e-5              # both stop at an RMS residual below 1e-5 e
        its_zero.append(r0.iterations)
        its_mlp.append(r1.iterations)
    log(f"  mean iterations: zero {np.mean(its_zero):.1f}, MLP {np.mean(its_mlp):.1f}")
    assert np.mean(its_mlp) <= np.mean(its_zero) - 3
