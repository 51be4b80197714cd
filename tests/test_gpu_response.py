"""Charge response and kernel-accelerated SCF on the GPU against the oracle.

* gdm_density_response (derivative of the recorded mixed-precision
  expansion, canonical chemical-potential shift) against the oracle's
  first-order perturbation theory on the eigenpairs, at the same mu, for
  the orthogonal and non-orthogonal model: element by element within a
  bound relative to the largest response; charge conserved; linear in dV
  to the precision of the split-FP16 products;
* the Krylov kernels (begin / add / apply) against the oracle's low-rank
  step on an explicit non-symmetric Jacobian;
* the quasi-Newton SCF on the mixed path reaches the oracle's SCC fixed
  point in a fraction of the Anderson iterations.
"""
import math

import numpy as np
import pytest
import torch

import waterbox
from oracle import graph as og
from oracle import model as om
from oracle import response as orsp
from oracle import scc as osc
from oracle import solve as osv
from tests.gpu_common import ctx, log, oracle_model, system_of, tb_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c():
    return ctx()


def oracle_subs(box, grid):
    L = box.box[0]
    rp, col = om.neighbour_list(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, grid)
    return og.extract_subgraphs(rp, col, core, nco)


@pytest.mark.parametrize("orthogonal,nw,seed", [(False, 48, 31), (True, 48, 32), (False, 300, 33)])
def test_density_response_matches_oracle(c, orthogonal, nw, seed):
    from paper_2606_03140_amd import pipeline
    log(f"charge response: {nw} waters, orthogonal={orthogonal}, seed {seed}")
    box = waterbox.water_box(nw, seed)
    L = box.box[0]
    sysm = system_of(box)
    tb = tb_params(orthogonal)
    grid = (2, 2, 2) if nw < 100 else (3, 3, 3)
    part = pipeline.cutoff_partition(c, sysm, tb, grid)
    subs = oracle_subs(box, grid)
    ap = part.sg.atom_ptr.cpu().numpy()
    at = part.sg.atoms.cpu().numpy()
    assert len(subs) == part.sg.n_sub
    for s, (atoms, _) in enumerate(subs):
        assert np.array_equal(at[ap[s]:ap[s + 1]], atoms)
    rng = np.random.default_rng(seed)
    n = len(box.species)
    V = 0.3 * rng.standard_normal(n)
    dV = rng.standard_normal(n)
    Vd = torch.as_tensor(V).to(c.dev)
    dVd = torch.as_tensor(dV).to(c.dev)
    H, S = c.build_hs(sysm, tb, part.nbr, Vd)
    c.set_response(16)
    try:
        sol = pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.MIXED_F16, mu_guess=-7.0)
        dq, dmu = c.density_response(sysm, part.sg, part.nbr, S, dVd)
        dq = dq.cpu().numpy()
        dq2, _ = c.density_response(sysm, part.sg, part.nbr, S, -2.0 * dVd)
        dq2 = dq2.cpu().numpy()
    finally:
        c.set_response(0)
    # the GPU's mu against the oracle's own search on the same potential
    # (the response below is then compared at the GPU's mu)
    mu_oracle = osv.solve_system(box.pos, box.species, L, oracle_model(orthogonal), subs, V_atom=V).mu
    log(f"  mu gpu {sol.mu:.6f}, oracle {mu_oracle:.6f} (|d| {abs(sol.mu - mu_oracle):.2e} eV)")
    assert abs(sol.mu - mu_oracle) < 5e-3
    ref, dmu_ref, _ = orsp.charge_response(box.pos, box.species, L, oracle_model(orthogonal), subs, V, dV,
                                           mu=sol.mu)
    scale = np.abs(ref).max()
    err = np.abs(dq - ref).max()
    log(f"  mu {sol.mu:.6f}; max|dq| {scale:.3e}; max|dq - oracle| {err:.2e} ({err / scale:.2e} rel); "
        f"dmu {dmu:.3e} (oracle {dmu_ref:.3e}); sum dq {dq.sum():.2e}")
    assert scale > 1e-2
    assert err < 1e-4 * scale
    assert abs(dq.sum()) < 1e-9 * np.abs(dq).sum()
    # linear in dV to the precision of the split-FP16 products (rounding of
    # FP16 subnormals does not commute with scaling; observed ~4e-7 relative)
    lin = np.abs(dq2 + 2.0 * dq).max()
    log(f"  linearity: max|dq(-2 dV) + 2 dq(dV)| {lin:.2e}")
    assert lin < 2e-6 * scale


def test_density_response_needs_recording(c):
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import GDMError
    box = waterbox.water_box(48, 31)
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 2))
    H, S = c.build_hs(sysm, tb, part.nbr)
    c.set_response(0)
    pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.MIXED_F16, mu_guess=-7.0)
    dV = torch.zeros(sysm.n_atoms, dtype=torch.float64, device=c.dev)
    with pytest.raises(GDMError):
        c.density_response(sysm, part.sg, part.nbr, S, dV)
    # room for fewer doublings than the expansion takes: not recorded either
    c.set_response(2)
    try:
        pipeline.solve(c, sysm, part, H, S, 0.1, pipeline.MIXED_F16, mu_guess=-7.0, plan=False)
        with pytest.raises(GDMError):
            c.density_response(sysm, part.sg, part.nbr, S, dV)
    finally:
        c.set_response(0)


@pytest.mark.parametrize("n,max_rank,k0,complete", [(200, 1, 1.0, False), (200, 4, 0.1, True), (1000, 8, 1.0, True),
                                                     (1000, 8, 0.1, False), (40, 16, 0.5, True)])
def test_krylov_kernels_match_oracle(c, n, max_rank, k0, complete):
    from paper_2606_03140_amd._lib import Context
    rng = np.random.default_rng(n + max_rank)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * -np.linspace(0.1, 40.0, n)) @ Q.T + 0.05 * rng.standard_normal((n, n))
    Jm = A - np.eye(n)
    nv0 = rng.standard_normal(n)
    q0 = rng.standard_normal(n)
    f = q0 - nv0
    rank_tol = 1e-3
    dn_ref, rank_ref, rel_ref = orsp.krylov_step(f, lambda v: Jm @ v, rank_tol=rank_tol, max_rank=max_rank,
                                                 k0=k0, complete=complete)
    nv = torch.as_tensor(nv0).to(c.dev)
    work = torch.empty(Context.krylov_work_size(n, max_rank), dtype=torch.float64, device=c.dev)
    rms = c.krylov_begin(nv, torch.as_tensor(q0).to(c.dev), max_rank, work, k0)
    assert abs(rms - math.sqrt(np.mean(f * f))) < 1e-12 * max(1.0, rms)
    Ad = torch.as_tensor(A).to(c.dev)
    rank = 0
    for j in range(max_rank):
        v = Context.krylov_vector(work, n, j)
        dq = Ad @ v                                  # J v + v for the affine map
        rel, exhausted = c.krylov_add(n, j, dq, max_rank, work)
        rank = j + 1
        if rel <= rank_tol or exhausted:
            break
    # a line-search trial at half length, then the full step from the same start
    c.krylov_apply(nv, rank, max_rank, work, 0.5, complete)
    half = nv.cpu().numpy() - nv0
    nv.copy_(torch.as_tensor(nv0).to(c.dev))
    c.krylov_apply(nv, rank, max_rank, work, 1.0, complete)
    got = nv.cpu().numpy() - nv0
    scale = max(1.0, np.abs(dn_ref).max())
    log(f"  Krylov n={n} cap {max_rank} k0 {k0} complete {complete}: rank {rank} (oracle {rank_ref}), "
        f"fit {rel:.3e} (oracle {rel_ref:.3e}), max|dn - oracle| {np.abs(got - dn_ref).max():.2e}")
    assert rank == rank_ref
    assert abs(rel - rel_ref) < 1e-9
    assert np.abs(got - dn_ref).max() < 1e-9 * scale
    assert np.abs(half - 0.5 * dn_ref).max() < 1e-9 * scale


def test_quasi_newton_scc_matches_oracle(c):
    from paper_2606_03140_amd import pipeline, scc
    log("quasi-Newton SCF, 32 waters, mixed path, vs the oracle's fixed point")
    box = waterbox.water_box(32, 11)
    L = box.box[0]
    sysm = system_of(box)
    tb = tb_params(False)
    part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 1))
    ew = scc.ewald_setup(c, sysm)
    res = scc.scc_quasi_newton(c, sysm, tb, part, 0.1, ewald=ew, mu_guess=-7.0)
    ra = scc.scc_loop(c, sysm, tb, part, 0.1, pipeline.MIXED_F16, ewald=ew, mu_guess=-7.0)
    subs = oracle_subs(box, (2, 2, 1))
    q_ref, it_ref, _ = osc.scc(box.pos, box.species, L, om.TBModel(), subs, short_cut=ew.rcut)
    err = np.abs(res.q.cpu().numpy() - q_ref).max()
    _, it_qn_ref, _, ranks_ref = orsp.scc_quasi_newton(box.pos, box.species, L, om.TBModel(), subs,
                                                         short_cut=ew.rcut)
    log(f"  quasi-Newton {res.iterations} iterations (oracle {it_qn_ref}), ranks {res.ranks} (oracle {ranks_ref}), "
        f"steps {res.alphas}, {res.solves} solves, {res.responses} responses; Anderson GPU {ra.iterations}, "
        f"oracle {it_ref}; max|q - oracle| {err:.2e}")
    assert res.converged and ra.converged
    assert res.iterations * 3 < ra.iterations
    assert abs(res.iterations - it_qn_ref) <= 2
    assert err < 1e-4
