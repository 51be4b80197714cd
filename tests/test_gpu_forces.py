"""GPU parity of the shadow-potential forces and of XL-BOMD against the oracle.

* energy-weighted density rows, band free energy, repulsive and Coulomb
  energy terms, band/Pulay/SCC-shift/repulsion forces and Coulomb forces of
  gdm_subgraph_edm, gdm_band_energy, gdm_forces and gdm_ewald_forces against
  oracle/forces.py on the same (R, n): one whole-system subgraph and
  grid-core partitions with one-hop halos, on a 24-water box and the
  96-water box (FP64: rows within 1e-9, energies within 1e-8 eV per atom,
  forces within 1e-7 eV/A);
* forces sum to zero;
* ten XL-BOMD steps of a water dimer follow the oracle's trajectory;
* the total free energy fluctuation grows by about four per time-step
  doubling (Shadow MD results);
* with the adaptive graph G_tau and one core per molecule, the halos of two
  colliding waters expand to the whole system and contract back to the
  cores (Shadow MD results, expansion and contraction of the subgraphs), with
  no jump in the total free energy.
"""
import numpy as np
import pytest
import torch

import waterbox
from oracle import forces as ofo
from oracle import graph as og
from oracle import model as om
from oracle import scc as oscc
from oracle import xlbomd as oxl
from paper_2606_03140_amd import pipeline, xlbomd
from paper_2606_03140_amd._lib import FP64_EIG, System, TBParams
from paper_2606_03140_amd.scc import HUBBARD_U, ewald_setup, slater_tau
from tests.gpu_common import ctx, log, system_of, unpack_dcore

pytestmark = pytest.mark.gpu

MD = dict(taper_on=3.5, rep_A=(500.0, 67.92, 12.79), rep_rho=0.3)
TH = np.radians(52.25)
WATER = np.array([[0.0, 0.0, 0.0], [0.96 * np.sin(TH), 0.0, 0.96 * np.cos(TH)],
                  [-0.96 * np.sin(TH), 0.0, 0.96 * np.cos(TH)]])
ROT = np.array([[0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])


@pytest.fixture(scope="module")
def c():
    return ctx()


def gpu_point(c, system, tb, part, n_vec, kT=0.1):
    ew = ewald_setup(c, system)
    tau = slater_tau(HUBBARD_U)
    V = c.ewald_potential(system, ew.graph, ew.rcut, ew.eta, ew.k_max, HUBBARD_U, n_vec, tau=tau)
    H, S = c.build_hs(system, tb, part.nbr, V)
    c.plan(part.sg, FP64_EIG)
    mu, _ = c.find_mu(system, part.sg, part.nbr, H, S, kT, FP64_EIG)
    D = c.subgraph_density(part.sg, mu, kT, FP64_EIG)
    W = c.subgraph_edm(part.sg, mu, kT)
    q = c.mulliken_charges(system, part.sg, part.nbr, S, D)
    omega = c.band_energy(part.sg, mu, kT)
    energy = torch.zeros(2, dtype=torch.float64, device="cuda")
    F = c.forces(system, tb, part.nbr, part.sg, D, W, V_atom=V, n_vec=n_vec, energy=energy)
    F_band = F.clone()
    c.ewald_forces(system, ew.graph, ew.rcut, ew.eta, ew.k_max, q, n_vec, F, tau=tau)
    c.check()
    e = energy.cpu().numpy()
    return dict(mu=mu, D=D, W=W, q=q.cpu().numpy(), omega=omega, e_rep=e[0], e_shift=e[1],
                U=omega + e[0] + e[1], F=F.cpu().numpy(), F_band=F_band.cpu().numpy(), V=V.cpu().numpy(), ew=ew)


def oracle_ewald(ew):
    return ofo.Ewald(eta=ew.eta, n_real=2, k_max=ew.k_max, screened=True, short_cut=ew.rcut)


def compare(c, box, part, n_vec, log_name):
    system = system_of(box)
    tb = TBParams(**MD)
    g = gpu_point(c, system, tb, part, torch.as_tensor(n_vec).to("cuda"))
    L = float(box.box[0])
    model = om.TBModel(**MD)
    subs = part.sg.host_lists()
    o = ofo.shadow_point(box.pos, box.species, L, model, subs, n_vec, oracle_ewald(g["ew"]))
    N = len(box.species)
    log(f"{log_name}: {part.sg.n_sub} subgraphs, |F| max {np.abs(o.F).max():.3f} eV/A")
    # energy-weighted rows
    beta = model.beta
    wo = [ofo.edm_core_rows(s, g["mu"], beta) for s in o.system.sols]
    for a, b in zip(unpack_dcore(part.sg, g["W"]), wo):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-9)
    np.testing.assert_allclose(g["V"], o.V, rtol=0, atol=1e-8)
    np.testing.assert_allclose(g["q"], o.q, rtol=0, atol=1e-9)
    assert abs(g["omega"] - o.omega) < 1e-8 * N
    assert abs(g["e_rep"] - o.e_rep) < 1e-9 * N
    assert abs(g["U"] - o.U) < 1e-8 * N
    np.testing.assert_allclose(g["F"], o.F, rtol=0, atol=1e-7)
    assert np.abs(g["F"].sum(axis=0)).max() < 1e-9 * N
    assert np.abs(g["F_band"].sum(axis=0)).max() < 1e-9 * N
    return g, o


@pytest.fixture(scope="module")
def box24():
    return waterbox.water_box(24, 21)


def test_forces_whole_system(c, box24):
    system = system_of(box24)
    part = pipeline.full_system_partition(c, system, TBParams(**MD))
    n = np.random.default_rng(4).normal(scale=0.05, size=len(box24.species))
    compare(c, box24, part, n, "whole 24 waters")


@pytest.mark.parametrize("nw,seed,grid", [(24, 21, (2, 2, 1)), (96, 1, (2, 2, 2))])
def test_forces_partitioned(c, nw, seed, grid):
    box = waterbox.water_box(nw, seed)
    system = system_of(box)
    part = pipeline.cutoff_partition(c, system, TBParams(**MD), grid)
    n = np.random.default_rng(5).normal(scale=0.05, size=len(box.species))
    compare(c, box, part, n, f"{nw} waters grid {grid}")


def dimer_box(gap=(3.3, 3.1, 5.9), L=24.0):
    pos = np.concatenate([WATER + 8.0, WATER @ ROT.T + np.add(gap, 5.0)])
    sp = np.array([0, 1, 1, 0, 1, 1], dtype=np.int32)
    anchor = np.array([0, 0, 0, 3, 3, 3], dtype=np.int32)
    return pos, sp, anchor, L


def gpu_md(c, pos, sp, anchor, L, vel, dt, steps, graph="cutoff", n0=None, **kw):
    system = System(pos, sp, anchor, (L, L, L))
    tb = xlbomd.md_params()
    core, nco = xlbomd.molecule_cores(system, anchor)
    if n0 is None:
        n0 = xlbomd.converged_charges(c, system, tb, core, nco, tol=1e-10, mixer="linear", mix=0.3)
    md = xlbomd.XLBOMD(c, system, tb, core, nco, dt=dt, c=0.3, graph=graph, **kw)
    md.start(n0, vel)
    md.run(steps)
    return md, system


def test_xlbomd_follows_oracle_trajectory(c):
    pos, sp, anchor, L = dimer_box()
    vel = xlbomd.maxwell_velocities(sp, 600.0, 5)
    md, system = gpu_md(c, pos, sp, anchor, L, vel, 0.25, 10)
    ew = md._ew                      # the run's own Ewald split and cutoff
    model = om.TBModel(**MD)
    oew = oracle_ewald(ew)
    core = np.array([0, 0, 0, 1, 1, 1])

    def subs(R):      # one core per molecule, halos one hop in the neighbour graph
        rp, col = om.neighbour_list(R, L)
        return og.extract_subgraphs(rp, col, core, 2)

    q0, _, _ = oscc.scc(pos, sp, L, model, subs(pos), mix=0.3, tol=1e-11, max_iter=400, eta=oew.eta,
                        n_real=oew.n_real, k_max=oew.k_max, short_cut=oew.short_cut)
    tr = oxl.run(pos, vel, sp, L, model, subs, q0, oew, 0.25, 10, c=0.3, keep_pos=True)
    log(f"dimer: E drift GPU {md.rec.e_tot[-1] - md.rec.e_tot[0]:.2e}, oracle {tr.e_tot[-1] - tr.e_tot[0]:.2e}")
    np.testing.assert_allclose(md.rec.e_tot, tr.e_tot, rtol=0, atol=1e-7)
    np.testing.assert_allclose(system.pos.cpu().numpy(), tr.pos[-1], rtol=0, atol=1e-9)


@pytest.mark.parametrize("response", ["fd", "mixed"])
def test_xlbomd_krylov_kernel_follows_oracle(c, response):
    """The Krylov kernel at full rank (every charge direction fitted) is
    -J^-1 itself; the GPU's responses (finite differences of the FP64
    solve, or the perturbation theory of the mixed expansion) and the
    oracle's perturbation theory then agree to about 1e-5."""
    pos, sp, anchor, L = dimer_box()
    vel = xlbomd.maxwell_velocities(sp, 600.0, 5)
    kw = dict(kernel="krylov", max_rank=6, rank_tol=1e-9, k0=0.1)
    md, system = gpu_md(c, pos, sp, anchor, L, vel, 0.25, 8, response=response, **kw)
    ew = md._ew                      # the run's own Ewald split and cutoff
    model = om.TBModel(**MD)
    oew = oracle_ewald(ew)
    core = np.array([0, 0, 0, 1, 1, 1])

    def subs(R):
        rp, col = om.neighbour_list(R, L)
        return og.extract_subgraphs(rp, col, core, 2)

    q0, _, _ = oscc.scc(pos, sp, L, model, subs(pos), mix=0.3, tol=1e-11, max_iter=400, eta=oew.eta,
                        n_real=oew.n_real, k_max=oew.k_max, short_cut=oew.short_cut)
    tr = oxl.run(pos, vel, sp, L, model, subs, q0, oew, 0.25, 8, keep_pos=True, **kw)
    log(f"dimer, Krylov kernel (ranks {md.ranks}): max rms(q - n) GPU {max(md.rec.rms_qn):.2e} "
        f"oracle {max(tr.rms_qn):.2e}")
    np.testing.assert_allclose(md.rec.rms_qn, tr.rms_qn, rtol=1e-3, atol=1e-9)
    np.testing.assert_allclose(md.rec.e_tot, tr.e_tot, rtol=0, atol=1e-6)
    np.testing.assert_allclose(system.pos.cpu().numpy(), tr.pos[-1], rtol=0, atol=1e-8)


def test_xlbomd_energy_fluctuation_fourfold(c):
    pos, sp, anchor, L = dimer_box()
    vel = xlbomd.maxwell_velocities(sp, 600.0, 7)
    amp = []
    for dt in (0.5, 0.25, 0.125):
        md, _ = gpu_md(c, pos, sp, anchor, L, vel, dt, int(round(10.0 / dt)))
        e = np.array(md.rec.e_tot)
        amp.append(e.max() - e.min())
        log(f"dt {dt}: fluctuation {amp[-1]:.3e} eV, max rms(q - n) {max(md.rec.rms_qn):.2e}")
    log(f"ratios {amp[0] / amp[1]:.2f} {amp[1] / amp[2]:.2f}")
    assert 3.3 < amp[0] / amp[1] < 4.7 and 3.3 < amp[1] / amp[2] < 4.7


def test_xlbomd_condensed_phase_krylov_kernel(c):
    """96 waters in their periodic box, 8 grid cores with one-hop halos: the
    strong collective charge response makes the kernel c I unstable, the
    Krylov kernel keeps q[n] - n small and the total free energy
    fluctuation falls with dt (Shadow MD results: about four per
    doubling)."""
    box = waterbox.water_box(96, 1)
    system = System(box.pos, box.species, box.anchor, box.box)
    tb = xlbomd.md_params()
    core, nco = c.grid_cores(system, (2, 2, 2))
    n0 = xlbomd.converged_charges(c, system, tb, core, nco, tol=1e-8)
    vel = xlbomd.maxwell_velocities(box.species, 300.0, 5005)
    amp = []
    for dt in (0.5, 0.25):
        sysm = System(box.pos, box.species, box.anchor, box.box)
        md = xlbomd.XLBOMD(c, sysm, tb, core, nco, dt=dt, kernel="krylov")
        md.start(n0, vel)
        md.run(int(round(6.0 / dt)))
        e = np.array(md.rec.e_tot)
        amp.append(e.max() - e.min())
        log(f"96 waters dt {dt}: fluctuation {amp[-1]:.3e} eV, max rms(q - n) {max(md.rec.rms_qn):.2e}, "
            f"kernel ranks {np.mean(md.ranks):.1f}")
        assert max(md.rec.rms_qn) < 1e-2
    log(f"ratio {amp[0] / amp[1]:.2f}")
    assert amp[1] < 1e-2 and 3.0 < amp[0] / amp[1] < 7.0


def test_halos_expand_and_contract(c):
    # two waters 6.5 A apart moving towards each other: no halo, then both
    # subgraphs hold all six atoms while they interact, then cores only again
    pos = np.concatenate([WATER + [8.0, 8.0, 8.0], WATER @ ROT.T + [14.5, 8.3, 8.2]])
    sp = np.array([0, 1, 1, 0, 1, 1], dtype=np.int32)
    anchor = np.array([0, 0, 0, 3, 3, 3], dtype=np.int32)
    vel = np.zeros((6, 3))
    vel[:3, 0] = 0.025
    vel[3:, 0] = -0.025
    md, _ = gpu_md(c, pos, sp, anchor, 24.0, vel, 0.25, 1000, graph="adaptive")
    sizes = np.array([s.tolist() for s in md.rec.sizes])      # [steps+1, 2] orbitals per subgraph
    e = np.array(md.rec.e_tot)
    full = np.nonzero((sizes == 12).all(axis=1))[0]
    log(f"halo sizes: start {sizes[0]}, full from step {full[0] if len(full) else None} to "
        f"{full[-1] if len(full) else None}, end {sizes[-1]}; E range {e.max() - e.min():.2e} eV")
    assert (sizes[0] == 6).all() and len(full) > 0
    assert (sizes[-1] == 6).all() and full[-1] < len(sizes) - 1
    assert e.max() - e.min() < 2e-3
    assert np.abs(np.diff(e)).max() < 2e-4
