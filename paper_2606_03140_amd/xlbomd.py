"""Extended-Lagrangian Born-Oppenheimer molecular dynamics over the libgdm
kernels (Shadow MD section).

Each step moves the nuclei by velocity Verlet on the forces of the shadow
potential U(R, n) at fixed extended charges n (gdm_md_verlet), propagates n
in a harmonic well centred on its Mulliken charges q[n] with the dissipative
Verlet form (gdm_xlbomd_charges), and evaluates the new point in one
linear solve, with no SCF iterations:

    neighbour graph -> halos (cutoff graph, or the adaptive graph G_tau of
    the previous step's density matrix) -> V[n] (gdm_ewald_potential) ->
    H[n], S -> mu, D, W (FP64 path) -> q[n], Omega -> forces (gdm_forces +
    gdm_ewald_forces).

The total free energy E = K + U(R, n), U = Omega + E_rep - sum (N0 + n/2) V,
is conserved up to the integrator's O(dt^2) fluctuation.  Only orchestration
lives here; every step is a libgdm call.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from ._lib import FP64_EIG, GRAPH_ADAPTIVE, MIXED_F16, Context, Subgraphs, System, TBParams
from .scc import HUBBARD_U, EwaldSetup, ewald_setup, scc_loop, scc_quasi_newton, slater_tau
from .pipeline import Partition, subgraph_cost

MASS = (15.999, 1.008)             # amu, O and H
KAPPA, ALPHA = 1.82, 0.018         # Niklasson et al. 2009, K = 5
EWALD_SKIN = 1.0                   # A, skin of the Ewald real-space pair list
# tapered radial functions and a repulsive pair term for the synthetic model:
# an isolated water has zero SCC force at r_OH = 0.96 A, 104.5 degrees
MD_TB = dict(taper_on=3.5, rep_A=(500.0, 67.92, 12.79), rep_rho=0.3)


def md_params(**kw) -> TBParams:
    return TBParams(**{**MD_TB, **kw})


def molecule_cores(system: System, anchor: np.ndarray) -> tuple[torch.Tensor, int]:
    """One core per molecule (the atoms sharing an anchor), numbered in
    anchor order."""
    anchor = np.asarray(anchor)
    mols = np.unique(anchor)
    core = np.searchsorted(mols, anchor).astype(np.int32)
    return torch.as_tensor(core).to(system.pos.device), int(len(mols))


@dataclass
class Point:
    """Shadow potential and forces at (R, n)."""
    F: torch.Tensor
    q: torch.Tensor
    U: float
    omega: float
    e_rep: float
    e_shift: float
    mu: float
    part: Partition
    D: torch.Tensor
    S: torch.Tensor | None = None
    ew: EwaldSetup | None = None
    H: torch.Tensor | None = None


@dataclass
class Record:
    t: list = field(default_factory=list)
    e_tot: list = field(default_factory=list)
    e_pot: list = field(default_factory=list)
    e_kin: list = field(default_factory=list)
    rms_qn: list = field(default_factory=list)
    sizes: list = field(default_factory=list)     # orbitals of each subgraph per step


class XLBOMD:
    """State and steps of one XL-BOMD run on the FP64 path.

    graph: "cutoff" (halos one hop in the neighbour graph) or "adaptive"
    (G_tau = (G^N G^D + G^D G^N)|_tau from the previous step's D, Eq.
    Graph_Adaptation, redrawn every `rebuild` steps so that halos expand and
    contract with the motion).

    kernel: "scaled" drives n with c (q[n] - n) (the kernel c I; stable only
    while kappa c times the largest |eigenvalue| of the charge Jacobian J
    stays below about 4, i.e. for a few molecules), or "krylov": with
    -J^-1 (q[n] - n) from the low-rank preconditioned Krylov kernel
    (gdm_krylov_*, K0 = -k0 I, completed on the unfitted remainder), rebuilt
    at every step.  Its directional derivatives J v = dq - v come from
    response="mixed": the perturbation-theory response of the
    mixed-precision expansion solved at the same H and S on a second
    context (gdm_density_response), or response="fd": one-sided finite
    differences of the FP64 solve, dq = (q[n + eps v] - q[n]) / eps (the
    FP64 path forms core rows only, so it has no perturbation-theory
    response of its own).  The kernel only preconditions the charge
    dynamics, so the responses' error (1e-5 relative either way) does not
    enter the forces or the energy."""

    def __init__(self, ctx: Context, system: System, tb: TBParams, core_of_atom: torch.Tensor, n_cores: int,
                 kT: float = 0.1, dt: float = 0.25, c: float = 0.3, graph: str = "cutoff", tau: float = 1e-5,
                 alpha: float = 0.7, screened: bool = True, ewald_tol: float = 1e-10, rebuild: int = 1,
                 timing: bool = False, kernel: str = "scaled", rank_tol: float = 0.1, max_rank: int = 6,
                 k0: float = 0.1, fd_eps: float = 1e-5, response: str = "mixed"):
        if kernel not in ("scaled", "krylov") or response not in ("mixed", "fd"):
            raise ValueError(f"kernel {kernel!r}, response {response!r}")
        self.kernel, self.rank_tol, self.max_rank, self.k0, self.fd_eps = kernel, rank_tol, max_rank, k0, fd_eps
        self.response = response
        self.ctx_m = None
        self._m_sg = None
        self._m_cap = 8
        self.ranks: list = []
        self.ctx, self.system, self.tb = ctx, system, tb
        self.core, self.n_cores = core_of_atom, n_cores
        self.kT, self.dt, self.c = kT, dt, c
        self.graph_mode, self.tau, self.alpha = graph, tau, alpha
        self.rebuild = max(1, int(rebuild))      # halos redrawn every `rebuild` steps
        self.steps_done = 0
        self._ew: EwaldSetup | None = None
        self._ew_pos: np.ndarray | None = None
        self.timing = {} if timing else None
        self.tau_s = slater_tau(HUBBARD_U) if screened else None
        self.ewald_tol = ewald_tol
        n = system.n_atoms
        dev = system.pos.device
        self.vel = torch.zeros(n, 3, dtype=torch.float64, device=dev)
        self.hist = torch.zeros(6, n, dtype=torch.float64, device=dev)
        self.energy = torch.zeros(2, dtype=torch.float64, device=dev)
        self.kin = torch.zeros(1, dtype=torch.float64, device=dev)
        if kernel == "krylov":
            self.kwork = torch.zeros(Context.krylov_work_size(n, max_rank), dtype=torch.float64, device=dev)
            self.delta = torch.zeros(n, dtype=torch.float64, device=dev)
            self.n_eps = torch.zeros(n, dtype=torch.float64, device=dev)
            self.dq = torch.zeros(n, dtype=torch.float64, device=dev)
            self.dV = torch.zeros(n, dtype=torch.float64, device=dev)
            if response == "mixed":
                self.ctx_m = Context(ctx.device)
                self.ctx_m.set_response(self._m_cap)
        self.mu = 0.0
        self.point: Point | None = None
        self.rec = Record()
        self.t = 0.0

    # ------------------------------------------------------------ pieces
    def _ewald(self) -> EwaldSetup:
        """Ewald split and real-space pair list, built with a 1 A skin and
        rebuilt once some atom has moved more than half the skin since the
        list was built (the kernels skip pairs at r >= rcut, so until then
        the list holds every pair within rcut)."""
        pos = self.system.pos.cpu().numpy()
        if self._ew is not None:
            moved = float(np.sqrt(((pos - self._ew_pos) ** 2).sum(axis=1).max()))
            if moved <= 0.5 * EWALD_SKIN:
                return self._ew
        self._ew = ewald_setup(self.ctx, self.system, tol=self.ewald_tol, skin=EWALD_SKIN)
        self._ew_pos = pos
        return self._ew

    def _partition(self, prev: Point | None) -> Partition:
        """Neighbour graph at the current positions; the halos are redrawn
        every `rebuild` steps (from the previous D in adaptive mode) and
        otherwise keep the previous subgraph atom lists."""
        ctx, sysm = self.ctx, self.system
        nbr = ctx.build_graph_cutoff(sysm, self.tb.cutoff)
        if prev is not None and self.steps_done % self.rebuild != 0:
            p = prev.part
            return Partition(nbr=nbr, graph=p.graph, core_of_atom=p.core_of_atom, n_cores=p.n_cores, sg=p.sg,
                             sizes=p.sizes, cost0=p.cost0)
        g = nbr
        if self.graph_mode == "adaptive" and prev is not None:
            g = ctx.build_graph_dm(sysm, GRAPH_ADAPTIVE, prev.part.sg, prev.D, self.tau, alpha=self.alpha, nbr=nbr)
        sg = ctx.extract_subgraphs(sysm, self.tb, g, self.core, self.n_cores)
        return Partition(nbr=nbr, graph=g, core_of_atom=self.core, n_cores=self.n_cores, sg=sg,
                         sizes=[sg.norb.copy()], cost0=subgraph_cost(sg))

    def _lap(self, name: str, t0: float) -> float:
        if self.timing is None:
            return t0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        self.timing[name] = self.timing.get(name, 0.0) + (t1 - t0)
        return t1

    def evaluate(self, n_vec: torch.Tensor, prev: Point | None = None) -> Point:
        """U(R, n), q[n] and the forces at the current positions."""
        ctx, sysm, tb = self.ctx, self.system, self.tb
        t = time.perf_counter()
        part = self._partition(prev)
        ew = self._ewald()
        t = self._lap("graphs", t)
        V = ctx.ewald_potential(sysm, ew.graph, ew.rcut, ew.eta, ew.k_max, HUBBARD_U, n_vec, tau=self.tau_s)
        H, S = ctx.build_hs(sysm, tb, part.nbr, V)
        t = self._lap("potential_hs", t)
        if prev is None or part.sg is not prev.part.sg:
            ctx.plan(part.sg, FP64_EIG)
        mu, _ = ctx.find_mu(sysm, part.sg, part.nbr, H, S, self.kT, FP64_EIG, self.mu)
        self.mu = mu
        D = ctx.subgraph_density(part.sg, mu, self.kT, FP64_EIG)
        t = self._lap("solve", t)
        W = ctx.subgraph_edm(part.sg, mu, self.kT)
        t = self._lap("edm", t)
        q = ctx.mulliken_charges(sysm, part.sg, part.nbr, S, D)
        omega = ctx.band_energy(part.sg, mu, self.kT)
        t = self._lap("charges_energy", t)
        F = ctx.forces(sysm, tb, part.nbr, part.sg, D, W, V_atom=V, n_vec=n_vec, energy=self.energy)
        t = self._lap("forces", t)
        ctx.ewald_forces(sysm, ew.graph, ew.rcut, ew.eta, ew.k_max, q, n_vec, F, tau=self.tau_s)
        t = self._lap("ewald_forces", t)
        e_rep, e_shift = (float(x) for x in self.energy.cpu())
        ctx.check()
        return Point(F=F, q=q, U=omega + e_rep + e_shift, omega=omega, e_rep=e_rep, e_shift=e_shift, mu=mu,
                     part=part, D=D, S=S, ew=ew, H=H)

    def _charges_at(self, p: Point, n_vec: torch.Tensor) -> torch.Tensor:
        """q[n_vec] at the positions and subgraphs of point p (FP64 solve)."""
        ctx, sysm = self.ctx, self.system
        ew = p.ew
        V = ctx.ewald_potential(sysm, ew.graph, ew.rcut, ew.eta, ew.k_max, HUBBARD_U, n_vec, tau=self.tau_s)
        H, S = ctx.build_hs(sysm, self.tb, p.part.nbr, V)
        mu, _ = ctx.find_mu(sysm, p.part.sg, p.part.nbr, H, S, self.kT, FP64_EIG, p.mu)
        D = ctx.subgraph_density(p.part.sg, mu, self.kT, FP64_EIG)
        return ctx.mulliken_charges(sysm, p.part.sg, p.part.nbr, S, D)

    def _mixed_solve(self, p: Point) -> None:
        """Mixed-precision solve at p's H and S on the second context, with
        the expansion recorded for its charge response."""
        cm, sysm = self.ctx_m, self.system
        if p.part.sg is not self._m_sg:
            cm.plan(p.part.sg, MIXED_F16)
            self._m_sg = p.part.sg
        cm.find_mu(sysm, p.part.sg, p.part.nbr, p.H, p.S, self.kT, MIXED_F16, p.mu)
        nd = cm.mixed_stats()["n_doublings"]
        if nd > self._m_cap:          # more doublings than the record holds: grow it, solve again
            self._m_cap = nd + 2
            cm.set_response(self._m_cap)
            cm.find_mu(sysm, p.part.sg, p.part.nbr, p.H, p.S, self.kT, MIXED_F16, p.mu)

    def _response(self, p: Point, n_t: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
        """dq = J v + v, the charge response to the potential of v."""
        ctx, sysm = self.ctx, self.system
        if self.response == "mixed":
            ew = p.ew
            ctx.ewald_potential(sysm, ew.graph, ew.rcut, ew.eta, ew.k_max, HUBBARD_U, v, tau=self.tau_s, out=self.dV)
            self.ctx_m.density_response(sysm, p.part.sg, p.part.nbr, p.S, self.dV, out=self.dq)
            return self.dq
        ctx.axpby(1.0, n_t, self.fd_eps, v, self.n_eps)
        q_eps = self._charges_at(p, self.n_eps)
        ctx.axpby(1.0 / self.fd_eps, q_eps, -1.0 / self.fd_eps, p.q, self.dq)
        return self.dq

    def _krylov_delta(self, p: Point, n_t: torch.Tensor) -> torch.Tensor:
        """-J^-1 (q[n_t] - n_t) at point p by the low-rank Krylov kernel."""
        ctx, N = self.ctx, self.system.n_atoms
        t = time.perf_counter()
        if self.response == "mixed":
            self._mixed_solve(p)
        ctx.krylov_begin(n_t, p.q, self.max_rank, self.kwork, self.k0)
        rank = 0
        for j in range(self.max_rank):
            v = Context.krylov_vector(self.kwork, N, j)
            dq = self._response(p, n_t, v)
            rel, exhausted = ctx.krylov_add(N, j, dq, self.max_rank, self.kwork)
            rank = j + 1
            if rel <= self.rank_tol or exhausted:
                break
        self.ranks.append(rank)
        self.delta.zero_()
        ctx.krylov_apply(self.delta, rank, self.max_rank, self.kwork, 1.0, complete=True)
        self._lap("kernel", t)
        return self.delta

    # ------------------------------------------------------------ run
    def start(self, n0: torch.Tensor, vel0) -> None:
        """n = n0 (the converged SCC charges) in every history slot."""
        self.hist.copy_(n0.to(self.hist.dtype).expand(6, -1))
        self.vel.copy_(torch.as_tensor(np.asarray(vel0, dtype=np.float64)))
        self.point = self.evaluate(self.hist[0].clone())
        if self.graph_mode == "adaptive":      # halos from the solved D
            self.point = self.evaluate(self.hist[0].clone(), self.point)
        self.ctx.md_verlet(self.system, MASS, 0.0, self.point.F, self.vel, drift=False, kinetic=self.kin)
        self._record()

    def _record(self) -> None:
        p = self.point
        ek = float(self.kin.cpu()[0])
        r = self.rec
        r.t.append(self.t)
        r.e_kin.append(ek)
        r.e_pot.append(p.U)
        r.e_tot.append(ek + p.U)
        d = p.q.cpu().numpy() - self.hist[0].cpu().numpy()
        r.rms_qn.append(float(np.sqrt(np.mean(d * d))))
        r.sizes.append(p.part.sg.norb.copy())

    def step(self) -> None:
        ctx, sysm = self.ctx, self.system
        p = self.point
        if self.kernel == "krylov":
            delta = self._krylov_delta(p, self.hist[0])
            ctx.xlbomd_charges(p.q, self.hist, KAPPA, ALPHA, delta=delta)
        else:
            ctx.xlbomd_charges(p.q, self.hist, KAPPA * self.c, ALPHA)
        ctx.md_verlet(sysm, MASS, self.dt, p.F, self.vel, drift=True)
        self.steps_done += 1
        self.point = self.evaluate(self.hist[0].clone(), p)
        ctx.md_verlet(sysm, MASS, self.dt, self.point.F, self.vel, drift=False, kinetic=self.kin)
        self.t += self.dt
        self._record()

    def run(self, steps: int) -> Record:
        for _ in range(steps):
            self.step()
        return self.rec


def converged_charges(ctx: Context, system: System, tb: TBParams, core, n_cores: int, kT: float = 0.1,
                      tol: float = 1e-9, screened: bool = True, mixer: str = "anderson", mix: float = 0.03,
                      depth: int = 8, max_iter: int = 400, log=None) -> torch.Tensor:
    """SCC ground-state charges on the cutoff-graph halos (the starting n).
    Anderson needs a memory well below the number of atoms; a few molecules
    converge with linear mixing (mixer="linear", mix=0.3); large boxes with
    the kernel-accelerated quasi-Newton SCF (mixer="quasi_newton", mixed
    path, whose fixed point lies within its 1e-5 accuracy of the FP64 one)."""
    nbr = ctx.build_graph_cutoff(system, tb.cutoff)
    sg = ctx.extract_subgraphs(system, tb, nbr, core, n_cores)
    part = Partition(nbr=nbr, graph=nbr, core_of_atom=core, n_cores=n_cores, sg=sg)
    if mixer == "quasi_newton":       # kernel-accelerated SCF on the mixed path (SI section C)
        res = scc_quasi_newton(ctx, system, tb, part, kT, tol=tol, max_iter=max_iter, screened=screened,
                               max_doublings=10, log=log)
        if not res.converged:
            raise RuntimeError(f"SCC did not converge in {res.iterations} iterations")
        return res.q
    res = scc_loop(ctx, system, tb, part, kT, FP64_EIG, tol=tol, max_iter=max_iter, screened=screened, mixer=mixer,
                   mix=mix, depth=depth)
    if not res.converged:
        raise RuntimeError(f"SCC did not converge in {res.iterations} iterations")
    return res.q


def maxwell_velocities(species: np.ndarray, temperature: float, seed: int) -> np.ndarray:
    """Seeded Maxwell velocities (A/fs) at `temperature` K, zero total momentum."""
    kB = 8.617333262e-5
    m = np.array(MASS)[species]
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(len(species), 3)) * np.sqrt(kB * temperature / (m[:, None] * 103.6426965))
    v -= (m[:, None] * v).sum(axis=0) / m.sum()
    return v


__all__ = ["XLBOMD", "MD_TB", "MASS", "KAPPA", "ALPHA", "md_params", "molecule_cores", "converged_charges",
           "maxwell_velocities"]
