"""Self-consistent-charge loop over the libgdm kernels.

The charge vector n of SI section D is iterated to self-consistency: the
Coulomb potential V = gamma n (periodic Ewald sum, screened at short range
by the interaction of exponential charge densities, Hubbard U on site:
gdm_ewald_potential) shifts H by 1/2 S_ab (V_I + V_J) (gdm_build_hs), one
density solve at a global mu gives the Mulliken charges q0[n], and the
update moves n towards the fixed point q0[n] = n: Anderson acceleration
(memory 8, mixing 0.03, gdm_scc_anderson) by default, or the scaled-delta
kernel K = -c I of the Shadow MD section (linear mixing, gdm_scc_mix).
scc_quasi_newton is the kernel-accelerated SCF of SI section C: each step
n <- n - (K0 J)^-1 K0 f(n) uses the low-rank preconditioned Krylov kernel
(gdm_krylov_*), whose directional derivatives J v are charge responses of
the mixed-precision solve (gdm_density_response) to the potential of v.
Iteration stops when the RMS residual is below the tolerance.  Only
orchestration lives here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from ._lib import FP64_EIG, MIXED_F16, Context, Graph, System, TBParams
from .pipeline import Partition, solve

HARTREE_EV = 27.211386
BOHR_A = 0.529177210903
HUBBARD_U = (0.5 * HARTREE_EV, 0.4 * HARTREE_EV)      # O-like, H-like (eV)


def slater_tau(hubbard_U) -> tuple:
    """Exponents (1/A) of the exponential charge densities whose Coulomb
    interaction is the screened gamma: tau = 16/5 U in atomic units."""
    return tuple(16.0 / 5.0 * (u / HARTREE_EV) / BOHR_A for u in hubbard_U)


@dataclass
class EwaldSetup:
    rcut: float
    eta: float
    k_max: int
    graph: Graph


def ewald_setup(ctx: Context, system: System, rcut_max: float = 12.0, tol: float = 1e-10,
                skin: float = 0.0) -> EwaldSetup:
    """Split parameters for a truncation error of about `tol` in both sums:
    erfc(eta rcut) ~ tol and exp(-k_c^2 / 4 eta^2) ~ tol, rcut + skin below
    half the shortest box edge, plus the real-space pair CSR at rcut + skin
    (the kernel skips pairs at r >= rcut, so the list stays valid while no
    atom moves more than skin / 2)."""
    L = system.box
    rcut = min(rcut_max, 0.499 * min(L) - skin)
    a = math.sqrt(-math.log(tol))
    eta = a / rcut
    k_c = 2.0 * eta * a
    k_max = int(math.ceil(k_c * max(L) / (2.0 * math.pi)))
    graph = ctx.build_graph_cutoff(system, rcut + skin)
    return EwaldSetup(rcut=rcut, eta=eta, k_max=k_max, graph=graph)


@dataclass
class SCCResult:
    q: torch.Tensor
    iterations: int
    converged: bool
    history: list = field(default_factory=list)
    mu: float = 0.0


def scc_loop(ctx: Context, system: System, tb: TBParams, part: Partition, kT: float, precision: int = FP64_EIG,
             q_start: torch.Tensor | None = None, mix: float = 0.03, tol: float = 1e-5, max_iter: int = 200,
             ewald: EwaldSetup | None = None, hubbard_U=HUBBARD_U, mu_guess: float = 0.0,
             plan: bool = True, mixer: str = "anderson", depth: int = 8, screened: bool = True) -> SCCResult:
    """Returns q0[n] at the first n whose residual RMS(q0[n] - n) < tol."""
    ew = ewald if ewald is not None else ewald_setup(ctx, system)
    tau = slater_tau(hubbard_U) if screened else None
    n = torch.zeros(system.n_atoms, dtype=torch.float64, device=ctx.dev) if q_start is None \
        else q_start.to(device=ctx.dev, dtype=torch.float64).clone()
    V = torch.empty_like(n)
    work = torch.empty((3 * depth + 2) * system.n_atoms, dtype=torch.float64, device=ctx.dev) \
        if mixer == "anderson" else None
    hist = []
    mu = mu_guess
    for it in range(1, max_iter + 1):
        ctx.ewald_potential(system, ew.graph, ew.rcut, ew.eta, ew.k_max, hubbard_U, n, tau=tau, out=V)
        H, S = ctx.build_hs(system, tb, part.nbr, V)
        sol = solve(ctx, system, part, H, S, kT, precision, mu_guess=mu, plan=plan and it == 1)
        mu = sol.mu
        if mixer == "anderson":
            rms = ctx.scc_anderson(n, sol.q, mix, depth, it - 1, work)
        else:
            rms = ctx.scc_mix(n, sol.q, mix)
        hist.append(rms)
        if rms < tol:
            return SCCResult(q=sol.q, iterations=it, converged=True, history=hist, mu=mu)
    return SCCResult(q=n, iterations=max_iter, converged=False, history=hist, mu=mu)


@dataclass
class QuasiNewtonResult(SCCResult):
    ranks: list = field(default_factory=list)        # Krylov vectors per step
    fits: list = field(default_factory=list)         # relative residual of each step's low-rank fit
    alphas: list = field(default_factory=list)       # accepted step lengths
    solves: int = 0                                  # density solves (including line-search trials)
    responses: int = 0                               # charge-response solves


E_NO_BRACKET = -4


def scc_quasi_newton(ctx: Context, system: System, tb: TBParams, part: Partition, kT: float,
                     q_start: torch.Tensor | None = None, tol: float = 1e-5, max_iter: int = 100,
                     rank_tol: float = 1e-2, max_rank: int = 8, k0: float = 0.1, complete: bool = True,
                     backtrack: int = 4, ewald: EwaldSetup | None = None, hubbard_U=HUBBARD_U,
                     mu_guess: float = 0.0, plan: bool = True, screened: bool = True, max_doublings: int = 20,
                     log=None) -> QuasiNewtonResult:
    """Kernel-accelerated SCF on the mixed-precision path.  Per step: begin
    the Krylov kernel with r = K0 f at the current solve (doubling history
    recorded), then for j = 0, 1, ...: the potential of v_j, its charge
    response dq_j, fit; stop the rank at a relative fit residual <= rank_tol
    (or max_rank); then n <- n - alpha (V c + complete (r - F_v c)) with
    alpha = 1, halved up to `backtrack` times while RMS(q0[n] - n) does not
    decrease (or no chemical potential matches the electron count).  The
    accepted trial's solve is the next step's.  Returns q0[n] at the first n
    with RMS(q0[n] - n) < tol."""
    from ._lib import GDMError
    ew = ewald if ewald is not None else ewald_setup(ctx, system)
    tau = slater_tau(hubbard_U) if screened else None
    N = system.n_atoms
    n = torch.zeros(N, dtype=torch.float64, device=ctx.dev) if q_start is None \
        else q_start.to(device=ctx.dev, dtype=torch.float64).clone()
    n_base = torch.empty_like(n)
    V = torch.empty_like(n)
    dV = torch.empty_like(n)
    dq = torch.empty_like(n)
    work = torch.empty(Context.krylov_work_size(N, max_rank), dtype=torch.float64, device=ctx.dev)
    res = QuasiNewtonResult(q=n, iterations=0, converged=False)
    state = {"cap": max_doublings}

    def evaluate(mu):
        """H[n] and the solve there; (None, None) when no chemical potential matches."""
        ctx.ewald_potential(system, ew.graph, ew.rcut, ew.eta, ew.k_max, hubbard_U, n, tau=tau, out=V)
        H, S = ctx.build_hs(system, tb, part.nbr, V)
        res.solves += 1
        try:
            sol = solve(ctx, system, part, H, S, kT, MIXED_F16, mu_guess=mu, plan=False)
            nd = ctx.mixed_stats()["n_doublings"]
            if nd > state["cap"]:
                # a wide spectrum (large potentials early in the iteration) took more
                # doublings than the history holds: grow it and solve again
                state["cap"] = nd + 2
                ctx.set_response(state["cap"])
                res.solves += 1
                sol = solve(ctx, system, part, H, S, kT, MIXED_F16, mu_guess=sol.mu, plan=False)
        except GDMError as e:
            if e.code != E_NO_BRACKET:
                raise
            return None, None
        return sol, S

    if plan:
        ctx.plan(part.sg, MIXED_F16)
    ctx.set_response(state["cap"])
    try:
        sol, S = evaluate(mu_guess)
        if sol is None:
            raise RuntimeError("scc_quasi_newton: no chemical potential at the starting charges")
        for it in range(1, max_iter + 1):
            rms = ctx.krylov_begin(n, sol.q, max_rank, work, k0)
            res.history.append(rms)
            res.iterations = it
            res.mu = sol.mu
            if rms < tol:
                res.q, res.converged = sol.q, True
                return res
            rank, rel = 0, 1.0
            for j in range(max_rank):
                v = Context.krylov_vector(work, N, j)
                ctx.ewald_potential(system, ew.graph, ew.rcut, ew.eta, ew.k_max, hubbard_U, v, tau=tau, out=dV)
                ctx.density_response(system, part.sg, part.nbr, S, dV, out=dq)
                res.responses += 1
                rel, exhausted = ctx.krylov_add(N, j, dq, max_rank, work)
                rank = j + 1
                if rel <= rank_tol or exhausted:
                    break
            res.ranks.append(rank)
            res.fits.append(rel)
            n_base.copy_(n)
            alpha = 1.0
            for k in range(backtrack + 1):
                n.copy_(n_base)
                ctx.krylov_apply(n, rank, max_rank, work, alpha, complete)
                trial, S_t = evaluate(sol.mu)
                rms_t = ctx.scc_mix(n, trial.q, 0.0) if trial is not None else math.inf
                if rms_t < rms or k == backtrack:
                    break
                alpha *= 0.5
            res.alphas.append(alpha)
            if log is not None:
                log(it, rms, rank, rel, alpha, sol.mu)
            if trial is None:
                break
            sol, S = trial, S_t
        res.q = n
        return res
    finally:
        ctx.set_response(0)


__all__ = ["HUBBARD_U", "slater_tau", "EwaldSetup", "ewald_setup", "SCCResult", "scc_loop", "QuasiNewtonResult",
           "scc_quasi_newton"]
