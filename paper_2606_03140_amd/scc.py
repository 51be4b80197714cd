"""Self-consistent-charge loop over the libgdm kernels.

The charge vector n of SI section D is iterated to self-consistency: the
Coulomb potential V = gamma n (periodic Ewald sum, screened at short range
by the interaction of exponential charge densities, Hubbard U on site:
gdm_ewald_potential) shifts H by 1/2 S_ab (V_I + V_J) (gdm_build_hs), one
density solve at a global mu gives the Mulliken charges q0[n], and the
update moves n towards the fixed point q0[n] = n: Anderson acceleration
(memory 8, mixing 0.03, gdm_scc_anderson) by default, or the scaled-delta
kernel K = -c I of the Shadow MD section (linear mixing, gdm_scc_mix).
Iteration stops when the RMS residual is below the tolerance.  Only
orchestration lives here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from ._lib import FP64_EIG, Context, Graph, System, TBParams
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


__all__ = ["HUBBARD_U", "slater_tau", "EwaldSetup", "ewald_setup", "SCCResult", "scc_loop"]
