"""Subgraph density matrices, global chemical potential and charges (oracle).

What is computed (Graph-Based Linear-Scaling section, Eqs. 1-3; SI A, D):

* For each core+halo subgraph with principal submatrices h, s, the dense
  Fermi-operator density matrix D = Z f(Z^T h Z) Z^T with Z = s^(-1/2)
  (the paper assumes S = I and defers the basis change; any Z with
  Z Z^T = s^-1 gives the same D).  f(x) = 1 / (1 + exp(beta (x - mu))).
  Here: eigh(s) -> Z, eigh(Z h Z) = Q diag(lam) Q^T, C = Z Q.
* D is per spin (occupations in [0, 1]); the electron count is
  N(mu) = 2 sum_s sum_k w_k f(lam_k) with core weights
  w_k = sum_{a in core} C_ak (s C)_ak.  mu solves N(mu) = N_e, found by
  bisection on [min lam - 1, max lam + 1]: if N(mid) < N_e then lo = mid else
  hi = mid, until hi - lo <= 1e-12 eV or 200 steps; mu = (lo + hi)/2.
* Collected core rows D[core, :] = C[core, :] diag(f) C^T (Eq. 3).
* Mulliken populations pop_a = 2 sum_b D_ab s_ba for core orbitals a, and
  net Mulliken electron charges q_I = sum_{a in I} pop_a - N_I^0 (SI D).

Pins: full-halo subgraphs equal full-system diagonalisation; 2 Tr[D S] = N_e
and sum q = 0 at mu; the 2x2 dimer closed form; Hermiticity and
idempotency as kT -> 0; the single water equals a generalized eigensolve;
Z = s^-1/2 and Z = L^-T give the same D (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from .model import N_ORB, N_VALENCE, TBModel, dense_hs, orbital_layout


def fermi(x: np.ndarray, beta: float) -> np.ndarray:
    """1 / (1 + exp(beta x)) evaluated without overflow."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    p = x > 0
    e = np.exp(-beta * x[p])
    out[p] = e / (1.0 + e)
    e = np.exp(beta * x[~p])
    out[~p] = 1.0 / (1.0 + e)
    return out


@dataclass
class SubgraphSolution:
    lam: np.ndarray        # [n] eigenvalues of Z h Z
    C: np.ndarray          # [n, n] generalized eigenvectors (columns)
    w: np.ndarray          # [n] core weights
    nc: int                # number of core orbitals
    s_core: np.ndarray     # [nc, n] core rows of s (identity rows if orthogonal)


def inv_sqrt_spd(s: np.ndarray) -> np.ndarray:
    sv, U = np.linalg.eigh(s)
    if sv[0] <= 0:
        raise np.linalg.LinAlgError("overlap matrix is not positive definite")
    return (U * sv ** -0.5) @ U.T


def solve_subgraph(h: np.ndarray, s: np.ndarray | None, nc: int, z: str = "invsqrt") -> SubgraphSolution:
    n = h.shape[0]
    if s is None:
        Z = np.eye(n)
        s_eff = np.eye(n)
    else:
        s_eff = s
        if z == "invsqrt":
            Z = inv_sqrt_spd(s)
        elif z == "cholesky":
            L = np.linalg.cholesky(s)
            Z = np.linalg.inv(L).T
        else:
            raise ValueError(z)
    hp = Z.T @ h @ Z
    lam, Q = np.linalg.eigh(hp)
    C = Z @ Q
    sC = s_eff @ C
    w = np.einsum("ak,ak->k", C[:nc], sC[:nc])
    return SubgraphSolution(lam=lam, C=C, w=w, nc=nc, s_core=np.array(s_eff[:nc]))


def electron_count(sols, mu: float, beta: float) -> float:
    return float(sum(2.0 * np.dot(s.w, fermi(s.lam - mu, beta)) for s in sols))


def find_mu(sols, n_e: float, beta: float, tol: float = 1e-12, maxit: int = 200) -> float:
    lam_all = np.concatenate([s.lam for s in sols])
    w_all = np.concatenate([s.w for s in sols])
    lo, hi = lam_all.min() - 1.0, lam_all.max() + 1.0
    for _ in range(maxit):
        mid = 0.5 * (lo + hi)
        n_mid = 2.0 * np.dot(w_all, fermi(lam_all - mid, beta))
        if n_mid < n_e:
            lo = mid
        else:
            hi = mid
        if hi - lo <= tol:
            break
    return 0.5 * (lo + hi)


def d_core_rows(sol: SubgraphSolution, mu: float, beta: float) -> np.ndarray:
    f = fermi(sol.lam - mu, beta)
    return (sol.C[:sol.nc] * f) @ sol.C.T


def mulliken_pop(D_core: np.ndarray, s_core: np.ndarray) -> np.ndarray:
    """pop_a = 2 sum_b D_ab s_ba for the core orbitals a (s symmetric)."""
    return 2.0 * np.einsum("ab,ab->a", D_core, s_core)


def charges_from_pops(subs, pops, species: np.ndarray) -> np.ndarray:
    q = -N_VALENCE[species].astype(np.float64)
    for (atoms, ncore), pop in zip(subs, pops):
        norb = N_ORB[species[atoms[:ncore]]]
        owner = np.repeat(atoms[:ncore], norb)
        np.add.at(q, owner, pop)
    return q


@dataclass
class SystemResult:
    mu: float
    n_count: float
    sols: list
    d_core: list           # per subgraph [nc, n]
    q: np.ndarray          # [N]
    subs: list


def _workers() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def solve_subgraphs(pos, species, L, model: TBModel, subs, V_atom=None, workers: int | None = None,
                    z: str = "invsqrt"):
    """eigen-solutions of every subgraph (thread pool over subgraphs, 1 BLAS thread each)."""
    def one(sub):
        atoms, ncore = sub
        h, s = dense_hs(pos, species, L, model, atoms, V_atom)
        nc = int(N_ORB[species[atoms[:ncore]]].sum())
        return solve_subgraph(h, s, nc, z=z)

    workers = workers or _workers()
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        if workers == 1:
            return [one(s) for s in subs]
        with ThreadPoolExecutor(workers) as ex:
            return list(ex.map(one, subs))


def solve_system(pos, species, L, model: TBModel, subs, V_atom=None, workers=None, n_e=None,
                 z: str = "invsqrt") -> SystemResult:
    sols = solve_subgraphs(pos, species, L, model, subs, V_atom, workers, z=z)
    n_e = float(N_VALENCE[species].sum()) if n_e is None else n_e
    beta = model.beta
    mu = find_mu(sols, n_e, beta)
    dcs = [d_core_rows(s, mu, beta) for s in sols]
    pops = [mulliken_pop(d, s.s_core) for d, s in zip(dcs, sols)]
    q = charges_from_pops(subs, pops, species)
    return SystemResult(mu=mu, n_count=electron_count(sols, mu, beta), sols=sols, d_core=dcs, q=q, subs=subs)


def full_system(pos, species, L, model: TBModel, V_atom=None) -> SystemResult:
    """The whole system as one subgraph whose core is every atom."""
    n = len(species)
    subs = [(np.arange(n, dtype=np.int64), n)]
    return solve_system(pos, species, L, model, subs, V_atom, workers=1)
