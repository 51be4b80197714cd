"""Charge response and the kernel-accelerated SCF (oracle; test infrastructure only).

Response (SI section B: the directional derivatives that build the low-rank
kernel, by quantum perturbation theory with fractional occupations).  A
change dV of the atomic potentials changes the SCC Hamiltonian of SI
section D by dH_ab = 1/2 s_ab (dV_I(a) + dV_J(b)).  In one subgraph, with
the generalized eigenpairs of the solve (h C = s C diag(lam), C^T s C = I)
and occupations f_k = f(lam_k - mu), first-order perturbation theory at
fixed mu gives

    dD = C (F o (C^T dH C)) C^T,   F_jk = (f_j - f_k) / (lam_j - lam_k),
                                   F_jk = -beta f_j (1 - f_j) when lam_j = lam_k,

and a shift dmu of the chemical potential adds dmu C diag(beta f (1 - f)) C^T
(d f / d mu).  The electron count is held fixed (canonical response): dmu is
chosen so that the collected charge changes sum to zero.  The charge
response is the Mulliken map of the collected core rows,
dq_I = 2 sum_{a in I} (dD s)_aa over core orbitals.

Kernel and SCF (SI sections B and C).  With the residual f(n) = q0[n] - n
and its Jacobian J (J v = dq[gamma v] - v, gamma the Coulomb map of
ewald.coulomb_potential, which is linear in the charges), a preconditioner
K0 ~ J^-1 and the orthonormalised preconditioned Krylov vectors
v_1 ~ K0 f, v_{j+1} ~ K0 J v_j (each orthogonalised against the earlier
ones), the low-rank kernel acting on r = K0 f is

    (K0 J)^-1 r ~ sum_ij v_i M_ij f_vj^T r,  f_vj = K0 J v_j,  M = O^-1,  O_ij = f_vi^T f_vj,

i.e. V c with c the least-squares solution of F_v c = r.  Vectors are added
until || F_v c - r || <= rank_tol || r || or the rank cap is hit.  K0 is
the scaled-delta kernel -c I.  With K0 ~ J^-1 the operator (K0 J)^-1 is
close to the identity, so on the part of r that the vectors do not fit
(r - F_v c, orthogonal to every f_v) it is taken as the identity: the step
is n <- n - alpha (V c + (r - F_v c)), exact Newton on the fitted subspace
and the plain preconditioned update K0 f on the rest (with a complete basis
the remainder vanishes and the step is the paper's).  alpha = 1, halved
while the residual norm does not decrease (at most 4 times), a
backtracking line search for starts far from the fixed point.

Pins (tests/test_oracle_response.py): the response equals central finite
differences of the full solve (solve.solve_system with mu re-solved) for
orthogonal and non-orthogonal models; the full-system susceptibility
dq_I / dV_J is symmetric; the response conserves charge; on an affine
charge map the quasi-Newton step with a full-rank kernel lands on the
closed-form fixed point in one step, a rank-m step is the minimiser over
the Krylov space, and the completed step adds exactly the unfitted
remainder; on a water box the SCF reaches the fixed point of the
Anderson-mixed SCC.
"""
from __future__ import annotations

import numpy as np

from .ewald import coulomb_potential, slater_short, slater_tau
from .model import COULOMB_EV_A, N_ORB, TBModel, dense_hs, min_image, r2_of
from .solve import fermi, solve_system


def delta_h(s: np.ndarray | None, dv_orb: np.ndarray) -> np.ndarray:
    """dH_ab = 1/2 s_ab (dv_a + dv_b) (s = I when orthogonal)."""
    if s is None:
        return np.diag(dv_orb)
    return 0.5 * s * (dv_orb[:, None] + dv_orb[None, :])


def occupation_differences(lam: np.ndarray, f: np.ndarray, beta: float, tie: float = 1e-9) -> np.ndarray:
    """F_jk = (f_j - f_k) / (lam_j - lam_k), and the derivative -beta f (1 - f)
    where the eigenvalues coincide (|lam_j - lam_k| <= tie)."""
    dl = lam[:, None] - lam[None, :]
    df = f[:, None] - f[None, :]
    deriv = -beta * f * (1.0 - f)
    close = np.abs(dl) <= tie
    F = np.where(close, 0.5 * (deriv[:, None] + deriv[None, :]), df / np.where(close, 1.0, dl))
    return F


def subgraph_response_rows(sol, s, dH: np.ndarray, mu: float, beta: float):
    """(dq at fixed mu, d pop / d mu) over the core orbitals of one subgraph:
    populations 2 (dD s)_aa of the core rows a."""
    C = sol.C
    f = fermi(sol.lam - mu, beta)
    F = occupation_differences(sol.lam, f, beta)
    H1 = C.T @ dH @ C
    dD_core = C[:sol.nc] @ (F * H1) @ C.T
    dmu_core = (C[:sol.nc] * (beta * f * (1.0 - f))) @ C.T
    s_core = sol.s_core
    return 2.0 * np.einsum("ab,ab->a", dD_core, s_core), 2.0 * np.einsum("ab,ab->a", dmu_core, s_core)


def charge_response(pos, species, L, model: TBModel, subs, V_atom, dV, mu=None, sols=None):
    """Canonical first-order change of the collected Mulliken charges for a
    change dV (eV per atom) of the atomic potentials at potentials V_atom.
    mu: the chemical potential of the unperturbed solve (None: found by
    bisection as in solve_system).  Returns (dq [N], dmu, mu)."""
    beta = model.beta
    if sols is None or mu is None:
        res = solve_system(pos, species, L, model, subs, V_atom=V_atom, workers=1)
        sols = res.sols
        mu = res.mu if mu is None else mu
    dq_mu0 = np.zeros(len(species))
    dq_mu1 = np.zeros(len(species))
    for (atoms, ncore), sol in zip(subs, sols):
        _, s = dense_hs(pos, species, L, model, atoms, V_atom)
        norb = N_ORB[species[atoms]]
        dv_orb = np.repeat(np.asarray(dV, dtype=np.float64)[atoms], norb)
        p0, p1 = subgraph_response_rows(sol, s, delta_h(s, dv_orb), mu, beta)
        owner = np.repeat(atoms[:ncore], N_ORB[species[atoms[:ncore]]])
        np.add.at(dq_mu0, owner, p0)
        np.add.at(dq_mu1, owner, p1)
    # canonical: sum dq = 0 fixes dmu
    t1 = dq_mu1.sum()
    dmu = -dq_mu0.sum() / t1 if t1 != 0.0 else 0.0
    return dq_mu0 + dmu * dq_mu1, dmu, mu


def krylov_step(f: np.ndarray, jv, rank_tol: float = 1e-2, max_rank: int = 8, k0=1.0,
                complete: bool = False):
    """Quasi-Newton update -(K0 J)^-1 K0 f from the low-rank preconditioned
    Krylov kernel with K0 = -k0 I (k0 a number) or K0 x = k0(x) (k0 a
    function, e.g. BlockPreconditioner.apply); complete=True adds the
    unfitted remainder -(r - F_v c).  jv(v) returns J v.  Returns (dn, rank,
    relative residual of the low-rank fit)."""
    precond = k0 if callable(k0) else (lambda x: -k0 * x)
    r = precond(f)
    nr = np.linalg.norm(r)
    if nr == 0.0:
        return np.zeros_like(f), 0, 0.0
    V, FV = [], []
    v = r / nr
    rel = 1.0
    c = np.zeros(0)
    for _ in range(max_rank):
        fv = precond(jv(v))                           # K0 J v
        V.append(v)
        FV.append(fv)
        Fm = np.stack(FV, axis=1)
        O = Fm.T @ Fm                                 # O_ij = f_vi . f_vj
        c = np.linalg.solve(O, Fm.T @ r)              # c = M F_v^T r
        rel = float(np.linalg.norm(Fm @ c - r) / nr)
        if rel <= rank_tol:
            break
        # next Krylov direction: f_v orthogonalised against the earlier v (twice)
        w = fv.copy()
        for _ in range(2):
            for u in V:
                w -= np.dot(u, w) * u
        nw = np.linalg.norm(w)
        if nw <= 1e-14 * np.linalg.norm(fv):
            break
        v = w / nw
    Fm = np.stack(FV, axis=1)
    dn = -np.stack(V, axis=1) @ c                     # n <- n - V c
    if complete:
        dn -= r - Fm @ c
    return dn, len(V), rel


class BlockPreconditioner:
    """Block-diagonal preconditioner K0 ~ J^-1 over the cores (SI sections B,
    C: low-rank updates combined with a block-diagonal preconditioner
    built on the graph).  For each core c, with its atoms in ascending
    order, K0_c = (chi_c G_c - I)^-1, where
      chi_c[:, j] = dq over the core's atoms for a unit potential on its j-th
        atom, probed for all cores at once (dV = 1 on the j-th core atom of
        every core; canonical response, charge_response);
      G_c = the charge-potential kernel inside the core: "local" gives
        U_I on the diagonal and k_e (1/r - S(tau_I, tau_J, r)) off it at the
        minimum image; "ewald" gives the periodic kernel of coulomb_potential
        restricted to the core (exact: with one core holding every atom and
        every atom probed alone, K0 = J^-1).
    apply(x) returns K0 x."""

    def __init__(self, subs, n_atoms: int):
        self.cores = [np.asarray(atoms[:nc], dtype=np.int64) for atoms, nc in subs]
        self.blocks = []
        self.n = n_atoms

    def apply(self, x: np.ndarray) -> np.ndarray:
        y = np.zeros(self.n)
        for idx, K in zip(self.cores, self.blocks):
            y[idx] = K @ x[idx]
        return y


def block_preconditioner(pos, species, L, model: TBModel, subs, V_atom, mu, sols, gamma: str = "local",
                         eta=None, n_real: int = 2, k_max: int = 8, short_cut: float = np.inf):
    U = np.asarray(model.hubbard_U)
    P = BlockPreconditioner(subs, len(species))
    width = max(len(c) for c in P.cores)
    chi = [np.zeros((len(c), len(c))) for c in P.cores]
    for j in range(width):
        dV = np.zeros(len(species))
        for c in P.cores:
            if j < len(c):
                dV[c[j]] = 1.0
        dq, _, _ = charge_response(pos, species, L, model, subs, V_atom, dV, mu=mu, sols=sols)
        for k, c in enumerate(P.cores):
            if j < len(c):
                chi[k][:, j] = dq[c]
    tau = slater_tau(U)
    for k, c in enumerate(P.cores):
        nc = len(c)
        if gamma == "ewald":
            G = np.zeros((nc, nc))
            for j in range(nc):
                e = np.zeros(len(species))
                e[c[j]] = 1.0
                G[:, j] = coulomb_potential(pos, species, e, L, U, eta=eta, n_real=n_real, k_max=k_max,
                                            short_cut=short_cut)[c]
        else:
            d = min_image(pos[c][None, :, :] - pos[c][:, None, :], L, 1.0 / L)
            r = np.sqrt(r2_of(d))
            G = np.zeros((nc, nc))
            for a in range(nc):
                for b in range(nc):
                    if a == b:
                        G[a, b] = U[species[c[a]]]
                    else:
                        G[a, b] = COULOMB_EV_A * (1.0 / r[a, b]
                                                  - slater_short(tau[species[c[a]]], tau[species[c[b]]], r[a, b]))
        P.blocks.append(np.linalg.inv(chi[k] @ G - np.eye(nc)))
    return P


def quasi_newton(charge_map, jacobian_vector, n0, tol: float = 1e-5, max_iter: int = 100,
                 rank_tol: float = 1e-2, max_rank: int = 8, k0=1.0, complete: bool = False,
                 backtrack: int = 0, make_k0=None):
    """Kernel-accelerated SCF: n <- n - alpha (K0 J)^-1 K0 f(n).  charge_map(n)
    returns q0[n] (or raises ArithmeticError where it has no solution);
    jacobian_vector(n, v) returns J(n) v at the n of the last accepted
    charge_map call.  backtrack: halvings of alpha allowed while RMS(f) does
    not decrease.  Stops at RMS(f) < tol.  Returns (q0 at the converged n,
    iterations, residual history, ranks, converged)."""
    n = np.array(n0, dtype=np.float64)
    hist, ranks = [], []
    q = charge_map(n)
    f = q - n
    rms = float(np.sqrt(np.mean(f * f)))
    if make_k0 is not None:          # preconditioner built once, at the starting charges
        k0 = make_k0()
    for it in range(1, max_iter + 1):
        hist.append(rms)
        if rms < tol:
            return q, it, hist, ranks, True
        dn, rank, _ = krylov_step(f, lambda v: jacobian_vector(n, v), rank_tol, max_rank, k0, complete)
        ranks.append(rank)
        alpha = 1.0
        for k in range(backtrack + 1):
            n_try = n + alpha * dn
            try:
                q_try = charge_map(n_try)
                f_try = q_try - n_try
                rms_try = float(np.sqrt(np.mean(f_try * f_try)))
            except ArithmeticError:
                rms_try = np.inf
            if rms_try < rms or k == backtrack:
                break
            alpha *= 0.5
        if not np.isfinite(rms_try):
            break
        n, q, f, rms = n_try, q_try, f_try, rms_try
    return n, max_iter, hist, ranks, False


def scc_quasi_newton(pos, species, L, model: TBModel, subs, q_start=None, tol: float = 1e-5,
                     max_iter: int = 100, rank_tol: float = 1e-2, max_rank: int = 8, k0: float = 0.1,
                     complete: bool = True, backtrack: int = 4, eta=None, n_real: int = 2, k_max: int = 8,
                     short_cut: float = np.inf, block: bool = False):
    """The SCC problem of scc.scc solved by the quasi-Newton iteration, the
    Jacobian-vector products from charge_response; block=True uses the
    block-diagonal preconditioner (local kernel) built at the start instead
    of K0 = -k0 I.  Returns (q, iterations, residual history, ranks)."""
    U = np.asarray(model.hubbard_U)

    def gamma(q):
        return coulomb_potential(pos, species, q, L, U, eta=eta, n_real=n_real, k_max=k_max, short_cut=short_cut)

    state = {}

    def charge_map(n):
        V = gamma(n)
        res = solve_system(pos, species, L, model, subs, V_atom=V)
        state.update(n=n, V=V, sols=res.sols, mu=res.mu)
        return res.q

    def jacobian_vector(n, v):
        assert state["n"] is n
        dq, _, _ = charge_response(pos, species, L, model, subs, state["V"], gamma(v), mu=state["mu"],
                                   sols=state["sols"])
        return dq - v

    def make_k0():
        return block_preconditioner(pos, species, L, model, subs, state["V"], state["mu"], state["sols"]).apply

    n0 = np.zeros(len(species)) if q_start is None else q_start
    q, it, hist, ranks, _ = quasi_newton(charge_map, jacobian_vector, n0, tol=tol, max_iter=max_iter,
                                         rank_tol=rank_tol, max_rank=max_rank, k0=k0, complete=complete,
                                         backtrack=backtrack, make_k0=make_k0 if block else None)
    return q, it, hist, ranks
