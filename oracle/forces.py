"""Shadow Born-Oppenheimer potential and its forces (oracle; test
infrastructure only).

What is computed (Shadow MD section, Eqs. Shadow_Energy and shadow_min and
the nuclear equation of motion NEQ; SCC-TB form of SI section D):

* For a charge vector n the Coulomb potential is V[n] = gamma n (Ewald sum
  plus the on-site U, ewald.coulomb_potential) and H[n] = H0 + 1/2 S (V_I +
  V_J).  The linearised energy functional, equilibrated in one step, gives
  the density matrix D of H[n] at the mu that fixes the electron count (the
  subgraph solve of solve.py) and the shadow potential

      U(R, n) = Omega(H[n]) - sum_I (N0_I + n_I / 2) V_I[n] + E_rep(R),
      Omega   = 2 sum_s sum_k w_k [f_k lam_k + kT (f_k ln f_k + (1 - f_k) ln(1 - f_k))],

  the electronic free energy (band energy and entropy) of H[n] collected
  with the core weights w_k of each subgraph.  With q the Mulliken charges
  of D this equals 2 Tr[H0 D] - T S + q^T gamma n - n^T gamma n / 2 + E_rep,
  the second-order SCC energy linearised around n, and at the
  self-consistent n = q it equals the SCC free energy itself.
* Forces at fixed n (Eq. NEQ), F_I = -dU/dR_I:
    - band: -2 Tr[D dH[n]/dR] + 2 Tr[W dS/dR] at fixed V (the free energy is
      stationary in the occupations at fixed electron count), with the
      energy-weighted density W = C diag(f lam) C^T.  Only off-diagonal atom
      blocks depend on the positions; for a neighbour pair I != J with
      d = R_J - R_I the pair term is
          e_IJ(d) = 4 sum_{a in I, b in J} [Dbar_ab (H0_ab + S_ab (V_I + V_J)/2) - Wbar_ab S_ab],
      Dbar = (D_IJ + D_JI^T)/2 from the core rows of I's and J's subgraphs
      (blocks of atoms outside a subgraph are zero), and F_I += grad_d e_IJ;
    - Coulomb: the position dependence of gamma, -d/dR [1/2 (2q - n)^T gamma n]
      (ewald.coulomb_forces);
    - repulsion: F_I += grad_d of A_pair exp(-r/rho) t(r).
  Slater-Koster derivatives: with u = d/r, dr/dd = u and du_a/dd_c =
  (delta_ac - u_a u_c)/r; the angular factor g of [s, s], [s, p_b],
  [p_a, s], [p_a, p_b] is 1, u_b, -u_a, u_a u_b.

Pins (tests/test_oracle_forces.py): the Slater-Koster blocks equal those of
model.dense_hs; their gradients and the taper's match central differences
and the taper has continuous value, slope and curvature at both ends; the
total force equals the central difference of U(R, n) at fixed n on a
non-orthogonal SCC system with taper and repulsion; forces sum to zero; the
partitioned forces with full halos equal the full-system ones; U(R, n)
differs from the SCC free energy by a term quadratic in q[n] - n (Eq. UErr);
the repulsion prefactors put an isolated water's SCC forces to zero at its
reference geometry.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ewald import coulomb_forces, coulomb_potential
from .model import N_ORB, N_VALENCE, TBModel, min_image, neighbour_list, r2_of, repulsion_energy, taper
from .solve import SystemResult, fermi, solve_system


def taper_deriv(r, r_on: float, r_c: float):
    """dt/dr of model.taper: -30 x^2 (1 - x)^2 / (r_c - r_on) inside [r_on, r_c]."""
    w = r_c - r_on
    x = np.clip((np.asarray(r, dtype=np.float64) - r_on) / w, 0.0, 1.0)
    return -30.0 * x * x * (1.0 - x) ** 2 / w


def radial(r: float, amp: float, r0: float, decay: float, model: TBModel):
    """amp exp(-(r - r0)/decay) t(r) and its derivative in r."""
    e = amp * np.exp(-(r - r0) / decay)
    de = -e / decay
    if model.taper_on > 0:
        t, dt = taper(r, model.taper_on, model.cutoff), taper_deriv(r, model.taper_on, model.cutoff)
        return float(e * t), float(de * t + e * dt)
    return float(e), float(de)


def sk_block(d: np.ndarray, si: int, sj: int, model: TBModel):
    """Two-centre blocks of a pair with d = R_J - R_I (r < cutoff): h0 [ni, nj],
    s [ni, nj] and their gradients with respect to d, [3, ni, nj] each."""
    r = float(np.sqrt(r2_of(d)))
    u = d / r
    V, dV = radial(r, model.v0, model.v_r0, model.v_decay, model)
    Sr, dSr = radial(r, model.s0, model.s_r0, model.s_decay, model)
    ni, nj = int(N_ORB[si]), int(N_ORB[sj])
    proj = (np.eye(3) - np.outer(u, u)) / r           # du_a/dd_c = proj[a, c]
    g = np.zeros((ni, nj))
    dg = np.zeros((3, ni, nj))
    for a in range(ni):
        for b in range(nj):
            if a == 0 and b == 0:
                g[a, b] = 1.0
            elif a == 0:
                g[a, b] = u[b - 1]
                dg[:, a, b] = proj[b - 1]
            elif b == 0:
                g[a, b] = -u[a - 1]
                dg[:, a, b] = -proj[a - 1]
            else:
                g[a, b] = u[a - 1] * u[b - 1]
                dg[:, a, b] = proj[a - 1] * u[b - 1] + u[a - 1] * proj[b - 1]
    h = V * g
    dh = dV * u[:, None, None] * g[None] + V * dg
    if model.orthogonal:
        return h, np.zeros_like(h), dh, np.zeros_like(dh)
    s = Sr * g
    ds = dSr * u[:, None, None] * g[None] + Sr * dg
    return h, s, dh, ds


def entropy_term(f: np.ndarray) -> np.ndarray:
    """f ln f + (1 - f) ln(1 - f), with 0 ln 0 = 0."""
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    m = (f > 0) & (f < 1)
    out[m] = f[m] * np.log(f[m]) + (1.0 - f[m]) * np.log1p(-f[m])
    return out


def band_free_energy(sols, mu: float, beta: float) -> float:
    """Omega = 2 sum_s sum_k w_k [f lam + kT (f ln f + (1 - f) ln(1 - f))]."""
    tot = 0.0
    for s in sols:
        f = fermi(s.lam - mu, beta)
        tot += 2.0 * float(np.dot(s.w, f * s.lam + entropy_term(f) / beta))
    return tot


def edm_core_rows(sol, mu: float, beta: float) -> np.ndarray:
    """Energy-weighted core rows W[core, :] = C[core, :] diag(f lam) C^T."""
    f = fermi(sol.lam - mu, beta)
    return (sol.C[:sol.nc] * (f * sol.lam)) @ sol.C.T


def core_blocks(subs, rows, species: np.ndarray, rp: np.ndarray, col: np.ndarray) -> dict:
    """{(I, J): block [nI, nJ]} of the collected core rows `rows` (per
    subgraph [nc, n]) for every neighbour pair (I, J) of the CSR (I the core
    atom); zero where J is outside I's subgraph."""
    out = {}
    for (atoms, ncore), R in zip(subs, rows):
        atoms = np.asarray(atoms)
        norb = N_ORB[species[atoms]]
        off = np.concatenate([[0], np.cumsum(norb)])
        local = {int(a): k for k, a in enumerate(atoms)}
        for p in range(ncore):
            I = int(atoms[p])
            for J in col[rp[I]:rp[I + 1]]:
                J = int(J)
                k = local.get(J)
                blk = np.zeros((norb[p], N_ORB[species[J]]))
                if k is not None:
                    blk = R[off[p]:off[p + 1], off[k]:off[k + 1]]
                out[(I, J)] = np.array(blk)
    return out


def band_forces(pos, species, L, model: TBModel, rp, col, Dblk: dict, Wblk: dict, V_atom=None) -> np.ndarray:
    """F_I = sum over neighbours J of grad_d e_IJ (module docstring)."""
    n = len(species)
    F = np.zeros((n, 3))
    inv_L = 1.0 / L
    for I in range(n):
        for J in col[rp[I]:rp[I + 1]]:
            J = int(J)
            d = min_image(pos[J] - pos[I], L, inv_L)
            _, _, dh, ds = sk_block(d, int(species[I]), int(species[J]), model)
            Db = 0.5 * (Dblk[(I, J)] + Dblk[(J, I)].T)
            Wb = 0.5 * (Wblk[(I, J)] + Wblk[(J, I)].T)
            vs = 0.0 if V_atom is None else 0.5 * (V_atom[I] + V_atom[J])
            XH = 4.0 * Db
            XS = 4.0 * (Db * vs - Wb)
            F[I] += np.einsum("ab,xab->x", XH, dh) + np.einsum("ab,xab->x", XS, ds)
    return F


def repulsion_forces(pos, species, L, model: TBModel) -> np.ndarray:
    """F_I = sum_J grad_d [A exp(-r/rho) t(r)] = sum_J e'(r) u."""
    n = len(species)
    F = np.zeros((n, 3))
    rp, col = neighbour_list(pos, L, model.cutoff)
    A = np.asarray(model.rep_A, dtype=np.float64)
    for I in range(n):
        for J in col[rp[I]:rp[I + 1]]:
            d = min_image(pos[J] - pos[I], L, 1.0 / L)
            r = float(np.sqrt(r2_of(d)))
            e = A[species[I] + species[J]] * np.exp(-r / model.rep_rho)
            de = -e / model.rep_rho
            if model.taper_on > 0:
                t, dt = taper(r, model.taper_on, model.cutoff), taper_deriv(r, model.taper_on, model.cutoff)
                de, e = de * t + e * dt, e * t
            F[I] += de * d / r
    return F


@dataclass
class Ewald:
    """Splitting and truncation of the Ewald sums (ewald.coulomb_potential)."""
    eta: float
    n_real: int = 2
    k_max: int = 8
    screened: bool = True
    short_cut: float = np.inf       # screening over pairs closer than this (A)


@dataclass
class ShadowResult:
    U: float                 # shadow potential (eV)
    F: np.ndarray            # [N, 3] eV/A
    q: np.ndarray            # Mulliken charges q[n]
    n: np.ndarray            # the extended charges n
    V: np.ndarray            # V[n]
    omega: float
    e_rep: float
    system: SystemResult


def shadow_point(pos, species, L, model: TBModel, subs, n: np.ndarray, ew: Ewald,
                 forces: bool = True) -> ShadowResult:
    """U(R, n), its forces at fixed n and q[n] for the subgraph set `subs`
    (a single subgraph of every atom for the full system)."""
    U_h = np.asarray(model.hubbard_U)
    V = coulomb_potential(pos, species, n, L, U_h, eta=ew.eta, n_real=ew.n_real, k_max=ew.k_max,
                          screened=ew.screened, short_cut=ew.short_cut)
    res = solve_system(pos, species, L, model, subs, V_atom=V)
    beta = model.beta
    omega = band_free_energy(res.sols, res.mu, beta)
    e_rep = repulsion_energy(pos, species, L, model) if any(model.rep_A) else 0.0
    U = omega - float(np.dot(N_VALENCE[species] + 0.5 * n, V)) + e_rep
    F = None
    if forces:
        rp, col = neighbour_list(pos, L, model.cutoff)
        w_rows = [edm_core_rows(s, res.mu, beta) for s in res.sols]
        Dblk = core_blocks(subs, res.d_core, species, rp, col)
        Wblk = core_blocks(subs, w_rows, species, rp, col)
        F = band_forces(pos, species, L, model, rp, col, Dblk, Wblk, V)
        F += coulomb_forces(pos, species, 2.0 * res.q - n, n, L, U_h, eta=ew.eta, n_real=ew.n_real,
                            k_max=ew.k_max, screened=ew.screened, short_cut=ew.short_cut)
        if any(model.rep_A):
            F += repulsion_forces(pos, species, L, model)
    return ShadowResult(U=U, F=F, q=res.q, n=np.array(n, dtype=np.float64), V=V, omega=omega, e_rep=e_rep,
                        system=res)


def whole(n_atoms: int):
    """The subgraph set of a full-system solve: one subgraph, every atom core."""
    return [(np.arange(n_atoms, dtype=np.int64), n_atoms)]
