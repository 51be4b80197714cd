"""Periodic charge-charge interaction for the SCC Hamiltonian (oracle).

The SCC-DFTB engine couples net Mulliken charges through a Coulomb
interaction that decays as 1/R at large separation and is screened at
short range, where the interacting charge densities overlap, with the
on-site value set by the Hubbard U (SI section D; the paper uses a GPU
Ewald solver for the all-to-all sum, Scalability section).  Here:

  V_I = U_I q_I + k_e [ sum_J q_J psi(R_J - R_I) ]
        - k_e sum_{J, images, (J, n) != (I, 0)} q_J S(tau_I, tau_J, |R_J - R_I + nL|)
  psi(r) = sum_n' erfc(eta |r + nL|)/|r + nL|
         + (4 pi / V) sum_{k != 0} exp(-k^2 / (4 eta^2)) / k^2 cos(k . r)
         - 2 eta / sqrt(pi) [r = 0],
  the n' sum skipping the J = I, n = 0 term, with k_e = 14.399645 eV A and
  a neutralising background (k = 0 term dropped), the screening sum taken
  over pairs closer than a cutoff (its tail is below 1e-12 eV beyond 12 A).
  gamma = 1/R - S(R) is the
  Coulomb energy of two normalised exponential (Slater 1s) charge densities
  with exponents tau = 16/5 U (atomic units), the screening of SCC-DFTB:
  gamma -> U as R -> 0 and S decays exponentially.

Pins: the rock-salt Madelung constant 1.747565 and independence of the
splitting parameter eta; the closed form of S against direct numerical
quadrature of the two-density Coulomb integral, and gamma(0) = U
(tests/test_oracle_pins.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .model import COULOMB_EV_A, HARTREE_EV

BOHR_A = 0.529177210903


def ewald_psi_matrix(pos: np.ndarray, L: float, eta: float, n_real: int, k_max: int) -> np.ndarray:
    """Dense [N, N] periodic 1/r kernel (including the self-image row terms)."""
    n = pos.shape[0]
    d = pos[None, :, :] - pos[:, None, :]
    psi = np.zeros((n, n))
    rng = range(-n_real, n_real + 1)
    for a in rng:
        for b in rng:
            for c in rng:
                sh = np.array([a, b, c], dtype=np.float64) * L
                r = np.linalg.norm(d + sh, axis=2)
                if a == 0 and b == 0 and c == 0:
                    np.fill_diagonal(r, np.inf)
                psi += erfc(eta * r) / r
    V = L ** 3
    ks = []
    for a in range(-k_max, k_max + 1):
        for b in range(-k_max, k_max + 1):
            for c in range(-k_max, k_max + 1):
                if a == 0 and b == 0 and c == 0:
                    continue
                ks.append((a, b, c))
    ks = np.array(ks, dtype=np.float64) * (2.0 * math.pi / L)
    k2 = (ks ** 2).sum(axis=1)
    coef = (4.0 * math.pi / V) * np.exp(-k2 / (4.0 * eta * eta)) / k2
    phase = pos @ ks.T                                   # [N, K]
    c, s = np.cos(phase), np.sin(phase)
    psi += (c * coef) @ c.T + (s * coef) @ s.T           # cos(k.(rj - ri))
    psi -= np.eye(n) * (2.0 * eta / math.sqrt(math.pi))
    return psi


def slater_tau(U_ev) -> np.ndarray:
    """Exponent of the Slater charge density of each species, 1/A, from the
    Hubbard U in eV: tau = 16/5 U in atomic units."""
    return 16.0 / 5.0 * (np.asarray(U_ev, dtype=np.float64) / HARTREE_EV) / BOHR_A


def slater_short(ta: float, tb: float, R):
    """S(R) with gamma(R) = 1/R - S(R) the Coulomb energy of two unit
    exponential densities tau^3/(8 pi) exp(-tau r) at distance R > 0 (any
    consistent length unit: S and 1/R in 1/length)."""
    R = np.asarray(R, dtype=np.float64)
    if abs(ta - tb) < 1e-6 * (ta + tb):
        t = 0.5 * (ta + tb)
        return np.exp(-t * R) * (1.0 / R + 11.0 * t / 16.0 + 3.0 * t * t * R / 16.0 + t ** 3 * R * R / 48.0)

    def part(a, b):
        d = a * a - b * b
        return np.exp(-a * R) * (b ** 4 * a / (2.0 * d * d) - (b ** 6 - 3.0 * b ** 4 * a * a) / (d ** 3 * R))

    return part(ta, tb) + part(tb, ta)


def short_range_matrix(pos: np.ndarray, species: np.ndarray, L: float, tau: np.ndarray, n_real: int,
                       short_cut: float = np.inf) -> np.ndarray:
    """Dense [N, N] sum over images of S(tau_I, tau_J, |R_J - R_I + nL|) for
    distances below short_cut, skipping J = I, n = 0."""
    n = pos.shape[0]
    d = pos[None, :, :] - pos[:, None, :]
    out = np.zeros((n, n))
    rng = range(-n_real, n_real + 1)
    pair = [(si, sj, (species[:, None] == si) & (species[None, :] == sj)) for si in (0, 1) for sj in (0, 1)]
    for a in rng:
        for b in rng:
            for c in rng:
                r = np.linalg.norm(d + np.array([a, b, c], dtype=np.float64) * L, axis=2)
                if a == 0 and b == 0 and c == 0:
                    np.fill_diagonal(r, np.inf)
                for si, sj, m in pair:
                    mm = m & (r < short_cut)
                    if mm.any():
                        out[mm] += slater_short(tau[si], tau[sj], r[mm])
    return out


def coulomb_potential(pos: np.ndarray, species: np.ndarray, q: np.ndarray, L: float, U: np.ndarray,
                      eta: float | None = None, n_real: int = 2, k_max: int = 8,
                      screened: bool = True, short_cut: float = np.inf) -> np.ndarray:
    """V [N] in eV; the screening term covers pairs closer than short_cut (A)."""
    eta = eta if eta is not None else 5.6 / L
    psi = ewald_psi_matrix(pos, L, eta, n_real, k_max)
    if screened:
        psi = psi - short_range_matrix(pos, species, L, slater_tau(U), n_real, short_cut)
    return U[species] * q + COULOMB_EV_A * (psi @ q)


def madelung_nacl(eta: float, n_real: int = 3, k_max: int = 8) -> float:
    """Madelung constant of rock salt from the Ewald kernel (unit cell of side 2,
    nearest-neighbour distance 1, charges +-1)."""
    pts, qs = [], []
    for a in range(2):
        for b in range(2):
            for c in range(2):
                pts.append((a, b, c))
                qs.append(1.0 if (a + b + c) % 2 == 0 else -1.0)
    pts = np.array(pts, dtype=np.float64)
    qs = np.array(qs)
    psi = ewald_psi_matrix(pts, 2.0, eta, n_real, k_max)
    phi0 = psi[0] @ qs
    return float(-phi0 * 1.0)      # potential at a + site is -M / r0 with r0 = 1


def slater_short_deriv(ta: float, tb: float, R):
    """dS/dR of slater_short, by differentiating its closed form term by term."""
    R = np.asarray(R, dtype=np.float64)
    if abs(ta - tb) < 1e-6 * (ta + tb):
        t = 0.5 * (ta + tb)
        p = 1.0 / R + 11.0 * t / 16.0 + 3.0 * t * t * R / 16.0 + t ** 3 * R * R / 48.0
        dp = -1.0 / (R * R) + 3.0 * t * t / 16.0 + t ** 3 * R / 24.0
        return np.exp(-t * R) * (dp - t * p)

    def part(a, b):
        d = a * a - b * b
        A = b ** 4 * a / (2.0 * d * d)
        B = (b ** 6 - 3.0 * b ** 4 * a * a) / d ** 3
        return np.exp(-a * R) * (-a * (A - B / R) + B / (R * R))

    return part(ta, tb) + part(tb, ta)


def kernel_gradient(pos: np.ndarray, species: np.ndarray, L: float, eta: float, n_real: int, k_max: int,
                    tau: np.ndarray | None = None, short_cut: float = np.inf) -> np.ndarray:
    """G[K, J, :] = gradient of the site-site kernel psi(d) - sum_images S(|d + nL|)
    with respect to d = R_J - R_K (the kernel of coulomb_potential without k_e
    and without the on-site U, which does not depend on the positions); the
    screening part only when tau is given.  Dense [N, N, 3]."""
    n = pos.shape[0]
    d = pos[None, :, :] - pos[:, None, :]
    G = np.zeros((n, n, 3))
    rng = range(-n_real, n_real + 1)
    two_over_sqrt_pi = 2.0 / math.sqrt(math.pi)
    for a in rng:
        for b in rng:
            for c in rng:
                dd = d + np.array([a, b, c], dtype=np.float64) * L
                r = np.linalg.norm(dd, axis=2)
                m = np.ones((n, n), dtype=bool)
                if a == 0 and b == 0 and c == 0:
                    np.fill_diagonal(m, False)
                rr = r[m]
                # d/dr [erfc(eta r)/r]
                gp = -erfc(eta * rr) / (rr * rr) - two_over_sqrt_pi * eta * np.exp(-(eta * rr) ** 2) / rr
                if tau is not None:
                    for si in (0, 1):
                        for sj in (0, 1):
                            pm = (species[:, None] == si) & (species[None, :] == sj)
                            sel = pm[m] & (rr < short_cut)
                            gp[sel] -= slater_short_deriv(tau[si], tau[sj], rr[sel])
                G[m] += (gp / rr)[:, None] * dd[m]
    V = L ** 3
    ks = []
    for a in range(-k_max, k_max + 1):
        for b in range(-k_max, k_max + 1):
            for c in range(-k_max, k_max + 1):
                if a == 0 and b == 0 and c == 0:
                    continue
                ks.append((a, b, c))
    ks = np.array(ks, dtype=np.float64) * (2.0 * math.pi / L)
    k2 = (ks ** 2).sum(axis=1)
    coef = (4.0 * math.pi / V) * np.exp(-k2 / (4.0 * eta * eta)) / k2
    phase = pos @ ks.T
    cs, sn = np.cos(phase), np.sin(phase)
    # d/dd cos(k.d) = -k sin(k.d), sin(k.(R_J - R_K)) = s_J c_K - c_J s_K
    for x in range(3):
        w = coef * ks[:, x]
        G[:, :, x] -= (cs * w) @ sn.T - (sn * w) @ cs.T
    return G


def coulomb_pair_energy(pos: np.ndarray, species: np.ndarray, a: np.ndarray, b: np.ndarray, L: float,
                        U: np.ndarray, eta: float | None = None, n_real: int = 2, k_max: int = 8,
                        screened: bool = True, short_cut: float = np.inf) -> float:
    """1/2 a^T gamma b with gamma the kernel of coulomb_potential (eV)."""
    return 0.5 * float(np.dot(a, coulomb_potential(pos, species, b, L, U, eta=eta, n_real=n_real, k_max=k_max,
                                                   screened=screened, short_cut=short_cut)))


def coulomb_forces(pos: np.ndarray, species: np.ndarray, a: np.ndarray, b: np.ndarray, L: float, U: np.ndarray,
                   eta: float | None = None, n_real: int = 2, k_max: int = 8, screened: bool = True,
                   short_cut: float = np.inf) -> np.ndarray:
    """F_K = -d/dR_K (1/2 a^T gamma b) [N, 3] in eV/A.  gamma_KJ depends on
    R_J - R_K, so F_K = 1/2 k_e sum_J (a_K b_J + a_J b_K) G[K, J]."""
    eta = eta if eta is not None else 5.6 / L
    tau = slater_tau(U) if screened else None
    G = kernel_gradient(pos, species, L, eta, n_real, k_max, tau, short_cut)
    w = a[:, None] * b[None, :] + b[:, None] * a[None, :]
    return 0.5 * COULOMB_EV_A * np.einsum("kj,kjx->kx", w, G)
