"""Periodic point-charge Coulomb potential by Ewald summation (oracle).

The SCC-DFTB engine couples Mulliken charges through a Coulomb interaction
that decays as 1/R, summed over the periodic system (SI section D; the paper
uses a GPU Ewald solver for this all-to-all sum, Scalability section).  The
stand-in drops the short-range screening and keeps the on-site Hubbard U:

  V_I = U_I q_I + k_e [ sum_J q_J psi(R_J - R_I) ]
  psi(r) = sum_n' erfc(eta |r + nL|)/|r + nL|
         + (4 pi / V) sum_{k != 0} exp(-k^2 / (4 eta^2)) / k^2 cos(k . r)
         - 2 eta / sqrt(pi) [r = 0],
  the n' sum skipping the J = I, n = 0 term, with k_e = 14.399645 eV A and
  a neutralising background (k = 0 term dropped).

Pins: the rock-salt Madelung constant 1.747565 and independence of the
splitting parameter eta (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .model import COULOMB_EV_A


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


def coulomb_potential(pos: np.ndarray, species: np.ndarray, q: np.ndarray, L: float, U: np.ndarray,
                      eta: float | None = None, n_real: int = 2, k_max: int = 8) -> np.ndarray:
    eta = eta if eta is not None else 5.6 / L
    psi = ewald_psi_matrix(pos, L, eta, n_real, k_max)
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
