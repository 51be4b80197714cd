"""Recursive Fermi-operator expansion in exact FP64 arithmetic (oracle).

The paper lets each subgraph's Fermi function be evaluated by a recursive
Fermi-operator expansion instead of diagonalisation (Density Matrix
Evaluation on Partitioned Graphs; the accelerator library of the Software
Design section).  The recursion used here is the grand-canonical
beta-doubling scheme:

* spectral bounds by Gershgorin discs of the orthogonalised h (FP64);
* R = max(|lo - mu|, |hi - mu|), n_d = ceil(log2(beta R)), b = beta / 2^n_d;
* X_0 = 1/2 I - (b/4)(h - mu I)   (first-order expansion of f_b);
* n_d times: X <- X^2 (X^2 + (I - X)^2)^-1, which maps f_b to f_2b exactly
  (f_2b = f_b^2 / (f_b^2 + (1 - f_b)^2)).

In exact arithmetic X_0 = f_b(phi_b(h - mu)) with phi_b(x) = (2/b) artanh(bx/2),
so the recursion returns Q diag(f_beta(phi_b(lam - mu))) Q^T exactly; the
difference to the true Fermi function shrinks like b^2.

Pins: recursion == closed form to 1e-12; closed form -> true Fermi as n_d
grows (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import math

import numpy as np

from .solve import fermi


def gershgorin(h: np.ndarray):
    d = np.diag(h)
    r = np.abs(h).sum(axis=1) - np.abs(d)
    return float((d - r).min()), float((d + r).max())


def n_doublings(beta: float, lo: float, hi: float, mu: float) -> int:
    R = max(abs(lo - mu), abs(hi - mu))
    return max(1, int(math.ceil(math.log2(beta * R))))


def foe_recursion(hp: np.ndarray, mu: float, beta: float, nd: int) -> np.ndarray:
    n = hp.shape[0]
    b = beta / 2.0 ** nd
    I = np.eye(n)
    X = 0.5 * I - (b / 4.0) * (hp - mu * I)
    for _ in range(nd):
        X2 = X @ X
        A = X2 + (I - X) @ (I - X)
        X = np.linalg.solve(A, X2)
        X = 0.5 * (X + X.T)
    return X


def foe_closed_form(hp: np.ndarray, mu: float, beta: float, nd: int) -> np.ndarray:
    b = beta / 2.0 ** nd
    lam, Q = np.linalg.eigh(hp)
    x = lam - mu
    phi = (2.0 / b) * np.arctanh(b * x / 2.0)
    return (Q * fermi(phi, beta)) @ Q.T


def fermi_exact(hp: np.ndarray, mu: float, beta: float) -> np.ndarray:
    lam, Q = np.linalg.eigh(hp)
    return (Q * fermi(lam - mu, beta)) @ Q.T
