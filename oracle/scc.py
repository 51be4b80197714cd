"""Self-consistent-charge loop (oracle; test infrastructure only).

The charge vector n of SI section D is iterated to self-consistency:
V = gamma n (Ewald 1/r between sites plus the on-site Hubbard U), H[n] adds
1/2 S_ab (V_I + V_J), q0[n] are the Mulliken charges of the subgraph density
solve at H[n], and the residual is F[n] = q0[n] - n.  Two updates:

* linear: the scaled-delta kernel K = -c I of the Shadow MD section / SI
  section B, n <- n + c F[n];
* anderson: Anderson acceleration of the same fixed-point map with memory m
  and mixing c (Anderson 1965; the "type II" form of Walker and Ni 2011):
  with the last m differences dF_j = F_{j+1} - F_j and dn_j = n_{j+1} - n_j,
  gamma = argmin || F_k - sum_j gamma_j dF_j ||_2 and
  n_{k+1} = n_k + c F_k - sum_j gamma_j (dn_j + c dF_j).
  With m = 0 it is the linear update.

Iteration stops at the first n with RMS(F[n]) below 1e-5 e (200-iteration
cap) and returns q0[n].  The default is Anderson with m = 8, c = 0.03: the
charge response of these water boxes is strong and grows with the box
(Jacobian eigenvalues far below -1), so the linear update needs c of a few
hundredths and then converges slowly, and Anderson diverges at c = 0.3 on
a few hundred waters and at c = 0.1 on 3,000.

Pins (tests/test_oracle_learned.py): on a real system the fixed point is
independent of the start and one more map application moves q by less than
the tolerance; on an affine map G(n) = A n + b the Anderson iteration
reaches the closed-form fixed point (I - A)^-1 b where linear mixing
diverges, and memory 0 reproduces linear mixing exactly.
"""
from __future__ import annotations

import numpy as np

from .ewald import coulomb_potential
from .model import TBModel
from .solve import solve_system


def anderson_step(n_hist, f_hist, mix: float, depth: int):
    """Next iterate from the histories (oldest first; the last entry is the
    current n_k, F_k)."""
    n_k, f_k = n_hist[-1], f_hist[-1]
    m = min(depth, len(n_hist) - 1)
    if m == 0:
        return n_k + mix * f_k
    dF = np.stack([f_hist[-m + j] - f_hist[-m + j - 1] for j in range(m)], axis=1)
    dn = np.stack([n_hist[-m + j] - n_hist[-m + j - 1] for j in range(m)], axis=1)
    gamma, *_ = np.linalg.lstsq(dF, f_k, rcond=None)
    return n_k + mix * f_k - (dn + mix * dF) @ gamma


def fixed_point(charge_map, n0, mix: float = 0.3, tol: float = 1e-5, max_iter: int = 200,
                mixer: str = "linear", depth: int = 5):
    """Iterate n -> q0[n] = charge_map(n).  Returns (q0 at the converged n,
    iterations, residual history, converged)."""
    n = np.array(n0, dtype=np.float64)
    n_hist, f_hist, hist = [], [], []
    for it in range(1, max_iter + 1):
        q = charge_map(n)
        f = q - n
        rms = float(np.sqrt(np.mean(f * f)))
        hist.append(rms)
        if rms < tol:
            return q, it, hist, True
        if mixer == "linear":
            n = n + mix * f
        else:
            n_hist.append(n)
            f_hist.append(f)
            n_hist, f_hist = n_hist[-(depth + 1):], f_hist[-(depth + 1):]
            n = anderson_step(n_hist, f_hist, mix, depth)
    return n, max_iter, hist, False


def scc(pos, species, L, model: TBModel, subs, q_start=None, mix: float = 0.03, tol: float = 1e-5,
        max_iter: int = 200, eta=None, n_real: int = 2, k_max: int = 8, mixer: str = "anderson", depth: int = 8,
        short_cut: float = np.inf, screened: bool = True):
    """Returns (q, iterations, residual history)."""
    U = np.asarray(model.hubbard_U)

    def charge_map(n):
        V = coulomb_potential(pos, species, n, L, U, eta=eta, n_real=n_real, k_max=k_max, short_cut=short_cut,
                              screened=screened)
        return solve_system(pos, species, L, model, subs, V_atom=V).q

    n0 = np.zeros(len(species)) if q_start is None else q_start
    q, it, hist, _ = fixed_point(charge_map, n0, mix=mix, tol=tol, max_iter=max_iter, mixer=mixer, depth=depth)
    return q, it, hist
