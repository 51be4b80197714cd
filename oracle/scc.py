"""Self-consistent-charge loop (oracle).

The charge vector n of SI section D is iterated to self-consistency:
V = gamma n (Ewald 1/r between sites plus the on-site Hubbard U), H[n] adds
1/2 S_ab (V_I + V_J), q0[n] are the Mulliken charges of the subgraph density
solve at H[n], and the update is the scaled-delta kernel K = -c I of the
Shadow MD section / SI section B (linear mixing):
    n <- n + c (q0[n] - n),  c = 0.3,
until the RMS residual of q0[n] - n is below 1e-5 e (200-iteration cap).

Pins: the fixed point is independent of the start (zero vs any guess) and
the residual at the returned charges is below the tolerance
(tests/test_oracle_learned.py).
"""
from __future__ import annotations

import numpy as np

from .ewald import coulomb_potential
from .model import TBModel
from .solve import solve_system


def scc(pos, species, L, model: TBModel, subs, q_start=None, mix: float = 0.3, tol: float = 1e-5,
        max_iter: int = 200, eta=None, n_real: int = 2, k_max: int = 8):
    """Returns (q, iterations, residual history)."""
    U = np.asarray(model.hubbard_U)
    n = np.zeros(len(species)) if q_start is None else np.array(q_start, dtype=np.float64)
    hist = []
    for it in range(1, max_iter + 1):
        V = coulomb_potential(pos, species, n, L, U, eta=eta, n_real=n_real, k_max=k_max)
        res = solve_system(pos, species, L, model, subs, V_atom=V)
        r = res.q - n
        rms = float(np.sqrt(np.mean(r * r)))
        hist.append(rms)
        if rms < tol:
            return res.q, it, hist
        n = n + mix * r
    return n, max_iter, hist
