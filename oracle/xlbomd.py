"""Extended-Lagrangian Born-Oppenheimer molecular dynamics (oracle; test
infrastructure only).

What is computed (Shadow MD section: equations of motion NEQ and HW,
integrated with a modified velocity Verlet scheme with weak dissipation):

* nuclei: velocity Verlet on the forces of the shadow potential at fixed n
  (forces.shadow_point): v += dt/2 F/M, R += dt v, (new forces), v += dt/2 F/M;
* the extended charge vector n: the Verlet form of n'' = w^2 K (q[n] - n)
  with the kernel K = c I (c = 1: the plain harmonic well; 0 < c < 1 damps
  the strong charge response of SCC systems, the scaled-delta kernel also
  used by the linear SCC mixer) plus the dissipation of Niklasson et al.,
  J. Chem. Phys. 130, 214109 (2009), for K = 5 previous steps:
      n_{t+1} = 2 n_t - n_{t-1} + kappa c (q_t - n_t) + alpha sum_{k=0..5} c_k n_{t-k},
  kappa = dt^2 w^2 = 1.82, alpha = 0.018, c_k = (-6, 14, -8, -3, 4, -1)
  (the published coefficients of that reference; sum c_k = sum k c_k = 0, so
  the dissipation leaves constant and linear histories untouched).
* n starts at the converged SCC charges with every history entry equal; the
  total free energy is the kinetic energy plus U(R, n).

Units: A, fs, eV, amu; a = F/M * 0.00964853321 A/fs^2 per eV/(A amu), and a
kinetic energy 1/2 M v^2 in amu A^2/fs^2 times 103.6426965 is in eV.

Pins (tests/test_oracle_forces.py): the coefficient identities above; on a
water dimer the fluctuation of the total free energy grows by about four
when dt doubles (the global second-order error of velocity Verlet that the
Shadow MD results report).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .ewald import coulomb_potential
from .forces import Ewald, shadow_point
from .model import TBModel
from .response import charge_response, krylov_step

KAPPA = 1.82
ALPHA = 0.018
C_DISS = np.array([-6.0, 14.0, -8.0, -3.0, 4.0, -1.0])
ACCEL = 0.00964853321         # A/fs^2 per eV/(A amu)
KE_EV = 103.6426965           # eV per amu A^2/fs^2
MASS = np.array([15.999, 1.008])


def next_charges(hist: list, q_t: np.ndarray, c: float, delta: np.ndarray | None = None) -> np.ndarray:
    """n_{t+1} from hist = [n_t, n_{t-1}, ..., n_{t-5}] and q_t = q[n_t]; the
    driving term is kappa c (q_t - n_t), or kappa delta with delta = K (q_t - n_t)
    of another kernel."""
    n_t, n_m1 = hist[0], hist[1]
    diss = sum(ck * hk for ck, hk in zip(C_DISS, hist))
    drive = KAPPA * c * (q_t - n_t) if delta is None else KAPPA * delta
    return 2.0 * n_t - n_m1 + drive + ALPHA * diss


def krylov_kernel(st, pos, species, L, model: TBModel, subs, ew: Ewald, rank_tol: float, max_rank: int,
                  k0: float) -> np.ndarray:
    """delta = -J^-1 (q[n] - n) by the low-rank preconditioned Krylov kernel
    (response.krylov_step, completed), J v = dq[gamma v] - v from the
    first-order charge response at the solve of `st`."""
    U = np.asarray(model.hubbard_U)

    def jv(v):
        dV = coulomb_potential(pos, species, v, L, U, eta=ew.eta, n_real=ew.n_real, k_max=ew.k_max,
                               screened=ew.screened, short_cut=ew.short_cut)
        dq, _, _ = charge_response(pos, species, L, model, subs, st.V, dV, mu=st.system.mu, sols=st.system.sols)
        return dq - v

    f = st.q - st.n
    dn, _, _ = krylov_step(f, jv, rank_tol=rank_tol, max_rank=max_rank, k0=k0, complete=True)
    return dn


def kinetic(v: np.ndarray, m: np.ndarray) -> float:
    return 0.5 * KE_EV * float(np.sum(m[:, None] * v * v))


@dataclass
class Trajectory:
    t: list = field(default_factory=list)          # fs
    e_tot: list = field(default_factory=list)      # eV, kinetic + U(R, n)
    e_pot: list = field(default_factory=list)
    rms_qn: list = field(default_factory=list)     # RMS(q[n] - n)
    pos: list = field(default_factory=list)


def run(pos0, vel0, species, L, model: TBModel, subs, n0, ew: Ewald, dt: float, steps: int, c: float = 1.0,
        keep_pos: bool = False, kernel: str = "scaled", rank_tol: float = 0.1, max_rank: int = 6,
        k0: float = 0.1) -> Trajectory:
    """XL-BOMD from (pos0, vel0) with n = n0 (converged SCC charges);
    `subs(pos)` returns the subgraph set at a geometry.  kernel "scaled":
    K = c I; "krylov": K = -J^-1 by the low-rank Krylov kernel, rebuilt at
    every step."""
    m = MASS[species]
    R = np.array(pos0, dtype=np.float64)
    v = np.array(vel0, dtype=np.float64)
    hist = [np.array(n0, dtype=np.float64) for _ in range(6)]
    st = shadow_point(R, species, L, model, subs(R), hist[0], ew)
    tr = Trajectory()

    def record(t, st):
        tr.t.append(t)
        tr.e_pot.append(st.U)
        tr.e_tot.append(kinetic(v, m) + st.U)
        tr.rms_qn.append(float(np.sqrt(np.mean((st.q - hist[0]) ** 2))))
        if keep_pos:
            tr.pos.append(R.copy())

    record(0.0, st)
    for k in range(1, steps + 1):
        v += 0.5 * dt * ACCEL * st.F / m[:, None]
        delta = None
        if kernel == "krylov":
            delta = krylov_kernel(st, R, species, L, model, subs(R), ew, rank_tol, max_rank, k0)
        R = R + dt * v
        n_new = next_charges(hist, st.q, c, delta)
        hist = [n_new] + hist[:5]
        st = shadow_point(R, species, L, model, subs(R), n_new, ew)
        v += 0.5 * dt * ACCEL * st.F / m[:, None]
        record(k * dt, st)
    return tr
