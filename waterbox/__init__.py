"""Seeded synthetic water boxes: the one input module that both the CPU
oracle and the GPU path consume.

This module builds geometry only (positions, species, molecule anchors,
periodic box, displaced snapshots, a prescribed rigid-body trajectory and
random initial network weights).  It holds none of the density-matrix
method's arithmetic: no Hamiltonian, no neighbour graph, no solver.

The recipe follows the water-like synthetic systems that stand in for the
paper's water boxes (Simulations section: 2,955-, 30,840- and 2,088-atom
water boxes; the LATTE inputs themselves are not available):

* N_w rigid waters, O-H 0.96 A, H-O-H 104.5 deg, at 0.1 atoms/A^3 in a cubic
  periodic box of side L = (3 N_w / 0.1)^(1/3).
* m = ceil(N_w^(1/3)) lattice sites per axis (spacing a = L/m); N_w of the m^3
  sites are chosen by a seeded permutation.
* O at the site centre plus U(-0.1a, 0.1a)^3 jitter; orientation from a unit
  quaternion built from 4 standard normals; the local frame puts the H atoms
  at (+-0.96 sin 52.25 deg, 0, 0.96 cos 52.25 deg) from O.
* A molecule with any atom closer than 1.5 A (minimum image) to an atom of an
  already placed molecule is redrawn from the same stream (<= 200 tries).
* Atom order is O, H, H per molecule; positions are wrapped into [0, L).
* RNG: numpy.random.default_rng(seed) (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

OH_BOND = 0.96                 # A
HALF_ANGLE_DEG = 52.25         # half of 104.5 deg
DENSITY = 0.1                  # atoms / A^3
CLASH = 1.5                    # A, minimum allowed inter-molecular distance
MAX_TRIES = 200

SPECIES_O = 0
SPECIES_H = 1

AMU_KG = 1.66053906660e-27
KB_J = 1.380649e-23
M_O_AMU = 15.999
M_H_AMU = 1.008


@dataclass
class WaterBox:
    """A periodic box of rigid waters.

    pos      float64 [N, 3] in A, wrapped into [0, L)
    species  int32 [N]   (0 = O, 1 = H)
    anchor   int32 [N]   index of the O atom of the atom's molecule
    box      float64 [3] box edge lengths (cubic: all equal)
    n_waters int
    seed     int
    tries    int32 [n_waters] number of draws each molecule needed
    """
    pos: np.ndarray
    species: np.ndarray
    anchor: np.ndarray
    box: np.ndarray
    n_waters: int
    seed: int
    tries: np.ndarray = field(default=None, repr=False)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    def with_positions(self, pos: np.ndarray) -> "WaterBox":
        return WaterBox(pos=np.ascontiguousarray(pos, dtype=np.float64),
                        species=self.species, anchor=self.anchor, box=self.box,
                        n_waters=self.n_waters, seed=self.seed, tries=self.tries)


def box_length(n_waters: int, density: float = DENSITY) -> float:
    return (3.0 * n_waters / density) ** (1.0 / 3.0)


def sites_per_axis(n_waters: int) -> int:
    m = 1
    while m * m * m < n_waters:
        m += 1
    return m


def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _local_frame() -> np.ndarray:
    th = math.radians(HALF_ANGLE_DEG)
    hx, hz = OH_BOND * math.sin(th), OH_BOND * math.cos(th)
    return np.array([[0.0, 0.0, 0.0], [hx, 0.0, hz], [-hx, 0.0, hz]])


def water_box(n_waters: int, seed: int, density: float = DENSITY) -> WaterBox:
    """Place n_waters rigid waters on a jittered cubic lattice (see module doc)."""
    if n_waters < 1:
        raise ValueError("n_waters must be >= 1")
    rng = np.random.default_rng(seed)
    L = box_length(n_waters, density)
    m = sites_per_axis(n_waters)
    a = L / m
    sites = rng.permutation(m ** 3)[:n_waters]
    frame = _local_frame()
    occupied = -np.ones(m ** 3, dtype=np.int64)   # site -> molecule index
    mol_pos = np.zeros((n_waters, 3, 3))
    tries = np.zeros(n_waters, dtype=np.int32)
    offs = [(di, dj, dk) for di in (-1, 0, 1) for dj in (-1, 0, 1) for dk in (-1, 0, 1)
            if (di, dj, dk) != (0, 0, 0)]
    for w, s in enumerate(sites):
        i, j, k = s // (m * m), (s // m) % m, s % m
        centre = (np.array([i, j, k], dtype=np.float64) + 0.5) * a
        near = []
        for di, dj, dk in offs:
            t = (((i + di) % m) * m + (j + dj) % m) * m + (k + dk) % m
            if occupied[t] >= 0:
                near.append(mol_pos[occupied[t]])
        near = np.concatenate(near, axis=0) if near else np.zeros((0, 3))
        for attempt in range(1, MAX_TRIES + 1):
            jit = rng.uniform(-0.1 * a, 0.1 * a, size=3)
            qv = rng.normal(size=4)
            q = qv / np.linalg.norm(qv)
            R = _quat_to_rot(q)
            atoms = centre + jit + frame @ R.T
            if near.shape[0]:
                d = atoms[:, None, :] - near[None, :, :]
                d -= L * np.rint(d / L)
                if np.min(np.einsum("ijk,ijk->ij", d, d)) < CLASH * CLASH:
                    continue
            break
        else:
            raise RuntimeError(f"molecule {w} could not be placed in {MAX_TRIES} tries")
        tries[w] = attempt
        mol_pos[w] = atoms
        occupied[s] = w
    pos = mol_pos.reshape(-1, 3)
    pos = pos - L * np.floor(pos / L)
    pos[pos >= L] -= L          # guard the x == L rounding edge
    n = 3 * n_waters
    species = np.tile(np.array([SPECIES_O, SPECIES_H, SPECIES_H], dtype=np.int32), n_waters)
    anchor = (np.arange(n, dtype=np.int32) // 3) * 3
    return WaterBox(pos=np.ascontiguousarray(pos), species=species, anchor=anchor.astype(np.int32),
                    box=np.array([L, L, L]), n_waters=n_waters, seed=seed, tries=tries)


def displaced(base: WaterBox, seed: int, sigma: float = 0.05) -> WaterBox:
    """A snapshot of `base` with N(0, sigma^2) A per Cartesian component per atom."""
    rng = np.random.default_rng(seed)
    L = base.box[0]
    pos = base.pos + rng.normal(0.0, sigma, size=base.pos.shape)
    pos = pos - L * np.floor(pos / L)
    pos[pos >= L] -= L
    return base.with_positions(pos)


def rigid_trajectory(base: WaterBox, n_steps: int, dt_fs: float, seed: int,
                     temperature: float = 300.0):
    """Prescribed rigid-water motion: yields positions for steps 0..n_steps.

    Each molecule translates with a Maxwell centre-of-mass velocity at
    `temperature` (total mass of H2O) and spins about its centre of mass with a
    constant lab-frame angular velocity whose principal-axis components are
    Maxwell-distributed with the rigid-body moments of inertia.  There is no
    force model, so the free-flight motion is integrated exactly.
    """
    rng = np.random.default_rng(seed)
    L = base.box[0]
    nw = base.n_waters
    masses = np.array([M_O_AMU, M_H_AMU, M_H_AMU])
    M = masses.sum()
    mol = base.pos.reshape(nw, 3, 3).copy()
    # unwrap each molecule around its O atom
    rel = mol - mol[:, :1, :]
    rel -= L * np.rint(rel / L)
    mol = mol[:, :1, :] + rel
    com = np.einsum("a,waj->wj", masses, mol) / M
    r_body = mol - com[:, None, :]
    kT = KB_J * temperature
    # A/fs = 1e5 m/s
    v_sigma = math.sqrt(kT / (M * AMU_KG)) / 1e5
    v_com = rng.normal(0.0, v_sigma, size=(nw, 3))
    v_com -= v_com.mean(axis=0)
    omega = np.zeros((nw, 3))
    draws = rng.normal(size=(nw, 3))
    for w in range(nw):
        I = np.zeros((3, 3))
        for a in range(3):
            r = r_body[w, a]
            I += masses[a] * (np.dot(r, r) * np.eye(3) - np.outer(r, r))
        evals, evecs = np.linalg.eigh(I)        # amu A^2
        # rad/fs: sqrt(kT / I) with I in kg m^2 -> 1/s, then * 1e-15
        om_p = draws[w] * np.sqrt(kT / (evals * AMU_KG * 1e-20)) * 1e-15
        omega[w] = evecs @ om_p
    frames = []
    for step in range(n_steps + 1):
        t = step * dt_fs
        th = np.linalg.norm(omega, axis=1) * t
        axis = omega / np.maximum(np.linalg.norm(omega, axis=1, keepdims=True), 1e-300)
        c, s = np.cos(th)[:, None, None], np.sin(th)[:, None, None]
        K = np.zeros((nw, 3, 3))
        K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -axis[:, 2], axis[:, 1], -axis[:, 0]
        K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = axis[:, 2], -axis[:, 1], axis[:, 0]
        Rm = np.eye(3)[None] + s * K + (1 - c) * np.einsum("wij,wjk->wik", K, K)
        pos = (com + v_com * t)[:, None, :] + np.einsum("wij,waj->wai", Rm, r_body)
        pos = pos.reshape(-1, 3)
        pos = pos - L * np.floor(pos / L)
        pos[pos >= L] -= L
        frames.append(np.ascontiguousarray(pos))
    return frames


def mlp_init(seed: int, n_in: int = 32, n_hidden: int = 64, n_species: int = 2):
    """Seeded initial weights for one 32-64-64-1 network per central species.

    Returns a list (per species) of dicts with W1 [64,32], b1 [64], W2 [64,64],
    b2 [64], W3 [1,64], b3 [1] (float64), drawn uniform(-1/sqrt(fan_in),
    1/sqrt(fan_in)) for weights and zeros for biases.
    """
    rng = np.random.default_rng(seed)
    nets = []
    for _ in range(n_species):
        net = {}
        for name, (o, i) in (("1", (n_hidden, n_in)), ("2", (n_hidden, n_hidden)), ("3", (1, n_hidden))):
            lim = 1.0 / math.sqrt(i)
            net["W" + name] = rng.uniform(-lim, lim, size=(o, i))
            net["b" + name] = np.zeros(o)
        nets.append(net)
    return nets


# The benchmark workloads (sizes and seeds of the synthetic systems).
WORKLOADS = {
    "water96": dict(n_waters=96, seed=1, orthogonal=True, grid=(2, 2, 2), tau=1e-5),
    "water3000": dict(n_waters=3000, seed=2, orthogonal=False, grid=(5, 5, 6), tau=1e-5),
    "water10000": dict(n_waters=10000, seed=3, orthogonal=False, grid=(10, 10, 10), tau=1e-3),
    "water3000_scc": dict(n_waters=3000, seed=4, orthogonal=False, grid=(5, 5, 6), tau=1e-3),
    "water30000": dict(n_waters=30000, seed=5, orthogonal=False, grid=(14, 14, 15), tau=1e-3),
}


def workload_box(name: str) -> WaterBox:
    w = WORKLOADS[name]
    return water_box(w["n_waters"], w["seed"])
