"""Synthetic tight-binding model and neighbour list (oracle).

The paper's engine receives coordinates, atom types, lattice vectors and
orbital indices and builds the Hamiltonian itself (Interface section, engine
inputs).  The SCC-DFTB tables it uses are not available, so the water-like
stand-in model is:

* orbitals: O has s, px, py, pz; H has s.  Neutral valence O 6, H 1.
* on-site energies (eV): O s -23.9, O p -9.0, H s -6.4; on-site overlap = I.
* every sigma two-centre integral uses one radial function
      V(r) = -4.0 exp(-(r - 1.0)/0.5) eV,   S(r) = 0.3 exp(-(r - 1.0)/0.6),
  with V_pp_pi = 0, cut off at r < 4 A (strict).
* Slater-Koster direction cosines u = (R_J - R_I)/r taken from the atom of the
  row orbital:  [s_I, s_J] = V, [s_I, p_J^b] = u_b V, [p_I^a, s_J] = -u_a V,
  [p_I^a, p_J^b] = u_a u_b V; the overlap uses the same pattern with S(r).
* SCC shift (SI section D): H_ab += 1/2 S_ab (V_I + V_J) with V = gamma q.
* For molecular dynamics: with taper_on > 0 the radial functions are
  multiplied by t(r) = 1 - x^3 (10 - 15 x + 6 x^2), x = (r - taper_on) /
  (cutoff - taper_on) on [taper_on, cutoff] (value, slope and curvature
  continuous at both ends), and a repulsive pair energy
  sum_{I<J} A_pair exp(-r/rho) t(r) (pairs O-O, O-H, H-H) stands in for the
  repulsive term of SCC-DFTB.

Minimum image: d = x_j - x_i; d -= L * rint(d * inv_L) with inv_L = 1/L
computed once; r^2 = (dx*dx + dy*dy) + dz*dz evaluated in exactly this order
(NumPy does not contract to FMA), and a pair is a neighbour iff r^2 < 16.

Pins: brute-force neighbour list == periodic k-d tree (library); H and S are
symmetric; S is positive definite; the 6x6 single-water problem equals a
textbook generalized eigensolve; every element of an O-H and an O-O pair
(s-s, s-p, p-s, p-p) equals the Slater-Koster value worked out by hand, and a
pair's spectrum does not depend on the direction of its axis; the SCC shift
of an O-H pair equals 1/2 S_ab (V_I + V_J) element by element (H_aa += V_I
in the orthogonal model), and a uniform potential c moves every generalized
eigenvalue by exactly c (tests/test_oracle_pins.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_ORB = np.array([4, 1], dtype=np.int64)            # orbitals per species (O, H)
N_VALENCE = np.array([6.0, 1.0])                    # neutral valence electrons
HARTREE_EV = 27.211386
COULOMB_EV_A = 14.399645                            # e^2 / (4 pi eps0) in eV*A


@dataclass(frozen=True)
class TBModel:
    eps_s_O: float = -23.9
    eps_p_O: float = -9.0
    eps_s_H: float = -6.4
    v0: float = -4.0
    v_r0: float = 1.0
    v_decay: float = 0.5
    s0: float = 0.3
    s_r0: float = 1.0
    s_decay: float = 0.6
    cutoff: float = 4.0
    orthogonal: bool = False
    kT: float = 0.1
    hubbard_U: tuple = (0.5 * HARTREE_EV, 0.4 * HARTREE_EV)
    taper_on: float = 0.0
    rep_A: tuple = (0.0, 0.0, 0.0)
    rep_rho: float = 0.3

    @property
    def beta(self) -> float:
        return 1.0 / self.kT


def orbital_layout(species: np.ndarray):
    """orb_ptr[N+1], atom_of_orb[n_orb], type_of_orb[n_orb] (0=s, 1..3 = px,py,pz)."""
    norb = N_ORB[species]
    orb_ptr = np.zeros(len(species) + 1, dtype=np.int64)
    orb_ptr[1:] = np.cumsum(norb)
    atom_of_orb = np.repeat(np.arange(len(species)), norb)
    type_of_orb = np.arange(orb_ptr[-1]) - orb_ptr[atom_of_orb]
    return orb_ptr, atom_of_orb, type_of_orb


def n_electrons(species: np.ndarray) -> float:
    return float(N_VALENCE[species].sum())


def min_image(d: np.ndarray, L: float, inv_L: float) -> np.ndarray:
    return d - L * np.rint(d * inv_L)


def r2_of(d: np.ndarray) -> np.ndarray:
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def neighbour_list(pos: np.ndarray, L: float, cutoff: float = 4.0, chunk: int = 512):
    """All ordered pairs (i, j), i != j, with r_ij < cutoff: CSR with rows and
    columns ascending.  Plain O(N^2) brute force over row chunks."""
    n = pos.shape[0]
    inv_L = 1.0 / L
    c2 = cutoff * cutoff
    rows, cols = [], []
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        d = pos[None, :, :] - pos[r0:r1, None, :]
        d = min_image(d, L, inv_L)
        r2 = r2_of(d)
        mask = r2 < c2
        mask[np.arange(r1 - r0), np.arange(r0, r1)] = False
        ii, jj = np.nonzero(mask)
        rows.append(ii + r0)
        cols.append(jj)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, cols.astype(np.int64)


def neighbour_list_kdtree(pos: np.ndarray, L: float, cutoff: float = 4.0):
    """Same CSR as neighbour_list, with candidate pairs from a periodic k-d tree
    (library routine) and the pair test redone with the exact expression above."""
    from scipy.spatial import cKDTree
    n = pos.shape[0]
    pairs = cKDTree(pos, boxsize=L).query_pairs(cutoff * (1.0 + 1e-9), output_type="ndarray")
    i = np.concatenate([pairs[:, 0], pairs[:, 1]])
    j = np.concatenate([pairs[:, 1], pairs[:, 0]])
    inv_L = 1.0 / L
    r2 = r2_of(min_image(pos[j] - pos[i], L, inv_L))
    keep = r2 < cutoff * cutoff
    i, j = i[keep], j[keep]
    order = np.lexsort((j, i))
    i, j = i[order], j[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, i + 1, 1)
    return np.cumsum(row_ptr), j.astype(np.int64)


def _pair_factor(u: np.ndarray, ta: np.ndarray, tb: np.ndarray) -> np.ndarray:
    """Slater-Koster angular factor g[a, b] for row orbital type ta[a] and
    column orbital type tb[b], given direction cosines u[a, b, :] (x_J - x_I)/r."""
    ext = np.concatenate([np.ones(u.shape[:2] + (1,)), u], axis=2)   # ext[..., 0] = 1 (s)
    ia = np.broadcast_to(ta[:, None], u.shape[:2])
    ib = np.broadcast_to(tb[None, :], u.shape[:2])
    ua = np.take_along_axis(ext, ia[..., None], axis=2)[..., 0]
    ub = np.take_along_axis(ext, ib[..., None], axis=2)[..., 0]
    sign = np.where((ia > 0) & (ib == 0), -1.0, 1.0)
    return sign * ua * ub


def dense_hs(pos: np.ndarray, species: np.ndarray, L: float, model: TBModel, atoms=None,
             V_atom: np.ndarray | None = None):
    """Dense principal submatrices h, s over the orbitals of `atoms` (in the
    given order; orbitals of an atom stay in s, px, py, pz order).  With
    atoms=None the whole system is used.  Returns (h, s) with s = None for an
    orthogonal model.  V_atom (eV per atom) adds the SCC shift."""
    if atoms is None:
        atoms = np.arange(len(species))
    atoms = np.asarray(atoms, dtype=np.int64)
    sp = species[atoms]
    norb = N_ORB[sp]
    a_of = np.repeat(np.arange(len(atoms)), norb)          # local atom of orbital
    t_of = np.concatenate([np.arange(k) for k in norb])
    p = pos[atoms]
    inv_L = 1.0 / L
    d = p[None, :, :] - p[:, None, :]                        # d[I,J] = x_J - x_I
    d = min_image(d, L, inv_L)
    r2 = r2_of(d)
    na = len(atoms)
    nb = (r2 < model.cutoff * model.cutoff) & ~np.eye(na, dtype=bool)
    r = np.sqrt(r2)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = d / r[..., None]
    u[~nb] = 0.0
    V = np.where(nb, model.v0 * np.exp(-(r - model.v_r0) / model.v_decay), 0.0)
    Sr = np.where(nb, model.s0 * np.exp(-(r - model.s_r0) / model.s_decay), 0.0)
    if model.taper_on > 0:
        t = taper(np.where(nb, r, model.cutoff), model.taper_on, model.cutoff)
        V = V * t
        Sr = Sr * t
    # orbital-level expansion
    uo = u[a_of][:, a_of]                                    # [n, n, 3]
    g = _pair_factor(uo, t_of, t_of)
    h = V[a_of][:, a_of] * g
    onsite = np.where(sp[a_of] == 0, np.where(t_of == 0, model.eps_s_O, model.eps_p_O), model.eps_s_H)
    h[np.arange(len(a_of)), np.arange(len(a_of))] = onsite
    if model.orthogonal:
        s = None
    else:
        s = Sr[a_of][:, a_of] * g
        s[np.arange(len(a_of)), np.arange(len(a_of))] = 1.0
    if V_atom is not None:
        v = V_atom[atoms][a_of]
        sm = np.eye(len(a_of)) if s is None else s
        h = h + 0.5 * sm * (v[:, None] + v[None, :])
    return h, s


def taper(r, r_on: float, r_c: float):
    """1 below r_on, 1 - x^3 (10 - 15 x + 6 x^2) for x = (r - r_on)/(r_c - r_on)
    in [0, 1], 0 beyond."""
    x = np.clip((np.asarray(r, dtype=np.float64) - r_on) / (r_c - r_on), 0.0, 1.0)
    return 1.0 - x ** 3 * (10.0 - 15.0 * x + 6.0 * x * x)


def repulsion_energy(pos: np.ndarray, species: np.ndarray, L: float, model: TBModel) -> float:
    """sum over neighbour pairs I < J of A_pair exp(-r/rho) t(r) (eV); pair
    index O-O 0, O-H 1, H-H 2."""
    rp, col = neighbour_list(pos, L, model.cutoff)
    n = len(species)
    rows = np.repeat(np.arange(n), np.diff(rp))
    keep = rows < col
    i, j = rows[keep], col[keep]
    r = np.sqrt(r2_of(min_image(pos[j] - pos[i], L, 1.0 / L)))
    pair = species[i] + species[j]
    A = np.asarray(model.rep_A, dtype=np.float64)[pair]
    t = taper(r, model.taper_on, model.cutoff) if model.taper_on > 0 else 1.0
    return float(np.sum(A * np.exp(-r / model.rep_rho) * t))


def single_water_reference(model: TBModel):
    """Geometry of one water in a 30 A box (used by the 6x6 textbook pin)."""
    th = np.radians(52.25)
    pos = np.array([[15.0, 15.0, 15.0],
                    [15.0 + 0.96 * np.sin(th), 15.0, 15.0 + 0.96 * np.cos(th)],
                    [15.0 - 0.96 * np.sin(th), 15.0, 15.0 + 0.96 * np.cos(th)]])
    return pos, np.array([0, 1, 1], dtype=np.int32), 30.0
