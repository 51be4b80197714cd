"""Graph construction and partitioning (oracle).

* Initial graph from a distance neighbour list (Determining the Subgraphs
  section; Fig. graph_partition a).
* Core partition: the paper uses community detection; the stand-in is a
  spatial grid on the wrapped anchor (O) position: per axis
  cell = min(g - 1, floor((x * inv_L) * g)), id = (i * g_y + j) * g_z + k;
  hydrogens follow their O; empty cells are skipped and the remaining cells are
  numbered in ascending id order.
* Cost-balanced cores for re-partitioning (stand-in for community detection
  when the halos have grown, Fig. graph_partition f; subgraph cost grows as
  size cubed, Scalability section): weighted recursive coordinate bisection
  of the molecules at their wrapped anchor positions; a set forming k cores
  is sorted along its widest axis (ties by index) and cut where the running
  weight is closest to floor(k/2)/k of its total (first such cut, at least one
  molecule per core); a molecule weighs its atom count plus its atoms'
  graph degrees.
* Halo = every atom outside the core with an edge to some core atom (one hop,
  Fig. graph_partition c; SI section A).  Subgraph atom order: core ascending,
  then halo ascending.
* Atom-condensed density-matrix graph G^D: the largest |D_ab| over each
  atom-atom block, from the collected core rows (Dynamic Graph Adaption).
* Weighted distance graph G^N_IJ = exp(-alpha R_IJ^2) over neighbour pairs
  (Eq. neigh_mat), with G^N_II = 1.
* Graph adaptation G_tau = (G^N G^D + G^D G^N)|_tau (Eq. Graph_Adaptation),
  a strict > tau threshold, symmetrised by max(G_IJ, G_JI).
* Adaptive initial graph: G_0 = neighbour graph, G_{k+1} = G_k union
  {G^D > tau} from a solve on G_k, until no edge is added (Determining the
  Subgraphs: edges are only added in the initial SCF iterations).

Pins: core/halo construction is checked by brute force on small boxes; the
graph-from-D rules are checked on hand-built matrices; G^N of three atoms
(one pair only through a periodic image) equals exp(-0.7 R^2) worked out by
hand with the unit diagonal; the all-to-all graph reproduces the full-system
density matrix (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .model import N_ORB, min_image, r2_of


def csr_from_pairs(n: int, rows: np.ndarray, cols: np.ndarray):
    """Deduplicated CSR (row_ptr[n+1], col) with ascending columns, no self edges."""
    keep = rows != cols
    key = np.unique(rows[keep].astype(np.int64) * n + cols[keep].astype(np.int64))
    r, c = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    return np.cumsum(row_ptr), c


def grid_cores(pos: np.ndarray, anchor: np.ndarray, L: float, grid):
    gx, gy, gz = grid
    inv_L = 1.0 / L
    p = pos[anchor]
    cell = []
    for ax, g in enumerate((gx, gy, gz)):
        c = np.floor((p[:, ax] * inv_L) * g).astype(np.int64)
        cell.append(np.minimum(g - 1, c))
    cid = (cell[0] * gy + cell[1]) * gz + cell[2]
    used = np.unique(cid)
    remap = -np.ones(gx * gy * gz, dtype=np.int64)
    remap[used] = np.arange(len(used))
    return remap[cid], len(used)


def rcb_parts(xyz, w, k):
    """Recursive coordinate bisection of points xyz [m, 3] with weights w into
    k parts (plain loops: running sums in sorted order)."""
    m = len(w)
    part = [0] * m

    def split(idx, k, first):
        if k == 1:
            for i in idx:
                part[i] = first
            return
        ext = [max(xyz[i][a] for i in idx) - min(xyz[i][a] for i in idx) for a in range(3)]
        ax = 0
        for a in (1, 2):
            if ext[a] > ext[ax]:
                ax = a
        idx = sorted(idx, key=lambda i: (xyz[i][ax], i))
        k1 = k // 2
        tot = 0.0
        for i in idx:
            tot += w[i]
        target = tot * k1 / k
        run = 0.0
        for i in idx[:k1]:
            run += w[i]
        best, cut = abs(run - target), k1
        for s in range(k1, len(idx) - (k - k1)):
            run += w[idx[s]]
            if abs(run - target) < best:
                best, cut = abs(run - target), s + 1
        split(idx[:cut], k1, first)
        split(idx[cut:], k - k1, first + k1)

    split(list(range(m)), k, 0)
    return part


def balanced_cores(pos: np.ndarray, anchor: np.ndarray, L: float, n_cores: int, row_ptr=None):
    """Core of every atom from the weighted bisection of the molecules."""
    n = len(anchor)
    mols = [a for a in range(n) if anchor[a] == a]
    mol_of = {a: i for i, a in enumerate(mols)}
    inv_L = 1.0 / L
    xyz = []
    for a in mols:
        xyz.append([float(pos[a][c] - L * np.floor(pos[a][c] * inv_L)) for c in range(3)])
    w = [0.0] * len(mols)
    for a in range(n):
        deg = 0 if row_ptr is None else int(row_ptr[a + 1] - row_ptr[a])
        w[mol_of[int(anchor[a])]] += 1.0 + deg
    part = rcb_parts(xyz, w, n_cores)
    return np.array([part[mol_of[int(anchor[a])]] for a in range(n)], dtype=np.int64)


def extract_subgraphs(row_ptr: np.ndarray, col: np.ndarray, core_of_atom: np.ndarray, n_cores: int):
    """List of (atoms, n_core_atoms): core atoms ascending, then one-hop halo ascending."""
    subs = []
    for c in range(n_cores):
        core = np.nonzero(core_of_atom == c)[0]
        nbrs = np.concatenate([col[row_ptr[i]:row_ptr[i + 1]] for i in core]) if len(core) else np.zeros(0, np.int64)
        halo = np.setdiff1d(np.unique(nbrs), core)
        subs.append((np.concatenate([core, halo]).astype(np.int64), len(core)))
    return subs


def subgraph_orbitals(atoms: np.ndarray, species: np.ndarray, orb_ptr: np.ndarray):
    return np.concatenate([np.arange(orb_ptr[a], orb_ptr[a] + N_ORB[species[a]]) for a in atoms])


def condensed_dm(subs, d_core_rows, species: np.ndarray, n_atoms: int):
    """G^D as a sparse [N, N] matrix: row I holds max |D_ab| over a in I and b in
    J for every atom J of the subgraph whose core contains I."""
    rows, cols, vals = [], [], []
    for (atoms, ncore), D in zip(subs, d_core_rows):
        norb = N_ORB[species[atoms]]
        optr = np.concatenate([[0], np.cumsum(norb)])
        A = np.abs(D)
        # column blocks: reduce max over each atom's orbitals
        colmax = np.maximum.reduceat(A, optr[:-1], axis=1)             # [nc_orb, n_atoms_sub]
        blk = np.maximum.reduceat(colmax, optr[:ncore], axis=0)        # [ncore, n_atoms_sub]
        rr, cc = np.meshgrid(atoms[:ncore], atoms, indexing="ij")
        rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(blk.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n_atoms, n_atoms))


def distance_graph(pos: np.ndarray, L: float, row_ptr: np.ndarray, col: np.ndarray, alpha: float):
    """G^N over neighbour-list pairs plus the unit diagonal."""
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    d = min_image(pos[col] - pos[rows], L, 1.0 / L)
    w = np.exp(-alpha * r2_of(d))
    g = sp.csr_matrix((w, (rows, col)), shape=(n, n)) + sp.identity(n, format="csr")
    return g.tocsr()


def graph_dm(gd, tau: float):
    """Edges where max(G^D_IJ, G^D_JI) > tau (strict), no self edges."""
    g = gd.tocoo()
    m = g.data > tau
    n = gd.shape[0]
    r = np.concatenate([g.row[m], g.col[m]])
    c = np.concatenate([g.col[m], g.row[m]])
    return csr_from_pairs(n, r, c)


def graph_adaptive(gn, gd, tau: float):
    """Edges of (G^N G^D + G^D G^N) > tau, symmetrised."""
    w = (gn @ gd + gd @ gn).tocoo()
    m = w.data > tau
    n = gn.shape[0]
    r = np.concatenate([w.row[m], w.col[m]])
    c = np.concatenate([w.col[m], w.row[m]])
    return csr_from_pairs(n, r, c), w


def near_ties(values: np.ndarray, tau: float, rel: float = 1e-9) -> int:
    """Number of graph weights within rel*tau of the threshold."""
    return int(np.count_nonzero(np.abs(values - tau) <= rel * tau))


def graph_union(n: int, a, b):
    ra = np.repeat(np.arange(n), np.diff(a[0]))
    rb = np.repeat(np.arange(n), np.diff(b[0]))
    return csr_from_pairs(n, np.concatenate([ra, rb]), np.concatenate([a[1], b[1]]))


def all_to_all(n: int):
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return csr_from_pairs(n, r.ravel(), c.ravel())
