"""Drivers over the C ABI: build the partition and run one density solve.

The sequence follows the paper's workflow (Fig. graph_partition a-e and the
Interface section): neighbour graph -> cores -> core+halo subgraphs -> H, S
-> per-subgraph solve with one global mu -> collected core rows -> charges ->
graph of the next step from D.  Only orchestration lives here; each step is a
libgdm call.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from ._lib import (FP64_EIG, GRAPH_ADAPTIVE, GRAPH_DM, MIXED_BF16, MIXED_F16, Context, Graph, Subgraphs, System,
                   TBParams)


@dataclass
class Partition:
    nbr: Graph                 # distance neighbour graph (H, S and G^N live on it)
    graph: Graph               # partition graph (from D after adaptation)
    core_of_atom: torch.Tensor
    n_cores: int
    sg: Subgraphs
    rounds: int = 0
    sizes: list = field(default_factory=list)
    cost0: float = 0.0         # sum of n^3 of the subgraphs when the cores were last chosen
    repartitions: int = 0


def subgraph_cost(sg: Subgraphs) -> float:
    """Dense-solve cost of a subgraph set: sum of n^3 (Scalability section)."""
    n = sg.norb.astype(np.float64)
    return float(np.sum(n ** 3))


@dataclass
class Solution:
    mu: float
    n_count: float
    D_core: torch.Tensor
    q: torch.Tensor
    eig: torch.Tensor | None = None


def solve(ctx: Context, system: System, part: Partition, H, S, kT: float, precision: int = FP64_EIG,
          mu_guess: float = 0.0, tol_N: float = 1e-6, plan: bool = True, eig: bool = False,
          n_electrons: float | None = None) -> Solution:
    if plan:
        ctx.plan(part.sg, precision)
    mu, n = ctx.find_mu(system, part.sg, part.nbr, H, S, kT, precision, mu_guess, tol_N, n_electrons)
    out = ctx.subgraph_density(part.sg, mu, kT, precision, eig=eig)
    D, E = out if eig else (out, None)
    q = ctx.mulliken_charges(system, part.sg, part.nbr, S, D)
    return Solution(mu=mu, n_count=n, D_core=D, q=q, eig=E)


def cutoff_partition(ctx: Context, system: System, tb: TBParams, grid) -> Partition:
    nbr = ctx.build_graph_cutoff(system, tb.cutoff)
    core, nco = ctx.grid_cores(system, grid)
    sg = ctx.extract_subgraphs(system, tb, nbr, core, nco)
    return Partition(nbr=nbr, graph=nbr, core_of_atom=core, n_cores=nco, sg=sg, sizes=[sg.norb.copy()],
                     cost0=subgraph_cost(sg))


def balanced_partition(ctx: Context, system: System, tb: TBParams, n_cores: int, graph: Graph | None = None,
                       nbr: Graph | None = None) -> Partition:
    """Cores from the weighted recursive bisection (gdm_balanced_cores), each
    molecule weighted by its atoms' degrees in `graph` (default: the
    neighbour graph), and their one-hop halos in `graph`."""
    if nbr is None:
        nbr = ctx.build_graph_cutoff(system, tb.cutoff)
    g = nbr if graph is None else graph
    core = ctx.balanced_cores(system, n_cores, g)
    sg = ctx.extract_subgraphs(system, tb, g, core, n_cores)
    return Partition(nbr=nbr, graph=g, core_of_atom=core, n_cores=n_cores, sg=sg, sizes=[sg.norb.copy()],
                     cost0=subgraph_cost(sg))


def maybe_repartition(ctx: Context, system: System, tb: TBParams, part: Partition, graph: Graph,
                      growth: float = 1.5) -> tuple[Partition, bool]:
    """Subgraphs of the new graph on the current cores; when their sum of n^3
    exceeds `growth` times its value when the cores were chosen, new
    cost-balanced cores are drawn from the new graph (Determining the
    Subgraphs, Fig. graph_partition f).  Returns the partition and whether
    the cores changed."""
    p = repartition(ctx, system, tb, part, graph)
    cost0 = part.cost0 if part.cost0 > 0 else subgraph_cost(part.sg)
    p.cost0 = cost0
    p.repartitions = part.repartitions
    if subgraph_cost(p.sg) <= growth * cost0:
        return p, False
    core = ctx.balanced_cores(system, part.n_cores, graph)
    sg = ctx.extract_subgraphs(system, tb, graph, core, part.n_cores)
    q = Partition(nbr=part.nbr, graph=graph, core_of_atom=core, n_cores=part.n_cores, sg=sg, rounds=part.rounds,
                  sizes=part.sizes + [sg.norb.copy()], cost0=subgraph_cost(sg), repartitions=part.repartitions + 1)
    return q, True


def full_system_partition(ctx: Context, system: System, tb: TBParams) -> Partition:
    """A single subgraph whose core is every atom (full diagonalisation)."""
    nbr = ctx.build_graph_cutoff(system, tb.cutoff)
    core = torch.zeros(system.n_atoms, dtype=torch.int32, device=ctx.dev)
    sg = ctx.extract_subgraphs(system, tb, nbr, core, 1)
    return Partition(nbr=nbr, graph=nbr, core_of_atom=core, n_cores=1, sg=sg)


def repartition(ctx: Context, system: System, tb: TBParams, part: Partition, graph: Graph) -> Partition:
    sg = ctx.extract_subgraphs(system, tb, graph, part.core_of_atom, part.n_cores)
    return Partition(nbr=part.nbr, graph=graph, core_of_atom=part.core_of_atom, n_cores=part.n_cores, sg=sg,
                     rounds=part.rounds, sizes=part.sizes + [sg.norb.copy()], cost0=part.cost0,
                     repartitions=part.repartitions)


def adaptive_partition(ctx: Context, system: System, tb: TBParams, grid, tau: float, kT: float,
                       max_rounds: int = 5, H=None, S=None) -> Partition:
    """Initial-SCF graph adaptation (Determining the Subgraphs): start from the
    neighbour graph and add every edge with G^D > tau found by a solve on the
    current graph, until no edge is added (at most max_rounds solves)."""
    part = cutoff_partition(ctx, system, tb, grid)
    if H is None:
        H, S = ctx.build_hs(system, tb, part.nbr)
    for r in range(max_rounds):
        sol = solve(ctx, system, part, H, S, kT, FP64_EIG)
        g = ctx.build_graph_dm(system, GRAPH_DM, part.sg, sol.D_core, tau, union=part.graph)
        grown = g.nnz > part.graph.nnz
        part = repartition(ctx, system, tb, part, g)
        part.rounds = r + 1
        if not grown:
            break
    return part


def graph_from_full_dm(ctx: Context, system: System, tb: TBParams, grid, tau: float, kT: float, H=None,
                       S=None) -> Partition:
    """Halos from |D| > tau of the full-system density matrix (small systems)."""
    full = full_system_partition(ctx, system, tb)
    if H is None:
        H, S = ctx.build_hs(system, tb, full.nbr)
    sol = solve(ctx, system, full, H, S, kT, FP64_EIG)
    g = ctx.build_graph_dm(system, GRAPH_DM, full.sg, sol.D_core, tau)
    core, nco = ctx.grid_cores(system, grid)
    sg = ctx.extract_subgraphs(system, tb, g, core, nco)
    return Partition(nbr=full.nbr, graph=g, core_of_atom=core, n_cores=nco, sg=sg, rounds=1, sizes=[sg.norb.copy()])


def rebuild_adaptive(ctx: Context, system: System, tb: TBParams, part: Partition, D_core, tau: float,
                     alpha: float = 0.7, nbr: Graph | None = None) -> Partition:
    """MD-step rebuild: G_tau = (G^N G^D + G^D G^N)|_tau from the previous D."""
    nbr = nbr if nbr is not None else part.nbr
    g = ctx.build_graph_dm(system, GRAPH_ADAPTIVE, part.sg, D_core, tau, alpha=alpha, nbr=nbr)
    sg = ctx.extract_subgraphs(system, tb, g, part.core_of_atom, part.n_cores)
    return Partition(nbr=nbr, graph=g, core_of_atom=part.core_of_atom, n_cores=part.n_cores, sg=sg,
                     rounds=part.rounds + 1, sizes=part.sizes + [sg.norb.copy()])


__all__ = ["Partition", "Solution", "solve", "cutoff_partition", "full_system_partition", "adaptive_partition",
           "graph_from_full_dm", "rebuild_adaptive", "repartition", "balanced_partition", "maybe_repartition",
           "subgraph_cost", "FP64_EIG", "MIXED_F16", "MIXED_BF16", "GRAPH_DM",
           "GRAPH_ADAPTIVE"]
