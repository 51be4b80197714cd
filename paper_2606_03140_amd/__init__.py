"""Graph-partitioned density matrices on MI355X (gfx950).

The density-matrix hot path of graph-based linear-scaling quantum molecular
dynamics: neighbour graph, spatial cores, core+halo subgraphs, per-subgraph
Fermi-operator density matrices at one global chemical potential (FP64
eigensolver path and mixed-precision recursive expansion path), Mulliken
charges and the density-matrix-driven graph of the next step.  All compute
runs in the HIP kernels of libgdm.so (C ABI in include/gdm.h); this package
is the ctypes binding plus thin drivers.
"""
from ._lib import (FP64_EIG, GRAPH_ADAPTIVE, GRAPH_CUTOFF, GRAPH_DM, MIXED_BF16, MIXED_F16, Context, GDMError, Graph,
                   Subgraphs, System, TBParams, load_library)

__all__ = ["Context", "System", "TBParams", "Graph", "Subgraphs", "GDMError", "load_library", "FP64_EIG",
           "MIXED_F16", "MIXED_BF16", "GRAPH_CUTOFF", "GRAPH_DM", "GRAPH_ADAPTIVE"]
