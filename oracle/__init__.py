"""CPU FP64 oracle for graph-partitioned density matrices.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check of the package
entry point and the CPU-baseline leg of the benchmark use it.  It shares no
code with the GPU path; the only common module is `waterbox` (seeded input
geometry, no method arithmetic).

Every function is a plain, slow, readable statement of what the paper
defines, written in NumPy/SciPy with float64 throughout:

* model.py   synthetic tight-binding model (Hamiltonian/overlap), neighbour
             list by brute force.
* graph.py   spatial-grid cores, one-hop halos, atom-condensed density-matrix
             graph and the weighted graph-adaptation rule (Dynamic Graph
             Adaption section, Eq. Graph_Adaptation and Eq. neigh_mat).
* solve.py   per-subgraph Fermi-operator density matrix by dense
             eigendecomposition, global chemical potential by bisection on the
             electron count, collected core rows (Eqs. 1-3 of the Graph-Based
             Linear-Scaling section) and Mulliken charges (SI section D).
* foe.py     the recursive Fermi-operator expansion in exact FP64 arithmetic
             and its closed form.
* ewald.py   periodic point-charge Ewald potential with on-site Hubbard U.
* scc.py     self-consistent-charge loop with linear mixing (the scaled-delta
             kernel of the Shadow MD section and SI section B).
* response.py canonical first-order charge response (fractional
             occupations), the low-rank preconditioned Krylov kernel and the
             quasi-Newton SCF built on it (SI sections B and C).
* learned.py per-atom radial descriptors and the per-species MLP with
             analytic gradients and Adam.
* forces.py  shadow Born-Oppenheimer potential U(R, n) of the linearised
             SCC energy and its forces at fixed n (Shadow MD section):
             band (Hellmann-Feynman, Pulay, SCC shift) from the collected
             core rows of D and of the energy-weighted W, Coulomb, repulsion.
* xlbomd.py  extended-Lagrangian MD: velocity Verlet for the nuclei, Verlet
             with dissipation for the extended charges.

Parity status of each function is listed in its module docstring; a module
that cannot be pinned says "parity unpinned".
"""
