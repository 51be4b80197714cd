/*
 * gdm.h -- graph-partitioned density matrices on MI355X (gfx950).
 *
 * C ABI of the data-parallel hot path of graph-based linear-scaling
 * electronic structure (SEDACS, "Graph-Based Linear-Scaling Electronic-
 * Structure Theory" and "Dynamic Graph Adaption" sections):
 *
 *   neighbour graph -> spatial cores -> core+halo subgraphs -> per-subgraph
 *   D = Z f(Z^T H Z) Z^T at one global chemical potential mu -> collected
 *   core rows of D -> Mulliken charges -> graph of the next step from D.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller unless the
 *   comment says HOST.  The library never frees caller memory.  It owns only
 *   its context and a workspace arena sized by gdm_plan (allocated there, not
 *   in the solve calls).
 * - All device work is enqueued on the stream given to gdm_create (or
 *   gdm_set_stream).  Calls that return a size or a scalar to a HOST pointer
 *   synchronise that stream before returning.
 * - Return value: GDM_OK (0) or a negative GDM_E_* code.  Arguments are
 *   validated on the host before anything is enqueued; on a validation error
 *   nothing is enqueued.  Conditions detected on the device (non-positive-
 *   definite overlap, non-converged iteration, NaN, capacity) are recorded
 *   in the context's device status word and reported by gdm_check and by the
 *   next call that synchronises.  gdm_last_error gives a message.
 * - Matrices are row-major.  Orbitals of an atom are ordered s, px, py, pz
 *   (hydrogen-like species have s only).  A subgraph's atoms are its core
 *   atoms in ascending order followed by its halo atoms in ascending order;
 *   its orbitals follow its atoms.
 * - Density matrices are per spin (occupations in [0, 1]); the electron count
 *   is 2 Tr[D S] (the paper writes Tr[D] = N_occ for an orthonormal basis).
 * - Stream capture: after gdm_find_mu, gdm_subgraph_density and
 *   gdm_mulliken_charges enqueue kernels only (no allocation, host
 *   synchronisation or memset), so both may be captured into a hipGraph on
 *   a non-default stream and replayed; a replay reads the context's state of
 *   the last gdm_find_mu and the mu given at capture.  On the FP64_EIG path
 *   with gdm_set_mu_outputs(ctx, 1), gdm_find_mu enqueues kernels only as
 *   well, so the whole solve (gather, factorisation, eigensolver, mu search,
 *   gdm_subgraph_density_dmu at the device mu, charges) captures into one
 *   graph that a replay runs on the current contents of H and S.  The same
 *   holds on the MIXED_F16 path: with device outputs its search launches a
 *   fixed number of expansion passes, doublings and inverse-overlap rounds
 *   (gdm_set_mixed_capture) and the device skips those it does not need.
 */
#ifndef GDM_H
#define GDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GDM_OK = 0,
    GDM_E_ARG = -1,           /* bad argument (null, size, range)                  */
    GDM_E_CAPACITY = -2,      /* output capacity too small; required size returned */
    GDM_E_NOT_PD = -3,        /* a subgraph overlap matrix is not positive definite */
    GDM_E_NO_BRACKET = -4,    /* electron count cannot be matched inside the bracket */
    GDM_E_NOT_CONVERGED = -5, /* an iteration hit its cap                          */
    GDM_E_NAN = -6,           /* NaN or Inf produced                               */
    GDM_E_HIP = -7,           /* HIP runtime error                                 */
    GDM_E_STATE = -8          /* call order violated (e.g. density before find_mu) */
};

enum { GDM_GRAPH_CUTOFF = 0, GDM_GRAPH_DM = 1, GDM_GRAPH_ADAPTIVE = 2 };

/* Subgraph solver.  GDM_FP64_EIG: FP64 Cholesky basis + FP64 symmetric
 * eigendecomposition (the "direct diagonalization" option; subgraphs of at
 * most 2048 orbitals).  GDM_MIXED_F16: GEMM-only recursive Fermi-operator
 * expansion with split FP16 operands (x = hi + 2^-11 lo, 22 significant
 * bits) and FP32 accumulation on the matrix cores, FP64 for bounds, traces,
 * mu and the final step (the recursive-FOE option).  GDM_MIXED_BF16: the
 * same expansion with split BF16 operands (x = hi + 2^-8 lo, 16 significant
 * bits, BF16 MFMA): same data volume and speed, rounding errors 2^6 times
 * larger.  Every call documented for GDM_MIXED_F16 (options, capture,
 * statistics, charge response) applies to GDM_MIXED_BF16 alike. */
enum { GDM_FP64_EIG = 0, GDM_MIXED_F16 = 1, GDM_MIXED_BF16 = 2 };

typedef struct gdm_ctx gdm_ctx;

/* The full system (Interface section: coordinates, atom types, lattice
 * vectors, orbital indices). */
typedef struct {
    int32_t n_atoms;
    const double* pos;        /* [n_atoms*3] A, wrapped into [0, box)            */
    const int32_t* species;   /* [n_atoms] 0 (O-like: s,p) or 1 (H-like: s)      */
    const int32_t* anchor;    /* [n_atoms] atom whose position picks the core cell
                                 (the O of a water for both its H)              */
    const int32_t* orb_ptr;   /* [n_atoms+1] first global orbital of each atom   */
    double box[3];            /* orthorhombic periodic box edges, A              */
    double inv_box[3];        /* 1/box as computed by the caller; used as given so
                                 that minimum images are reproducible bit for bit */
} gdm_system;

/* Synthetic two-centre tight-binding model (stand-in for the SCC-DFTB tables):
 * V(r) = v0 exp(-(r - v_r0)/v_decay), S(r) = s0 exp(-(r - s_r0)/s_decay) for
 * r < cutoff, Slater-Koster sigma blocks with direction cosines from the row
 * atom, V_pp_pi = 0.  For molecular dynamics (forces) the radial functions
 * can be tapered to zero with two continuous derivatives: with
 * taper_on > 0 they are multiplied by t(r) = 1 - x^3 (10 - 15 x + 6 x^2),
 * x = (r - taper_on)/(cutoff - taper_on), between taper_on and cutoff; the
 * repulsive pair energy sum_{I<J} rep_A[pair] exp(-r/rep_rho) t(r) (pair 0
 * O-O, 1 O-H, 2 H-H; used by gdm_forces only) stands in for the repulsive
 * term of SCC-DFTB, which the synthetic model otherwise lacks. */
typedef struct {
    double onsite[2][4];      /* eV per species and orbital type (s, px, py, pz) */
    int32_t n_orb[2];         /* orbitals per species: 4 and 1                  */
    double v0, v_r0, v_decay;
    double s0, s_r0, s_decay;
    double cutoff;            /* A, strict r < cutoff                            */
    int32_t orthogonal;       /* 1: S = I                                        */
    double taper_on;          /* A; 0: hard cutoff (no taper)                    */
    double rep_A[3];          /* eV, repulsive prefactors O-O, O-H, H-H           */
    double rep_rho;           /* A, repulsive decay length (> 0 when rep_A used)  */
} gdm_tb_params;

/* Subgraph set.  Device arrays plus HOST copies of the per-subgraph sizes
 * (planning needs them on the host). */
typedef struct {
    int32_t n_sub;
    const int32_t* atom_ptr;     /* [n_sub+1]                                      */
    const int32_t* atoms;        /* [atom_ptr[n_sub]] core ascending, then halo ascending */
    const int32_t* n_core;       /* [n_sub] core atoms per subgraph                 */
    const int32_t* h_norb;       /* HOST [n_sub] orbitals n_s of each subgraph       */
    const int32_t* h_ncore_orb;  /* HOST [n_sub] core orbitals nc_s                  */
} gdm_subgraphs;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (NULL:
 * the default stream).  Allocates the device status word. */
int gdm_create(gdm_ctx** out, int device, void* hip_stream);
int gdm_destroy(gdm_ctx* ctx);
int gdm_set_stream(gdm_ctx* ctx, void* hip_stream);
/* Message of the last error recorded in the context (never NULL). */
const char* gdm_last_error(const gdm_ctx* ctx);
/* Synchronise the stream and return the device status word as a GDM code
 * (GDM_OK if no device-side condition was raised); clears it. */
int gdm_check(gdm_ctx* ctx);

/* ------------------------------------------------------------ graph: a1, a3 */

/* Build the atom graph as CSR (rows ascending, columns ascending, no self
 * edges).
 *  mode GDM_GRAPH_CUTOFF: edge (i, j) iff r_ij^2 < cutoff^2 with the minimum
 *    image d = x_j - x_i, d -= L rint(d inv_L), r^2 = (dx dx + dy dy) + dz dz
 *    evaluated without contraction (Determining the Subgraphs: initial graph
 *    from a distance neighbour list).  Cell-list search.
 *  mode GDM_GRAPH_DM: edge iff max(G^D_ij, G^D_ji) > tau, where G^D is the
 *    atom-condensed |D| (largest |D_ab| of each atom-atom block) taken from the
 *    collected core rows `D_core` of subgraph set `prev` (packed as written by
 *    gdm_subgraph_density).
 *  mode GDM_GRAPH_ADAPTIVE: edge iff max(W_ij, W_ji) > tau with
 *    W = G^N G^D + G^D G^N, G^N_ij = exp(-alpha r_ij^2) on the neighbour CSR
 *    (nbr_row_ptr, nbr_col) plus G^N_ii = 1 (Eq. neigh_mat, Eq.
 *    Graph_Adaptation).
 * `union_row_ptr/union_col` (nullable, DM and ADAPTIVE modes): edges of this
 * graph are kept as well (the initial-SCF rule: edges are only added).
 * Output: row_ptr [n_atoms+1], col [cap].  *nnz_out (HOST) receives the edge
 * count; if it exceeds cap the call returns GDM_E_CAPACITY and col is not
 * written. */
int gdm_build_graph(gdm_ctx* ctx, const gdm_system* sys, int mode, double cutoff,
                    double alpha, double tau,
                    const gdm_subgraphs* prev, const double* D_core,
                    const int32_t* nbr_row_ptr, const int32_t* nbr_col,
                    const int32_t* union_row_ptr, const int32_t* union_col,
                    int32_t* row_ptr, int32_t* col, int64_t cap, int64_t* nnz_out);

/* ----------------------------------------------------- partition: a4, a5 */

/* Spatial-grid core partition (stand-in for the community detection of
 * Determining the Subgraphs): per axis cell = min(g-1, floor((x inv_L) g)) of
 * the anchor atom's position, id = (i g_y + j) g_z + k; empty cells skipped,
 * remaining cells numbered in ascending id.  core_of_atom [n_atoms];
 * *n_cores_out HOST. */
int gdm_grid_cores(gdm_ctx* ctx, const gdm_system* sys, const int32_t grid[3],
                   int32_t* core_of_atom, int32_t* n_cores_out);

/* Cost-balanced core partition for re-partitioning (Determining the
 * Subgraphs: a new core partitioning when the halos have grown, Fig.
 * graph_partition f; Scalability section: subgraph cost grows as its size
 * cubed).  Weighted recursive coordinate bisection of the molecules (atoms
 * with anchor[a] == a, at their wrapped positions): a set that must form k
 * cores is sorted along its widest axis (ties by index) and cut where the
 * running weight is closest to k/2 / k of its total, keeping at least one
 * molecule per core; both sides recurse.  A molecule weighs the number of its
 * atoms plus their degrees in the graph row_ptr (DEVICE [n_atoms + 1],
 * nullable: atom counts only), so cores shrink where the graph is dense.
 * core_of_atom DEVICE [n_atoms] (cores 0 .. n_cores-1, every core
 * non-empty).  GDM_E_ARG for n_cores outside [1, molecules] or an atom whose
 * anchor does not anchor itself.  Synchronises the stream (host algorithm). */
int gdm_balanced_cores(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr, int32_t n_cores,
                       int32_t* core_of_atom);

/* The bisection of gdm_balanced_cores on host arrays (no context, no GPU):
 * xyz HOST [n x 3], weight HOST [n] (nullable: all 1; each > 0),
 * part HOST [n] out (0 .. n_parts-1).  GDM_E_ARG for n <= 0,
 * n_parts outside [1, n] or a non-finite value. */
int gdm_rcb_partition(const double* xyz, const double* weight, int32_t n, int32_t n_parts, int32_t* part);

/* Core+halo subgraphs (Fig. graph_partition b-c; SI section A): the halo of a
 * core is every atom outside it with an edge to one of its atoms.  Outputs
 * atom_ptr [n_cores+1], atoms [cap_atoms], n_core [n_cores]; HOST outputs
 * h_norb [n_cores], h_ncore_orb [n_cores] (orbital counts, nullable) and
 * *total_atoms_out.  GDM_E_CAPACITY if the packed atom list exceeds
 * cap_atoms (nothing written to atoms).  n_atoms <= 1,000,000. */
int gdm_extract_subgraphs(gdm_ctx* ctx, const gdm_system* sys, const gdm_tb_params* tb,
                          const int32_t* row_ptr, const int32_t* col,
                          const int32_t* core_of_atom, int32_t n_cores,
                          int32_t* atom_ptr, int32_t* atoms, int64_t cap_atoms,
                          int32_t* n_core, int32_t* h_norb, int32_t* h_ncore_orb,
                          int64_t* total_atoms_out);

/* ------------------------------------------------------- H and S: a2 */

/* Block-sparse H and S over the neighbour CSR (row_ptr, col, nnz edges):
 * block k < nnz is edge k, block nnz + i is atom i's on-site block; every
 * block is 4x4 doubles row-major over (s, px, py, pz) (unused entries 0).
 * V_atom (nullable, eV per atom) adds the SCC shift 1/2 S_ab (V_I + V_J)
 * (SI section D).  H, S: [(nnz + n_atoms) * 16]; S may be NULL when
 * tb->orthogonal. */
int gdm_build_hs(gdm_ctx* ctx, const gdm_system* sys, const gdm_tb_params* tb,
                 const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                 const double* V_atom, double* H, double* S);

/* ------------------------------------------------- subgraph solve: a6-a14 */

/* Size the workspace for subgraph set `sg` and solver `precision` and record
 * the plan (per-subgraph offsets of the dense tiles, and for GDM_MIXED_F16 the
 * tile lists of the matrix-core products, built largest subgraph first over
 * eight per-XCD queues).  The only call of the solve path that allocates.  Required before gdm_find_mu.  Subgraphs hold at most 8,192
 * orbitals (GDM_E_ARG otherwise); a failed plan leaves no plan, so the
 * solve calls then return GDM_E_STATE until a plan succeeds. */
int gdm_plan(gdm_ctx* ctx, const gdm_subgraphs* sg, int precision);

/* Gather every subgraph's principal submatrices h, s from the block-sparse
 * H, S (one workgroup per subgraph; its atom list and orbital offsets staged in
 * LDS, the blocks of each atom's neighbour edges copied into the dense tiles),
 * solve it with `precision`, and find the global chemical
 * potential mu with N(mu) = 2 sum_s sum_k w_k f(lam_k) = n_electrons
 * (Density Matrix Evaluation on Partitioned Graphs: mu fixes the occupation).
 * FP64_EIG: multisection on the eigenvalues and core weights to an interval
 * of 1e-12 eV, mu_guess ignored.  MIXED_F16: Newton steps from mu_guess on
 * FP64 core traces with a bisection safeguard, one full expansion per pass,
 * until |N - n_electrons| <= max(tol_N, 1e-10 n_electrons), or the Newton
 * step is below 1e-2 kT, or the pass budget runs out; the first-order
 * correction mu + (n_electrons - N)/N'(mu) is then applied when the count is
 * not yet matched and the correction lies within kT, and the result must
 * count within max(tol_N, 1e-7 n_electrons) (the rounding level of the
 * traces), else GDM_E_NO_BRACKET.  The search converges to where the mixed
 * count equals n_electrons (not to the first mu inside the count's rounding
 * level): inside a gap N(mu) is nearly flat, and only the zero of the count
 * places mu where the FP64 path does, to the count's rounding bias divided by
 * N'(mu).  *mu_out, *n_out HOST (DEVICE scalars after
 * gdm_set_mu_outputs(ctx, 1)).  The factorisation / expansion state is cached
 * in the context for gdm_subgraph_density. */
int gdm_find_mu(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                const double* H, const double* S, double n_electrons, double kT,
                int precision, double mu_guess, double tol_N,
                double* mu_out, double* n_out);

/* Where gdm_find_mu puts mu and N(mu).  device = 0 (default): HOST pointers;
 * the call synchronises the stream and checks the electron count on the
 * host.  device = 1: DEVICE pointers to one double each; the whole search is
 * enqueued without host synchronisation, so gdm_find_mu can be captured into
 * a hipGraph with the density and charge calls (gdm_subgraph_density_dmu at
 * the device mu), and a count off by more than the tolerance (FP64_EIG
 * 1e-6 n_electrons, MIXED_F16 max(tol_N, 1e-7 n_electrons)) or a NaN is
 * recorded in the device status word, reported by gdm_check.  MIXED_F16 with
 * device outputs: the search starts from *mu_out's value when it is finite
 * and inside the spectral bounds (the previous result, so a replayed graph
 * warm-starts from the last step; the caller writes NaN to start from
 * mu_guess), runs at most the passes set by gdm_set_mixed_capture with the
 * degree-7 start and at least 5 doublings, and does not record the expansion
 * for the charge response (GDM_E_ARG while gdm_set_response is on).  A
 * setting of the context, kept until changed.  Returns GDM_E_ARG for other
 * values of device. */
int gdm_set_mu_outputs(gdm_ctx* ctx, int device);

/* Launch budget of the MIXED_F16 search with device outputs: `passes`
 * expansion passes (1..16, default 3) of `nd_launch` doublings each (5..40,
 * default 12); a pass or a doubling the search does not need exits at once
 * on the device.  A problem needing more doublings than nd_launch (spectral
 * half-width R with beta R > 8 * 2^nd_launch) raises GDM_E_CAPACITY in the
 * status word.  The host-driven search (device outputs off) is unaffected. */
int gdm_set_mixed_capture(gdm_ctx* ctx, int passes, int nd_launch);

/* State of the last MIXED_F16 search (HOST outputs, nullable; synchronises):
 * the chemical potential of its last expansion pass, the electron count N
 * there and dN/dmu = beta M.  D of gdm_subgraph_density is evaluated to first
 * order about mu_pass. */
int gdm_mixed_mu_state(gdm_ctx* ctx, double* mu_pass, double* n_pass, double* slope);

/* Collected core rows D[core, :] of every subgraph (Eq. 3) at chemical
 * potential mu, from the state cached by gdm_find_mu (same precision).
 * Output packed in subgraph order: subgraph s occupies nc_s * n_s doubles,
 * row-major (core orbital, subgraph orbital), at offset sum_{t<s} nc_t n_t.
 * eig_out (nullable): FP64_EIG only, eigenvalues packed at sum_{t<s} n_t.
 * FP64_EIG: any mu (the eigenpairs are exact for every occupation).
 * MIXED_F16: the expansion was evaluated at the chemical potential mu_p of
 * gdm_find_mu's last pass and at its kT; D(mu) is taken to first order,
 * D(mu_p) + (mu - mu_p) beta Z X (I - X) Z^T, which holds only near mu_p, so
 * kT must equal gdm_find_mu's (relative 1e-12) and |mu - mu_p| <= kT, else
 * GDM_E_ARG (nothing enqueued).  The mu that gdm_find_mu returns always
 * satisfies this. */
int gdm_subgraph_density(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, double kT,
                         int precision, double* D_core, double* eig_out);

/* gdm_subgraph_density at a chemical potential held in DEVICE memory
 * (*mu_device, read when the kernel runs), e.g. the mu_out of a gdm_find_mu in
 * device-output mode (gdm_set_mu_outputs), so that a captured graph of
 * gdm_find_mu, this call and gdm_mulliken_charges uses the mu each replay
 * finds.  MIXED_F16: D is taken to first order about the last pass's mu (read
 * on the device too), which the mu of a device-side search keeps within kT;
 * kT must equal gdm_find_mu's.  D_core as for gdm_subgraph_density.
 * GDM_E_ARG for null pointers or another kT; GDM_E_STATE before
 * gdm_find_mu. */
int gdm_subgraph_density_dmu(gdm_ctx* ctx, const gdm_subgraphs* sg, const double* mu_device, double kT,
                             int precision, double* D_core);

/* Mulliken charges from the collected core rows (SI section D):
 * q_I = 2 sum_{a in I} sum_b D_ab S_ba - n0[species_I] for every atom (each
 * atom is a core atom of exactly one subgraph).  S is read from the
 * block-sparse overlap (NULL: orthogonal).  n0 HOST [2]; q_out [n_atoms]. */
int gdm_mulliken_charges(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                         const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                         const double* S, const double* D_core, const double n0[2],
                         double* q_out);

/* ------------------------------------------------- forces and XL-BOMD (MD) */

/* Energy-weighted density core rows W[core,:] = C[core,:] diag(f lam) C^T of
 * every subgraph (C the generalized eigenvectors, lam the eigenvalues, f the
 * Fermi occupations at mu, kT), the matrix of the Pulay term of the forces
 * (Shadow MD section: forces of the shadow potential at fixed n).  FP64_EIG
 * path only, after gdm_find_mu, with the same mu and kT as the density.
 * W_core packed like gdm_subgraph_density's D_core.  GDM_E_STATE before
 * gdm_find_mu or on another planned precision. */
int gdm_subgraph_edm(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, double kT, double* W_core);

/* Electronic free energy of the collected solve (the band term of the shadow
 * potential, Shadow MD section):
 *   Omega = 2 sum_s sum_k w_k [f_k lam_k + kT (f_k ln f_k + (1 - f_k) ln(1 - f_k))]
 * with the core weights w_k of each subgraph (0 ln 0 = 0), at mu and kT.
 * FP64_EIG path only, after gdm_find_mu.  *omega_out HOST (eV).
 * Synchronises the stream. */
int gdm_band_energy(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, double kT, double* omega_out);

/* Forces of the shadow Born-Oppenheimer potential at fixed extended charges n
 * (Shadow MD section, nuclear equation of motion), except the Coulomb term
 * (gdm_ewald_forces adds it):
 *   F_I = sum_{J in nbr(I)} grad_d e_IJ(d),  d = R_J - R_I (minimum image),
 *   e_IJ = 4 sum_{a in I, b in J} [Dbar_ab (H0_ab + S_ab (V_I + V_J)/2) - Wbar_ab S_ab]
 *          + rep_A[pair] exp(-r/rep_rho) t(r),
 * the Hellmann-Feynman, Pulay and SCC-shift terms of -2 Tr[D dH[n]/dR] +
 * 2 Tr[W dS/dR] and the repulsion, with Dbar = (D_IJ + D_JI^T)/2 from the core
 * rows of I's and J's subgraphs (a block whose far atom is outside the
 * subgraph counts as zero) and Wbar likewise; H0, S, the taper t and the
 * repulsion as in gdm_tb_params.  row_ptr/col/nnz: the neighbour CSR H and S
 * were built on; sg: the planned subgraph set (every atom a core atom of
 * exactly one subgraph, else the status word reports GDM_E_ARG at
 * gdm_check); D_core, W_core: gdm_subgraph_density and gdm_subgraph_edm
 * output; V_atom [n_atoms] (nullable: no SCC shift) the potential H was
 * built with.  F [n_atoms x 3] eV/A, overwritten.  energy (DEVICE [2],
 * nullable): energy[0] = the repulsive energy, energy[1] =
 * -sum_I (n0[species_I] + n_vec_I / 2) V_I (0 when V_atom or n_vec is NULL;
 * n0 HOST [2] then required); with gdm_band_energy they give
 * U(R, n) = Omega + energy[0] + energy[1].  Enqueues kernels only; the
 * per-pair workspace (32 B per CSR entry) grows on demand. */
int gdm_forces(gdm_ctx* ctx, const gdm_system* sys, const gdm_tb_params* tb, const int32_t* row_ptr,
               const int32_t* col, int64_t nnz, const gdm_subgraphs* sg, const double* D_core,
               const double* W_core, const double* V_atom, const double n0[2], const double* n_vec,
               double* F, double* energy);

/* Velocity Verlet half step of XL-BOMD (Shadow MD section, nuclear equation
 * of motion): vel += dt/2 F / m (m = mass[species], HOST [2] amu; F eV/A;
 * vel A/fs, [n x 3]); then, when pos is not NULL, pos += dt vel (A).
 * kinetic (DEVICE [1], nullable): 1/2 sum m vel^2 in eV after the update.
 * Enqueues kernels only. */
int gdm_md_verlet(gdm_ctx* ctx, int32_t n, const int32_t* species, const double mass[2], double dt,
                  const double* F, double* vel, double* pos, double* kinetic);

/* Extended charges of XL-BOMD (Shadow MD section, harmonic equation of the
 * extended density with the kernel K, Verlet form with the dissipation of
 * Niklasson et al., J. Chem. Phys. 130, 214109 (2009), K = 5):
 *   n_{t+1} = 2 n_t - n_{t-1} + kappa_c d + alpha sum_k c_k n_{t-k},
 *   c = (-6, 14, -8, -3, 4, -1), d = K (q[n_t] - n_t):
 *   delta NULL: d = q - n_t (the kernel c I with kappa_c = kappa c);
 *   else d = delta (e.g. -J^-1 (q - n_t) from the low-rank Krylov kernel of
 *   gdm_krylov_*, with kappa_c = kappa);  kappa = 1.82, alpha = 0.018 in
 *   that reference.
 * hist DEVICE [6 x n]: row k holds n_{t-k}; it is shifted in place so that
 * row 0 becomes n_{t+1}.  q = q[n_t] [n] (used when delta is NULL), delta
 * [n] (nullable); n_out [n] (nullable) receives n_{t+1}.  Enqueues one
 * kernel. */
int gdm_xlbomd_charges(gdm_ctx* ctx, int32_t n, const double* q, const double* delta, double* hist,
                       double kappa_c, double alpha, double* n_out);

/* out = a x + b y over n doubles (device; out may alias x or y): the charge
 * vectors of the finite-difference responses of the XL-BOMD kernel.
 * Enqueues one kernel. */
int gdm_axpby(gdm_ctx* ctx, int32_t n, double a, const double* x, double b, const double* y, double* out);

/* Options of the mixed-precision expansion (GDM_MIXED_F16; its last doubling
 * of every pass runs in FP64 on the matrix cores, which squares away the
 * split products' errors in the fully occupied and empty states so that the
 * electron count carries no systematic bias).  ns_z: coupled
 * Newton-Schulz iterations for s^-1/2 to try first (default 3).  With x the
 * eigenvalues of s/c (c the largest absolute row sum) and the start
 * Z0 = 2.598551 I - 1.834840 s/c (the linear minimax approximation of
 * x^-1/2 for |1 - x z^2| on [0.1, 1]: e0 <= 0.417 there), the error falls
 * as e -> 3/4 e^2 + 1/4 e^3, and one third-order residual refinement
 * step Z <- Z (I - E/2 + 3/8 E^2), E = Z s Z - I (E in FP64, the correction
 * terms on the split products), then cubes it; before that
 * step gdm_find_mu checks max |E_ij| and, while it exceeds 1e-3, runs one
 * more iteration,
 * at most ns_z_extra times (default 8), after which it returns
 * GDM_E_NOT_CONVERGED (overlap too ill-conditioned).  ns_inv: Newton-Schulz
 * iterations per inverse in each doubling after its minimax start (default
 * 1; a start with error e0 reaches e0^(2^k) after k iterations, see
 * gdm_set_mixed_inverse_start).  max_passes: expansion
 * passes allowed while matching the electron count (default 16: a cold
 * start next to subgraph states near mu can need 9 Newton/bisection passes;
 * a warm start from the previous mu takes 1).  Values
 * <= 0 (ns_z_extra: < 0) keep the current setting. */
int gdm_set_mixed_options(gdm_ctx* ctx, int ns_z, int ns_inv, int max_passes, int ns_z_extra);

/* Options of the FP64 path, read by the next gdm_plan: the largest leaf of
 * the tridiagonal divide and conquer (leaves are solved by QL with the
 * eigenvectors accumulated, one wave each; smaller leaves shorten that
 * serial chain and add a merge level).  leaf_rows in [8, 64] (default 64);
 * GDM_E_ARG otherwise.  Results agree to FP64 rounding for every value. */
int gdm_set_fp64_options(gdm_ctx* ctx, int leaf_rows);

/* Storage of the symmetric matrices of a MIXED_F16 expansion pass (the start
 * polynomial, X_k, X_k^2, 2 X_k^2 - 2 X_k + I, its inverse and Newton-Schulz
 * factors).  upper_tiles = 1 (default): only the upper 64 x 64 tiles are
 * written, and a product reads a lower tile as the stored upper tile
 * transposed, which cuts the HBM traffic of those products by about a third
 * at the benchmark sizes.  With upper_tiles = 0 every product also writes
 * the mirror tiles, from registers with its own rounding of the epilogue,
 * so those lower tiles may differ from the upper ones in the last bit; the
 * two settings agree to FP32 rounding.  The pass's final X and passes
 * recorded for the charge response are always stored whole.  GDM_E_ARG for
 * other values. */
int gdm_set_mixed_storage(gdm_ctx* ctx, int upper_tiles);

/* Start of the Newton-Schulz inverse of A = 2 X^2 - 2 X + I in every doubling
 * of a MIXED_F16 / MIXED_BF16 pass (the A^-1 of Eq. 3's recursive expansion;
 * eigenvalues of A in [1/2, 1]): the minimax polynomial of the given degree,
 * whose residual |1 - a y(a)| on [1/2, 1] is at most 1/|T_{d+1}(3)| (T the
 * Chebyshev polynomial).  degree = 4 (default): two products, residual
 * <= 1/3363, then ns_inv = 1 step reaches 8.8e-8; degree = 2: one product,
 * residual <= 1/99, two steps reach 1.0e-8 (one product more per doubling).
 * Read by the next gdm_find_mu; GDM_E_ARG for other degrees. */
int gdm_set_mixed_inverse_start(gdm_ctx* ctx, int degree);

/* Statistics of the last GDM_MIXED_F16 gdm_find_mu (HOST outputs, nullable):
 * expansion passes, doublings per pass, split GEMM launches, and the mean
 * flops of one split GEMM launch counted once per product (2 P^2 per output
 * tile row of P, over the tiles computed: products of commuting symmetric
 * matrices compute the upper tiles only); each launch executes three FP16
 * products.  bytes_per_launch: mean algorithmic HBM bytes of a launch (each
 * operand, E matrix and output read or written once, over their upper tiles
 * for matrices in upper-tile storage, gdm_set_mixed_storage).  ns_z_used: coupled
 * Newton-Schulz iterations taken for s^-1/2. */
int gdm_mixed_stats(gdm_ctx* ctx, int* passes, int* n_doublings, int64_t* gemm_launches,
                    double* flops_per_launch, double* bytes_per_launch, int* ns_z_used);

/* Diagnostics: copy the FP32 matrix `which` (0 Z, the inverse-overlap
 * factor before FP64 refinement; 1 h_perp; 2 X of the last expansion pass)
 * of subgraph `sub` of the last GDM_MIXED_F16 solve into `out` (device, P*P
 * floats, P the padded size = 64 ceil(n/64)). */
int gdm_debug_slot(gdm_ctx* ctx, int which, int sub, float* out);

/* -------------------------------------------- SCC shell: Coulomb and mixing */

/* Periodic Coulomb potential of the net Mulliken charges q (e) for the
 * self-consistent-charge Hamiltonian (SI section D: 1/R at large separation,
 * screened where the charge densities overlap, Hubbard U on site; the
 * paper's all-to-all Coulomb sum of the Scalability section), in eV:
 *   V_I = U[species_I] q_I + k_e [ sum_{J != I, r < rcut} q_J (erfc(eta r)/r - S_IJ(r))
 *         + (4 pi / vol) sum_{k != 0, |k| <= 2 pi k_max / max(L)} exp(-k^2/4eta^2)/k^2
 *           sum_J q_J cos(k . (R_J - R_I))  -  2 eta / sqrt(pi) q_I ],
 * k_e = 14.399645 eV A, neutralising background (k = 0 dropped), minimum
 * image in the real-space sum.  S_IJ(r): the short-range part of the
 * interaction of two exponential charge densities tau^3/(8 pi) exp(-tau r)
 * with tau = tau[species] (HOST [2], 1/A; 16/5 U in atomic units), so that
 * 1/r - S -> U as r -> 0; tau NULL gives bare point charges.
 * row_ptr/col: a neighbour CSR containing every pair with r < rcut (e.g.
 * gdm_build_graph CUTOFF at rcut, or at rcut + skin: pairs at r >= rcut are
 * skipped).  Requires 2 rcut < every box side,
 * eta > 0, 1 <= k_max <= 64; hubbard_U HOST [2] eV.  q, V: [n_atoms] FP64.
 * Accuracy is the caller's choice of (rcut, eta, k_max): erfc(eta rcut),
 * exp(-(pi k_max / (eta L))^2) and S(rcut) bound the truncation.
 * Enqueues kernels only (no host synchronisation): the k-vector table is
 * built on the device over the full grid a = 0..k_max, b, c = -k_max..k_max
 * with zero weight outside the half space and the sphere, in context
 * workspace (grown on the first call for a larger k_max or atom count). */
int gdm_ewald_potential(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr,
                        const int32_t* col, double rcut, double eta, int32_t k_max,
                        const double hubbard_U[2], const double* tau, const double* q, double* V);

/* Coulomb forces of the shadow potential (Shadow MD section): F += -d/dR of
 * q^T gamma n - n^T gamma n / 2 = 1/2 (2q - n)^T gamma n at fixed q and n,
 * with gamma the kernel of gdm_ewald_potential without the on-site U (which
 * does not depend on the positions); q = q[n] the Mulliken charges, n_vec
 * the extended charges (q = n_vec gives the plain Coulomb force of
 * 1/2 q^T gamma q).  Real space over
 * row_ptr/col (pairs at r >= rcut skipped), reciprocal space over the
 * half space of k with |k| <= 2 pi k_max / max(L); tau (HOST [2], nullable)
 * adds the derivative of the screening.  Same limits as
 * gdm_ewald_potential (2 rcut < every box side, 1 <= k_max <= 64).
 * q, n_vec [n_atoms]; F [n_atoms x 3] eV/A, ADDED to.  Enqueues kernels
 * only; its k-vector table and structure factors use context workspace. */
int gdm_ewald_forces(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr, const int32_t* col,
                     double rcut, double eta, int32_t k_max, const double* tau, const double* q,
                     const double* n_vec, double* F);

/* gdm_ewald_potential without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments and result (to FP64
 * rounding: its k-vector table is built on the device over the full grid
 * a = 0..k_max, b, c = -k_max..k_max, with zero weight outside the half space
 * and the sphere), 1 <= k_max <= 32 (GDM_E_ARG above).  Its working memory is
 * a fixed device array of the library (6.7 MB per GPU, held until the process
 * ends) rather than context workspace; every call on one GPU shares it, so
 * calls that overlap on one GPU (two streams, two contexts) race and must be
 * ordered by the caller.  Enqueues kernels only (no host synchronisation,
 * allocation or memset), so it may be captured into a hipGraph. */
int gdm_ewald_potential_noalloc(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr,
                                const int32_t* col, double rcut, double eta, int32_t k_max,
                                const double hubbard_U[2], const double* tau, const double* q, double* V);

/* Linear charge mixing of the SCC iteration, the scaled-delta kernel
 * K = -c I of the Shadow MD section: n <- n + mix (q0 - n), and the RMS of
 * the residual q0 - n before the update (HOST *rms_out).  n_vec, q0: [n].
 * Synchronises the stream. */
int gdm_scc_mix(gdm_ctx* ctx, int32_t n, double* n_vec, const double* q0, double mix,
                double* rms_out);

/* Anderson-accelerated update of the same fixed-point iteration (memory
 * depth <= 8, mixing mix): with F = q0 - n stored as the k-th iterate
 * (k = 0, 1, ... counts the calls of one SCC run) and the differences dF_j,
 * dn_j of the last min(depth, k) consecutive iterates,
 * gamma = argmin || F - sum_j gamma_j dF_j || (QR by modified Gram-Schmidt;
 * columns that are numerically dependent are dropped) and
 * n <- n + mix F - sum_j gamma_j (dn_j + mix dF_j).  depth 0 is linear
 * mixing.  work: caller-owned FP64 [(3 depth + 2) n], kept between the calls
 * of one run (the iterate history).  *rms_out (HOST): RMS of F.
 * Synchronises the stream. */
int gdm_scc_anderson(gdm_ctx* ctx, int32_t n, double* n_vec, const double* q0, double mix,
                     int32_t depth, int32_t k, double* work, double* rms_out);

/* ------------------------------- charge response and kernel-accelerated SCF */

/* Keep the doubling history of the mixed-precision expansion (GDM_MIXED_F16)
 * so that gdm_density_response can differentiate it: every later
 * gdm_find_mu stores X_k and the inverse Y_k = (2 X_k^2 - 2 X_k + I)^-1 of
 * each doubling of its last expansion pass, if the pass has at most
 * max_doublings doublings (ceil(log2(beta * spectral radius)): 9 for
 * kT = 0.1 eV and a 30 eV half-width).  Allocates 8 * max_doublings bytes
 * per padded matrix element (P = 64 ceil(n/64), sum of P^2 over the
 * subgraphs) plus the FP64 response workspace, now if a GDM_MIXED_F16 plan
 * exists, else at the next gdm_plan; max_doublings = 0 stops recording and
 * frees it.  0 <= max_doublings <= 40. */
int gdm_set_response(gdm_ctx* ctx, int max_doublings);

/* Canonical first-order response of the collected Mulliken charges to a
 * change dV of the atomic potentials (SI section B: the directional
 * derivatives of the charge residual that build the low-rank kernel, by
 * perturbation theory at fractional occupation).  The SCC Hamiltonian
 * changes by dH_ab = 1/2 S_ab (dV_I + dV_J); in each subgraph
 * dD = d/dlambda Z f(Z^T (h + lambda dh) Z) Z^T at fixed mu, computed as the
 * exact derivative of the recorded recursive expansion of the last
 * gdm_find_mu (three split-FP16 products per doubling), plus the chemical
 * potential shift dmu dD/dmu with dmu chosen so that the electron count
 * 2 sum_s Tr_core[dD s] stays unchanged.  dq_I = 2 sum_{a in I} (dD S)_aa.
 * Requires gdm_find_mu with GDM_MIXED_F16 after gdm_set_response with room
 * for its doublings (GDM_E_STATE otherwise); the state it reads is that of
 * the last find_mu and the last gdm_subgraph_density.  row_ptr/col/nnz/S as
 * for gdm_mulliken_charges; dV, dq_out [n_atoms] FP64; *dmu_out (HOST,
 * nullable) receives dmu.  The response is linear in dV.  Synchronises the
 * stream. */
int gdm_density_response(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                         const int32_t* row_ptr, const int32_t* col, int64_t nnz, const double* S,
                         const double* dV, double* dq_out, double* dmu_out);

/* Quasi-Newton SCF step with the low-rank preconditioned Krylov kernel (SI
 * sections B and C): n <- n - alpha (K0 J)^-1 K0 f(n), f = q0[n] - n,
 * J = df/dn, K0 = -k0 I (the scaled-delta kernel), and (K0 J)^-1 on
 * r = K0 f approximated by sum_ij v_i M_ij f_vj^T r over orthonormal
 * preconditioned Krylov vectors v_0 ~ r, v_{j+1} ~ K0 J v_j, f_vj = K0 J v_j,
 * M = (F_v^T F_v)^-1 (computed as the least-squares fit F_v c = r by QR).
 * Optionally ("complete") the part of r the vectors do not fit, r - F_v c,
 * is added as is, taking (K0 J)^-1 as the identity there (exact when
 * K0 = J^-1; with a complete basis the remainder is zero).  One step:
 *   gdm_krylov_begin: r and v_0 from n_vec and q0 = q0[n]; *rms_out (HOST)
 *     = RMS(f).  k0 > 0.
 *   for j = 0, 1, ...: the caller evaluates J v_j + v_j = dq_j, the charge
 *     response to the potential of the charges v_j (v_j is work + n + j n),
 *     and gdm_krylov_add fits it; *rel_out (HOST) = ||F_v c - r|| / ||r||,
 *     *exhausted_out (HOST, nullable) = 1 when no new direction exists.
 *     Stop when rel_out is small enough or j + 1 = max_rank.
 *   gdm_krylov_apply: n_vec <- n_vec - alpha (V c + complete (r - F_v c))
 *     with the first `rank` vectors; may be called again on a saved n_vec
 *     with a smaller alpha (line search) until the next begin.
 * work: caller-owned FP64 [(2 max_rank + 1) n + max_rank^2 + 2 max_rank + 2],
 * kept over the calls of one step.  1 <= max_rank <= 16.  begin and add
 * synchronise the stream. */
int gdm_krylov_begin(gdm_ctx* ctx, int32_t n, const double* n_vec, const double* q0, double k0,
                     int32_t max_rank, double* work, double* rms_out);
int gdm_krylov_add(gdm_ctx* ctx, int32_t n, int32_t j, const double* dq, int32_t max_rank, double* work,
                   double* rel_out, int32_t* exhausted_out);
int gdm_krylov_apply(gdm_ctx* ctx, int32_t n, int32_t rank, int32_t max_rank, double alpha, int32_t complete,
                     double* n_vec, double* work);

/* ------------------------------------- learned starting charges (MLP) */

/* Per-atom radial descriptors for the charge network, FP64 [n_atoms, 32]:
 * feats[I, 16 s + k] = sum over neighbours J of species s with r < 5 A of
 * exp(-(r - c_k)^2 / (2 * 0.3^2)) (cos(pi r / 5) + 1) / 2,
 * c_k = 0.8 + 3.2 k / 15 (k = 0..15), minimum image.  row_ptr/col: a
 * neighbour CSR containing every pair with r < 5 A (e.g. gdm_build_graph
 * CUTOFF at 5.0, or wider: pairs at r >= 5 A are skipped). */
int gdm_descriptors(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr,
                    const int32_t* col, double* feats);

/* Accumulate per-species feature statistics for standardisation:
 * stats[(s*3 + m)*32 + f] += count (m = 0), sum (m = 1), sum of squares
 * (m = 2) of feats[:, f] over the atoms of species s.  stats FP64 [192],
 * zeroed by the caller before the first call.  gdm_feature_norm turns them
 * into norm FP32 [2][64]: per species the 32 means, then the 32 population
 * standard deviations (floored at 1e-6). */
int gdm_feature_sums(gdm_ctx* ctx, int32_t n, const double* feats, const int32_t* species,
                     double* stats);
int gdm_feature_norm(gdm_ctx* ctx, const double* stats, float* norm);

/* One network per central species (0, 1), each 32 -> 64 -> 64 -> 1 with
 * SiLU; params FP32 [2][6337], per species W1 [64][32], b1 [64], W2
 * [64][64], b2 [64], W3 [64], b3 [1] (row-major, output index first).
 * x = (feats - mean) / std with norm from gdm_feature_norm.
 * gdm_mlp_forward: y[i] = net_{species[i]}(x_i) for i < n; bf16 != 0 rounds
 * weights, inputs and hidden activations to bfloat16 (inference) with FP32
 * accumulation; bf16 = 0 is the FP32 training forward.  y FP32 [n]. */
int gdm_mlp_forward(gdm_ctx* ctx, int32_t n, const int32_t* species, const double* feats,
                    const float* params, const float* norm, int bf16, float* y);

/* Neutral predicted charges q = y - mean(y) (FP64 [n]): the starting
 * charges of the SCC iteration. */
int gdm_mlp_charges(gdm_ctx* ctx, int32_t n, const float* y, double* q);

/* Loss of the neutral prediction q = y - mean(y) against q_ref over the n
 * atoms of one configuration: stats3[0] = mean(y), stats3[1] = mean(r),
 * stats3[2] = mean(r^2) with r = q - q_ref (FP64, device). */
int gdm_mlp_loss(gdm_ctx* ctx, int32_t n, const float* y, const double* q_ref, double* stats3);

/* Gradient of mean(r^2) with respect to both networks' parameters, from the
 * FP32 forward y and gdm_mlp_loss's stats3 (dL/dy_i = 2/n (r_i - mean r)).
 * partial: FP32 workspace [ceil(n/64)][2][6337]; grad FP32 [2][6337]
 * (overwritten; per-block partial sums added in a fixed order, so the
 * result is deterministic). */
int gdm_mlp_backward(gdm_ctx* ctx, int32_t n, const int32_t* species, const double* feats,
                     const float* params, const float* norm, const float* y,
                     const double* q_ref, const double* stats3, float* partial, float* grad);

/* One Adam update of n parameters at step t >= 1 (bias-corrected first and
 * second moments m, v, FP32, zero before the first step). */
int gdm_adam_step(gdm_ctx* ctx, int32_t n, float* params, const float* grad, float* m, float* v,
                  int32_t t, float lr, float b1, float b2, float eps);

/* ------------------------------------------------------------- tracing */

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every kernel launch of the solve path.  gdm_profile(ctx, 1) clears and
 * starts recording, gdm_profile(ctx, 0) stops.  gdm_profile_query
 * synchronises and returns, for the kernel named `kernel` (e.g. "sytrd"),
 * the summed duration in ms and the number of launches since recording
 * started (HOST outputs).  Unknown names give 0 launches.  At most 65536
 * launches are recorded; later ones are not timed. */
int gdm_profile(gdm_ctx* ctx, int enable);
int gdm_profile_query(gdm_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* GDM_H */
