// Forces of the shadow Born-Oppenheimer potential at fixed extended charges
// n (Shadow MD section, nuclear equation of motion NEQ), from the collected
// core rows of the density matrix D and of the energy-weighted density
// W = C diag(f lam) C^T:
//
//   U(R, n) = Omega(H[n]) - sum_I (N0_I + n_I/2) V_I + E_rep,
//   -dOmega/dR = -2 Tr[D dH[n]/dR] + 2 Tr[W dS/dR]   (V held fixed),
//
// H[n] = H0 + S (V_I + V_J)/2.  Only off-diagonal atom blocks depend on the
// positions.  For a neighbour pair (I, J) with d = R_J - R_I the pair term is
//   e_IJ(d) = 4 sum_{a in I, b in J} [Dbar_ab (H0_ab + S_ab (V_I + V_J)/2) - Wbar_ab S_ab]
//             + A_pair exp(-r/rho) t(r)          (repulsion, per unordered pair)
// with Dbar = (D_IJ + D_JI^T)/2 assembled from the core rows of I's and of
// J's subgraph (zero where the other atom is outside the subgraph), and
// F_I = sum_J grad_d e_IJ.  The Coulomb part of the force (the position
// dependence of gamma) is gdm_ewald_forces.
//
// One thread per directed neighbour pair computes its contribution into a
// per-pair buffer (no atomics); one thread per atom then adds its row in
// neighbour order, so the result does not depend on scheduling.  Each pair's
// contribution is the exact negative of its mirror's up to rounding, so the
// forces sum to zero to rounding.
#include "gdm_internal.h"

#include <algorithm>

namespace {

constexpr int kThreads = 256;

// Local orbital offset of every atom of every subgraph (prefix sum of the
// orbital counts over the subgraph's atom list), and for each core atom its
// subgraph and position in that list; cnt counts how often an atom is core.
__global__ void __launch_bounds__(kThreads) k_force_map(const SubDesc* __restrict__ desc,
                                                       const int32_t* __restrict__ atoms,
                                                       const int32_t* __restrict__ orb_ptr, int32_t* __restrict__ loff,
                                                       int32_t* __restrict__ sub_of, int32_t* __restrict__ loc_of,
                                                       int32_t* __restrict__ cnt) {
    __shared__ int tmp[kThreads / 64];
    const SubDesc d = desc[blockIdx.x];
    const int na = d.natoms, t = threadIdx.x, lane = t & 63, w = t >> 6;
    int run = 0;
    for (int base = 0; base < na; base += kThreads) {
        const int i = base + t;
        const int g = i < na ? atoms[d.atom0 + i] : 0;
        const int no = i < na ? orb_ptr[g + 1] - orb_ptr[g] : 0;
        int incl = no;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) tmp[w] = incl;
        __syncthreads();
        int pre = 0, tot = 0;
        for (int q = 0; q < kThreads / 64; ++q) {
            if (q < w) pre += tmp[q];
            tot += tmp[q];
        }
        if (i < na) {
            loff[d.atom0 + i] = run + pre + incl - no;
            if (i < d.ncore_atoms) {
                sub_of[g] = blockIdx.x;
                loc_of[g] = i;
                atomicAdd(&cnt[g], 1);
            }
        }
        run += tot;
        __syncthreads();
    }
}

// index of g in the sorted a[lo, hi), or -1
__device__ __forceinline__ int find_sorted(const int32_t* __restrict__ a, int lo, int hi, int g) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int v = a[mid];
        if (v == g) return mid;
        if (v < g) lo = mid + 1;
        else hi = mid;
    }
    return -1;
}

// local position of atom g in subgraph d (core part, then halo part), or -1
__device__ __forceinline__ int find_local(const SubDesc& d, const int32_t* __restrict__ atoms, int g) {
    int k = find_sorted(atoms, d.atom0, d.atom0 + d.ncore_atoms, g);
    if (k < 0) k = find_sorted(atoms, d.atom0 + d.ncore_atoms, d.atom0 + d.natoms, g);
    return k < 0 ? -1 : k - d.atom0;
}

// value and r-derivative of amp exp(-(r - r0)/decay) t(r)
__device__ __forceinline__ void radial(double r, double amp, double r0, double decay, const gdm_tb_params& tb,
                                       double* v, double* dv) {
    const double e = amp * exp(-(r - r0) / decay);
    double de = -e / decay;
    if (tb.taper_on > 0.0) {
        double dt;
        const double t = gdm_taper(r, tb.taper_on, tb.cutoff, &dt);
        *v = e * t;
        *dv = de * t + e * dt;
        return;
    }
    *v = e;
    *dv = de;
}

__global__ void __launch_bounds__(kThreads) k_pair_forces(
    int n_atoms, int64_t nnz, const double* __restrict__ pos, const int32_t* __restrict__ species,
    const int32_t* __restrict__ orb_ptr, double3 L, double3 iL, gdm_tb_params tb, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ cl, const SubDesc* __restrict__ desc, const int32_t* __restrict__ atoms,
    const int32_t* __restrict__ loff, const int32_t* __restrict__ sub_of, const int32_t* __restrict__ loc_of,
    const int32_t* __restrict__ cnt, const double* __restrict__ Dc, const double* __restrict__ Wc,
    const double* __restrict__ V_atom, double* __restrict__ fpair, double* __restrict__ epair,
    int* __restrict__ status) {
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= nnz) return;
    // row of entry k: the last I with rp[I] <= k
    int lo = 0, hi = n_atoms;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rp[mid] <= k) lo = mid;
        else hi = mid;
    }
    const int I = lo, J = cl[k];
    if (cnt[I] != 1 || cnt[J] != 1) {
        gdm_raise(status, GDM_STATUS_PARTITION);
        fpair[3 * k] = fpair[3 * k + 1] = fpair[3 * k + 2] = 0.0;
        epair[k] = 0.0;
        return;
    }
    const int si = species[I], sj = species[J];
    const int ni = min(4, orb_ptr[I + 1] - orb_ptr[I]), nj = min(4, orb_ptr[J + 1] - orb_ptr[J]);
    double dx = pos[3 * J] - pos[3 * I], dy = pos[3 * J + 1] - pos[3 * I + 1], dz = pos[3 * J + 2] - pos[3 * I + 2];
    dx = dx - L.x * rint(dx * iL.x);
    dy = dy - L.y * rint(dy * iL.y);
    dz = dz - L.z * rint(dz * iL.z);
    const double r = sqrt((dx * dx + dy * dy) + dz * dz);
    const double u[3] = {dx / r, dy / r, dz / r};
    // symmetrised blocks Dbar, Wbar (rows: orbitals of I, columns: of J)
    // (loops over the 4 x 4 block fully unrolled so that the blocks stay
    // in registers; entries beyond the atoms' orbital counts stay zero)
    double Db[4][4], Wb[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) Db[a][b] = Wb[a][b] = 0.0;
    {
        const SubDesc d = desc[sub_of[I]];
        const int kj = find_local(d, atoms, J);
        if (kj >= 0) {
            const int64_t row0 = loff[d.atom0 + loc_of[I]], c0 = loff[d.atom0 + kj];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (a < ni && b < nj) {
                        const int64_t e = d.offd + (row0 + a) * d.n + c0 + b;
                        Db[a][b] += 0.5 * Dc[e];
                        Wb[a][b] += 0.5 * Wc[e];
                    }
        }
    }
    {
        const SubDesc d = desc[sub_of[J]];
        const int ki = find_local(d, atoms, I);
        if (ki >= 0) {
            const int64_t row0 = loff[d.atom0 + loc_of[J]], c0 = loff[d.atom0 + ki];
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    if (a < ni && b < nj) {
                        const int64_t e = d.offd + (row0 + b) * d.n + c0 + a;
                        Db[a][b] += 0.5 * Dc[e];
                        Wb[a][b] += 0.5 * Wc[e];
                    }
        }
    }
    double V, dV, Sr = 0.0, dS = 0.0;
    radial(r, tb.v0, tb.v_r0, tb.v_decay, tb, &V, &dV);
    if (!tb.orthogonal) radial(r, tb.s0, tb.s_r0, tb.s_decay, tb, &Sr, &dS);
    const double vs = V_atom ? 0.5 * (V_atom[I] + V_atom[J]) : 0.0;
    // A = sum XH g, B = sum XS g and their gradients in u (Slater-Koster
    // factor g: s,s 1; s,p_b u_b; p_a,s -u_a; p_a,p_b u_a u_b)
    double A = 0.0, B = 0.0, gA[3] = {0.0, 0.0, 0.0}, gB[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (a >= ni || b >= nj) continue;
            const double xh = 4.0 * Db[a][b];
            const double xs = 4.0 * (Db[a][b] * vs - Wb[a][b]);
            double g;
            if (a == 0 && b == 0) {
                g = 1.0;
            } else if (a == 0) {
                g = u[b - 1];
                gA[b - 1] += xh;
                gB[b - 1] += xs;
            } else if (b == 0) {
                g = -u[a - 1];
                gA[a - 1] -= xh;
                gB[a - 1] -= xs;
            } else {
                g = u[a - 1] * u[b - 1];
                gA[a - 1] += xh * u[b - 1];
                gA[b - 1] += xh * u[a - 1];
                gB[a - 1] += xs * u[b - 1];
                gB[b - 1] += xs * u[a - 1];
            }
            A += xh * g;
            B += xs * g;
        }
    // grad_d e = (V' A + S' B) u + (V P gA + S P gB)/r, P = I - u u^T
    const double uA = u[0] * gA[0] + u[1] * gA[1] + u[2] * gA[2];
    const double uB = u[0] * gB[0] + u[1] * gB[1] + u[2] * gB[2];
    double radial_part = dV * A + dS * B;
    // repulsion A_pair exp(-r/rho) t(r), half of the pair energy per direction
    double erep = 0.0;
    const double Ap = tb.rep_A[si + sj];
    if (Ap != 0.0) {
        double e = Ap * exp(-r / tb.rep_rho), de = -e / tb.rep_rho;
        if (tb.taper_on > 0.0) {
            double dt;
            const double t = gdm_taper(r, tb.taper_on, tb.cutoff, &dt);
            de = de * t + e * dt;
            e = e * t;
        }
        radial_part += de;
        erep = 0.5 * e;
    }
    for (int c = 0; c < 3; ++c)
        fpair[3 * k + c] = radial_part * u[c] + (V * (gA[c] - u[c] * uA) + Sr * (gB[c] - u[c] * uB)) / r;
    epair[k] = erep;
}

// F_I = sum over row I of the pair contributions; per-atom energies
// (repulsion, -(N0_I + n_I/2) V_I) summed per workgroup
__global__ void __launch_bounds__(kThreads) k_force_reduce(int n_atoms, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ species,
                                                          const double* __restrict__ fpair,
                                                          const double* __restrict__ epair,
                                                          const double* __restrict__ V_atom,
                                                          const double* __restrict__ n_vec, double n0_0, double n0_1,
                                                          double* __restrict__ F, double* __restrict__ part) {
    __shared__ double r0[kThreads], r1[kThreads];
    const int I = blockIdx.x * kThreads + threadIdx.x;
    double e_rep = 0.0, e_sh = 0.0;
    if (I < n_atoms) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int k = rp[I]; k < rp[I + 1]; ++k) {
            fx += fpair[3 * (int64_t)k];
            fy += fpair[3 * (int64_t)k + 1];
            fz += fpair[3 * (int64_t)k + 2];
            e_rep += epair[k];
        }
        F[3 * I] = fx;
        F[3 * I + 1] = fy;
        F[3 * I + 2] = fz;
        if (V_atom && n_vec) e_sh = -((species[I] == 0 ? n0_0 : n0_1) + 0.5 * n_vec[I]) * V_atom[I];
    }
    r0[threadIdx.x] = e_rep;
    r1[threadIdx.x] = e_sh;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r0[0];
        part[2 * blockIdx.x + 1] = r1[0];
    }
}

__global__ void __launch_bounds__(kThreads) k_energy_sum(int nb, const double* __restrict__ part,
                                                        double* __restrict__ out) {
    __shared__ double r0[kThreads], r1[kThreads];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = r0[0];
        out[1] = r1[0];
    }
}

}  // namespace

extern "C" int gdm_forces(gdm_ctx* ctx, const gdm_system* sys, const gdm_tb_params* tb, const int32_t* row_ptr,
                          const int32_t* col, int64_t nnz, const gdm_subgraphs* sg, const double* D_core,
                          const double* W_core, const double* V_atom, const double n0[2], const double* n_vec,
                          double* F, double* energy) {
    if (!ctx) return GDM_E_ARG;
    if (!sys || !sys->pos || !sys->species || !sys->orb_ptr || sys->n_atoms <= 0 || !tb || !row_ptr ||
        (!col && nnz > 0) || nnz < 0 || !sg || !D_core || !W_core || !F)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_forces: null argument or empty system");
    if (sg->n_sub != ctx->plan.n_sub || ctx->plan.n_sub <= 0)
        return gdm_fail(ctx, GDM_E_STATE, "gdm_forces: subgraph set does not match the plan (call gdm_plan)");
    if ((V_atom || n_vec) && energy && !n0)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_forces: the Coulomb energy term needs n0");
    if (tb->taper_on < 0.0 || (tb->taper_on > 0.0 && !(tb->taper_on < tb->cutoff)))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_forces: taper_on must be 0 or in (0, cutoff)");
    if ((tb->rep_A[0] != 0.0 || tb->rep_A[1] != 0.0 || tb->rep_A[2] != 0.0) && !(tb->rep_rho > 0.0))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_forces: rep_rho must be positive when rep_A is used");
    const int n = sys->n_atoms, ns = ctx->plan.n_sub;
    const int nb = (n + kThreads - 1) / kThreads;
    int64_t tot_atoms = 0;
    for (const SubDesc& d : ctx->plan.desc) tot_atoms = std::max<int64_t>(tot_atoms, (int64_t)d.atom0 + d.natoms);
    bool ok = true;
    double* fp = (double*)gdm_buf(ctx, BUF_FPAIR, sizeof(double) * 4 * (size_t)std::max<int64_t>(nnz, 1), &ok);
    const size_t map_bytes = sizeof(int32_t) * ((size_t)tot_atoms + 3 * (size_t)n) + sizeof(double) * (2 * nb + 2);
    char* mp = (char*)gdm_buf(ctx, BUF_FMAP, map_bytes + 64, &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_forces: workspace allocation failed");
    double* part = (double*)mp;
    double* esum = part + 2 * nb;
    int32_t* loff = (int32_t*)(esum + 2);
    int32_t* sub_of = loff + tot_atoms;
    int32_t* loc_of = sub_of + n;
    int32_t* cnt = loc_of + n;
    double* epair = fp + 3 * std::max<int64_t>(nnz, 1);
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const double3 L = make_double3(sys->box[0], sys->box[1], sys->box[2]);
    const double3 iL = make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]);
    int rc;
    GDM_TIMED(ctx, "forces");
    if ((rc = gdm_fill_i32(ctx, cnt, n, 0))) return rc;
    hipLaunchKernelGGL(k_force_map, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, sg->atoms, sys->orb_ptr, loff,
                       sub_of, loc_of, cnt);
    GDM_LAUNCH_CHECK(ctx);
    if (nnz > 0) {
        hipLaunchKernelGGL(k_pair_forces, dim3((unsigned)((nnz + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                           ctx->stream, n, nnz, sys->pos, sys->species, sys->orb_ptr, L, iL, *tb, row_ptr, col, desc,
                           sg->atoms, loff, sub_of, loc_of, cnt, D_core, W_core, V_atom, fp, epair, ctx->d_status);
        GDM_LAUNCH_CHECK(ctx);
    }
    hipLaunchKernelGGL(k_force_reduce, dim3(nb), dim3(kThreads), 0, ctx->stream, n, row_ptr, sys->species, fp, epair,
                       V_atom, n_vec, n0 ? n0[0] : 0.0, n0 ? n0[1] : 0.0, F, part);
    GDM_LAUNCH_CHECK(ctx);
    if (energy) {
        hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(kThreads), 0, ctx->stream, nb, part, energy);
        GDM_LAUNCH_CHECK(ctx);
    }
    return GDM_OK;
}
