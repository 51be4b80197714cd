// Block-sparse H and S over the neighbour graph, and the gather of every
// subgraph's principal submatrices h, s into dense tiles.
#include "gdm_internal.h"

namespace {

// H/S block of edge (I -> J): direction cosines u = (x_J - x_I)/r from the
// row atom I; sigma-only Slater-Koster pattern g(a, b):
//   s,s = 1 ; s,p_b = u_b ; p_a,s = -u_a ; p_a,p_b = u_a u_b
// The products are formed in the same order as the reference expression
// (sign * u_a) * u_b so that only exp() may differ in the last ulp.
__device__ __forceinline__ void sk_factor(const double u[3], int a, int b, double* g) {
    double ua = a > 0 ? u[a - 1] : 1.0;
    double ub = b > 0 ? u[b - 1] : 1.0;
    double sign = (a > 0 && b == 0) ? -1.0 : 1.0;
    *g = (sign * ua) * ub;
}

__global__ void k_build_hs(int n_atoms, const double* __restrict__ pos, const int32_t* __restrict__ species,
                           double3 L, double3 iL, gdm_tb_params tb, const int32_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ col, int64_t nnz, const double* __restrict__ V_atom,
                           double* __restrict__ H, double* __restrict__ S) {
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_atoms) return;
    const int si = species[i];
    const int ni = tb.n_orb[si];
    const double vi = V_atom ? V_atom[i] : 0.0;
    // on-site block
    {
        double* hb = H + (nnz + i) * 16;
        double* sb = S ? S + (nnz + i) * 16 : nullptr;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double hv = 0.0, sv = 0.0;
                if (a < ni && b < ni && a == b) {
                    hv = tb.onsite[si][a];
                    sv = 1.0;
                    if (V_atom) hv = hv + (0.5 * sv) * (vi + vi);
                }
                hb[a * 4 + b] = hv;
                if (sb) sb[a * 4 + b] = sv;
            }
    }
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        const int j = col[k];
        const int sj = species[j];
        const int nj = tb.n_orb[sj];
        double dx = pos[3 * j + 0] - pos[3 * i + 0];
        double dy = pos[3 * j + 1] - pos[3 * i + 1];
        double dz = pos[3 * j + 2] - pos[3 * i + 2];
        double tx = rint(dx * iL.x), ty = rint(dy * iL.y), tz = rint(dz * iL.z);
        dx = dx - L.x * tx;
        dy = dy - L.y * ty;
        dz = dz - L.z * tz;
        double r2 = (dx * dx + dy * dy) + dz * dz;
        double r = sqrt(r2);
        double u[3] = {dx / r, dy / r, dz / r};
        double V = tb.v0 * exp(-(r - tb.v_r0) / tb.v_decay);
        double Sr = tb.orthogonal ? 0.0 : tb.s0 * exp(-(r - tb.s_r0) / tb.s_decay);
        if (tb.taper_on > 0.0) {
            const double t = gdm_taper(r, tb.taper_on, tb.cutoff, nullptr);
            V = V * t;
            Sr = Sr * t;
        }
        const double vj = V_atom ? V_atom[j] : 0.0;
        double* hb = H + (int64_t)k * 16;
        double* sb = S ? S + (int64_t)k * 16 : nullptr;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double hv = 0.0, sv = 0.0;
                if (a < ni && b < nj) {
                    double g;
                    sk_factor(u, a, b, &g);
                    hv = V * g;
                    sv = Sr * g;
                    if (V_atom) {
                        double sm = tb.orthogonal ? 0.0 : sv;
                        hv = hv + (0.5 * sm) * (vi + vj);
                    }
                }
                hb[a * 4 + b] = hv;
                if (sb) sb[a * 4 + b] = sv;
            }
    }
}

// One workgroup per subgraph: zero the n x n tiles (padding of the leading
// dimension untouched), then every local atom writes its on-site block and
// the blocks of its neighbour edges whose far atom is in the subgraph (local
// index by binary search in the sorted core and halo lists, both staged in
// LDS together with the local orbital offsets).
constexpr int kGatherThreads = 256;
constexpr int kGatherMaxAtoms = 4096;

__global__ void __launch_bounds__(kGatherThreads)
k_gather(const SubDesc* __restrict__ desc, const int32_t* __restrict__ atoms_all,
         const int32_t* __restrict__ orb_ptr, const int32_t* __restrict__ row_ptr,
         const int32_t* __restrict__ col, int64_t nnz, const double* __restrict__ Hb,
         const double* __restrict__ Sb, double* __restrict__ A, double* __restrict__ Sd) {
    __shared__ int32_t s_atoms[kGatherMaxAtoms];
    __shared__ int32_t s_off[kGatherMaxAtoms + 1];
    __shared__ int tmp[8];
    const SubDesc d = desc[blockIdx.x];
    const int t = threadIdx.x;
    const int na = d.natoms;
    const int ld = d.ld;
    double* a = A + d.off2;
    double* s = Sd ? Sd + d.off2 : nullptr;
    for (int e = t; e < d.n * ld; e += kGatherThreads) {
        int r = e / ld, c = e - r * ld;
        if (c < d.n) {
            a[e] = 0.0;
            if (s) s[e] = 0.0;
        }
    }
    // local atoms and orbital offsets (prefix sum over atoms in chunks of 256)
    int run = 0;
    for (int base = 0; base < na; base += kGatherThreads) {
        int i = base + t;
        int g = i < na ? atoms_all[d.atom0 + i] : 0;
        int no = i < na ? orb_ptr[g + 1] - orb_ptr[g] : 0;
        int lane = t & 63, w = t >> 6;
        int incl = no;
        for (int o = 1; o < 64; o <<= 1) {
            int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) tmp[w] = incl;
        __syncthreads();
        int pre = 0, tot = 0;
        for (int q = 0; q < 4; ++q) {
            if (q < w) pre += tmp[q];
            tot += tmp[q];
        }
        if (i < na) {
            s_atoms[i] = g;
            s_off[i] = run + pre + incl - no;
        }
        run += tot;
        __syncthreads();
    }
    if (t == 0) s_off[na] = run;
    __syncthreads();
    const int ncore = d.ncore_atoms;
    // one wave per local atom row; lanes stride over its edges
    const int lane = t & 63, wave = t >> 6;
    for (int i = wave; i < na; i += kGatherThreads / 64) {
        const int g = s_atoms[i];
        const int oi = s_off[i], ni = s_off[i + 1] - oi;
        if (lane < ni * ni) {
            int p = lane / ni, q = lane - p * ni;
            a[(int64_t)(oi + p) * ld + oi + q] = Hb[(nnz + g) * 16 + p * 4 + q];
            if (s) s[(int64_t)(oi + p) * ld + oi + q] = Sb ? Sb[(nnz + g) * 16 + p * 4 + q] : (p == q ? 1.0 : 0.0);
        }
        for (int k = row_ptr[g] + lane; k < row_ptr[g + 1]; k += 64) {
            const int j = col[k];
            int loc = gdm_lower_bound(s_atoms, ncore, j);
            if (loc >= ncore || s_atoms[loc] != j) {
                int h = gdm_lower_bound(s_atoms + ncore, na - ncore, j) + ncore;
                loc = (h < na && s_atoms[h] == j) ? h : -1;
            }
            if (loc < 0) continue;
            const int oj = s_off[loc], nj = s_off[loc + 1] - oj;
            for (int p = 0; p < ni; ++p)
                for (int q = 0; q < nj; ++q) {
                    a[(int64_t)(oi + p) * ld + oj + q] = Hb[(int64_t)k * 16 + p * 4 + q];
                    if (s) s[(int64_t)(oi + p) * ld + oj + q] = Sb ? Sb[(int64_t)k * 16 + p * 4 + q] : 0.0;
                }
        }
    }
}


// Mulliken charges from the collected core rows: for each core atom I of the
// subgraph, pop_I = sum_{a in I} sum_b D_ab S_ba with S read block-wise from
// the neighbour BSR (S_ba = S_ab for the edge I -> J) plus the on-site block;
// q_I = 2 pop_I - n0[species_I].  Each atom is the core atom of exactly one
// subgraph, so every q_I has exactly one writer.
__global__ void __launch_bounds__(kGatherThreads)
k_mulliken(const SubDesc* __restrict__ desc, const int32_t* __restrict__ atoms_all,
           const int32_t* __restrict__ orb_ptr, const int32_t* __restrict__ species,
           const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t nnz,
           const double* __restrict__ Sb, const double* __restrict__ Dc, double n0_0, double n0_1,
           double* __restrict__ q) {
    __shared__ int32_t s_atoms[kGatherMaxAtoms];
    __shared__ int32_t s_off[kGatherMaxAtoms + 1];
    __shared__ int tmp[8];
    const SubDesc d = desc[blockIdx.x];
    const int t = threadIdx.x;
    const int na = d.natoms;
    int run = 0;
    for (int base = 0; base < na; base += kGatherThreads) {
        int i = base + t;
        int g = i < na ? atoms_all[d.atom0 + i] : 0;
        int no = i < na ? orb_ptr[g + 1] - orb_ptr[g] : 0;
        int lane = t & 63, w = t >> 6;
        int incl = no;
        for (int o = 1; o < 64; o <<= 1) {
            int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) tmp[w] = incl;
        __syncthreads();
        int pre = 0, tot = 0;
        for (int qq = 0; qq < 4; ++qq) {
            if (qq < w) pre += tmp[qq];
            tot += tmp[qq];
        }
        if (i < na) {
            s_atoms[i] = g;
            s_off[i] = run + pre + incl - no;
        }
        run += tot;
        __syncthreads();
    }
    if (t == 0) s_off[na] = run;
    __syncthreads();
    const int ncore = d.ncore_atoms;
    const int n = d.n;
    const double* D = Dc + d.offd;
    const int lane = t & 63, wave = t >> 6;
    for (int i = wave; i < ncore; i += kGatherThreads / 64) {
        const int g = s_atoms[i];
        const int oi = s_off[i], ni = s_off[i + 1] - oi;
        double acc = 0.0;
        if (lane < ni * ni) {
            int p = lane / ni, qq = lane - p * ni;
            double sv = Sb ? Sb[(nnz + g) * 16 + p * 4 + qq] : (p == qq ? 1.0 : 0.0);
            acc += D[(int64_t)(oi + p) * n + oi + qq] * sv;
        }
        if (Sb) {
            for (int k = row_ptr[g] + lane; k < row_ptr[g + 1]; k += 64) {
                const int j = col[k];
                int loc = gdm_lower_bound(s_atoms, ncore, j);
                if (loc >= ncore || s_atoms[loc] != j) {
                    int h = gdm_lower_bound(s_atoms + ncore, na - ncore, j) + ncore;
                    loc = (h < na && s_atoms[h] == j) ? h : -1;
                }
                if (loc < 0) continue;
                const int oj = s_off[loc], nj = s_off[loc + 1] - oj;
                for (int p = 0; p < ni; ++p)
                    for (int qq = 0; qq < nj; ++qq)
                        acc += D[(int64_t)(oi + p) * n + oj + qq] * Sb[(int64_t)k * 16 + p * 4 + qq];
            }
        }
        acc = gdm_wave_sum(acc);
        if (lane == 0) q[g] = 2.0 * acc - (species[g] == 0 ? n0_0 : n0_1);
    }
}

}  // namespace

extern "C" int gdm_build_hs(gdm_ctx* ctx, const gdm_system* sys, const gdm_tb_params* tb, const int32_t* row_ptr,
                            const int32_t* col, int64_t nnz, const double* V_atom, double* H, double* S) {
    if (!ctx) return GDM_E_ARG;
    if (!sys || !tb || !row_ptr || (!col && nnz > 0) || !H || (!S && !tb->orthogonal) || !sys->pos ||
        !sys->species || sys->n_atoms <= 0 || nnz < 0)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_build_hs: null argument or bad size");
    if (tb->n_orb[0] < 1 || tb->n_orb[0] > 4 || tb->n_orb[1] < 1 || tb->n_orb[1] > 4)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_build_hs: orbitals per species must be 1..4");
    if (tb->taper_on < 0.0 || (tb->taper_on > 0.0 && !(tb->taper_on < tb->cutoff)))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_build_hs: taper_on must be 0 or in (0, cutoff)");
    double3 L = make_double3(sys->box[0], sys->box[1], sys->box[2]);
    double3 iL = make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]);
    const int n = sys->n_atoms;
    hipLaunchKernelGGL(k_build_hs, dim3((n + 127) / 128), dim3(128), 0, ctx->stream, n, sys->pos, sys->species, L,
                       iL, *tb, row_ptr, col, nnz, V_atom, H, tb->orthogonal ? nullptr : S);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

int gdm_launch_gather(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg, const int32_t* row_ptr,
                      const int32_t* col, int64_t nnz, const double* H, const double* S, double* A, double* Sd,
                      int orthogonal) {
    const Plan& P = ctx->plan;
    if (P.max_natoms > kGatherMaxAtoms)
        return gdm_fail(ctx, GDM_E_ARG, "subgraph with %d atoms exceeds the gather limit %d", P.max_natoms,
                        kGatherMaxAtoms);
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    GDM_TIMED(ctx, "gather");
    hipLaunchKernelGGL(k_gather, dim3(P.n_sub), dim3(kGatherThreads), 0, ctx->stream, desc, sg->atoms, sys->orb_ptr,
                       row_ptr, col, nnz, H, orthogonal ? nullptr : S, A, Sd);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

int gdm_launch_mulliken(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg, const int32_t* row_ptr,
                        const int32_t* col, int64_t nnz, const double* S, const double* D_core, const double n0[2],
                        double* q_out) {
    const Plan& P = ctx->plan;
    if (P.max_natoms > kGatherMaxAtoms)
        return gdm_fail(ctx, GDM_E_ARG, "subgraph with %d atoms exceeds the limit %d", P.max_natoms, kGatherMaxAtoms);
    GDM_TIMED(ctx, "mulliken");
    hipLaunchKernelGGL(k_mulliken, dim3(P.n_sub), dim3(kGatherThreads), 0, ctx->stream,
                       (const SubDesc*)ctx->b[BUF_DESC].p, sg->atoms, sys->orb_ptr, sys->species, row_ptr, col, nnz,
                       S, D_core, n0[0], n0[1], q_out);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}
