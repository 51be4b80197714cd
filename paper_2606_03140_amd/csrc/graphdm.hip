// Graph of the next step from the collected density-matrix core rows
// (Dynamic Graph Adaption section):
//   G^D_IJ = max_{a in I, b in J} |D_ab| over the core rows of I's subgraph,
//   DM mode:        edge iff max(G^D_IJ, G^D_JI) > tau,
//   ADAPTIVE mode:  edge iff max(W_IJ, W_JI) > tau,  W = G^N G^D + G^D G^N,
//                   G^N_IK = exp(-alpha r_IK^2) on neighbour pairs, G^N_II = 1
//                   (Eq. neigh_mat and Eq. Graph_Adaptation),
// optionally united with a given graph.  Candidate edges are counted,
// scattered, then sorted and de-duplicated per row.
#include "gdm_internal.h"

#include <algorithm>

namespace {

constexpr int kThreads = 256;
constexpr int kMaxSubAtoms = 4096;
constexpr int kHashSlots = 4096;
constexpr int kRowSortMax = 8192;

__global__ void k_atom_map(const SubDesc* __restrict__ desc, const int32_t* __restrict__ atoms,
                           int32_t* __restrict__ sub_of, int32_t* __restrict__ loc_of) {
    const SubDesc d = desc[blockIdx.x];
    for (int i = threadIdx.x; i < d.ncore_atoms; i += blockDim.x) {
        int g = atoms[d.atom0 + i];
        sub_of[g] = blockIdx.x;
        loc_of[g] = i;
    }
}

// gd[gbase[s] + i * natoms + j] = max |D| over the (core atom i, atom j) block
__global__ void __launch_bounds__(kThreads) k_gd_rows(const SubDesc* __restrict__ desc, const int64_t* __restrict__ gbase,
                                               const int32_t* __restrict__ atoms, const int32_t* __restrict__ orb_ptr,
                                               const double* __restrict__ Dc, double* __restrict__ gd) {
    __shared__ int32_t s_off[kMaxSubAtoms + 1];
    __shared__ int tmp[8];
    const SubDesc d = desc[blockIdx.x];
    const int na = d.natoms, t = threadIdx.x;
    int run = 0;
    for (int base = 0; base < na; base += kThreads) {
        int i = base + t;
        int g = i < na ? atoms[d.atom0 + i] : 0;
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
        if (i < na) s_off[i] = run + pre + incl - no;
        run += tot;
        __syncthreads();
    }
    if (t == 0) s_off[na] = run;
    __syncthreads();
    const int n = d.n;
    const double* D = Dc + d.offd;
    double* out = gd + gbase[blockIdx.x];
    for (int64_t e = t; e < (int64_t)d.ncore_atoms * na; e += kThreads) {
        int i = (int)(e / na), j = (int)(e - (int64_t)i * na);
        double m = 0.0;
        for (int a = s_off[i]; a < s_off[i + 1]; ++a)
            for (int b = s_off[j]; b < s_off[j + 1]; ++b) m = fmax(m, fabs(D[(int64_t)a * n + b]));
        out[e] = m;
    }
}

// DM mode candidates: (I, J) and (J, I) for every core-row entry above tau
template <bool FILL>
__global__ void __launch_bounds__(kThreads) k_cand_dm(const SubDesc* __restrict__ desc, const int64_t* __restrict__ gbase,
                                               const int32_t* __restrict__ atoms, const double* __restrict__ gd,
                                               double tau, int32_t* __restrict__ cnt, int32_t* __restrict__ cursor,
                                               int32_t* __restrict__ cand) {
    const SubDesc d = desc[blockIdx.x];
    const int na = d.natoms;
    const double* g = gd + gbase[blockIdx.x];
    for (int64_t e = threadIdx.x; e < (int64_t)d.ncore_atoms * na; e += kThreads) {
        int i = (int)(e / na), j = (int)(e - (int64_t)i * na);
        int I = atoms[d.atom0 + i], J = atoms[d.atom0 + j];
        if (I == J || !(g[e] > tau)) continue;
        if (FILL) {
            cand[atomicAdd(&cursor[I], 1)] = J;
            cand[atomicAdd(&cursor[J], 1)] = I;
        } else {
            atomicAdd(&cnt[I], 1);
            atomicAdd(&cnt[J], 1);
        }
    }
}

template <bool FILL>
__global__ void k_cand_union(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ cl,
                             int32_t* __restrict__ cnt, int32_t* __restrict__ cursor, int32_t* __restrict__ cand) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n) return;
    for (int k = rp[I]; k < rp[I + 1]; ++k) {
        int J = cl[k];
        if (J == I) continue;
        if (FILL) cand[atomicAdd(&cursor[I], 1)] = J;
        else atomicAdd(&cnt[I], 1);
    }
}

__device__ __forceinline__ double gn_weight(const double* __restrict__ pos, int i, int j, double3 L, double3 iL,
                                            double alpha) {
#pragma clang fp contract(off)
    double dx = pos[3 * j + 0] - pos[3 * i + 0];
    double dy = pos[3 * j + 1] - pos[3 * i + 1];
    double dz = pos[3 * j + 2] - pos[3 * i + 2];
    double tx = rint(dx * iL.x), ty = rint(dy * iL.y), tz = rint(dz * iL.z);
    dx = dx - L.x * tx;
    dy = dy - L.y * ty;
    dz = dz - L.z * tz;
    double r2 = (dx * dx + dy * dy) + dz * dz;
    return exp(-alpha * r2);
}

// Insert key J in the LDS hash table and return its slot (or -1 when full).
__device__ __forceinline__ int hash_slot(int32_t* keys, int J) {
    unsigned h = ((unsigned)J * 2654435761u) & (kHashSlots - 1);
    for (int probe = 0; probe < kHashSlots; ++probe) {
        int k = keys[h];
        if (k == J) return (int)h;
        if (k == -1) {
            int prev = atomicCAS(&keys[h], -1, J);
            if (prev == -1 || prev == J) return (int)h;
        }
        h = (h + 1) & (kHashSlots - 1);
    }
    return -1;
}

// ADAPTIVE mode: one workgroup per row I accumulates W_I. = sum_K G^N_IK G^D_K.
// + sum_K G^D_IK G^N_K. in an LDS hash keyed by J.  Within one K step each J
// occurs once, so each slot receives its contributions in a fixed K order.
template <bool FILL>
__global__ void __launch_bounds__(kThreads) k_cand_adaptive(
    int n_atoms, const double* __restrict__ pos, double3 L, double3 iL, double alpha, double tau,
    const int32_t* __restrict__ nrp, const int32_t* __restrict__ ncl, const SubDesc* __restrict__ desc,
    const int64_t* __restrict__ gbase, const int32_t* __restrict__ atoms, const int32_t* __restrict__ sub_of,
    const int32_t* __restrict__ loc_of, const double* __restrict__ gd, int32_t* __restrict__ cnt,
    int32_t* __restrict__ cursor, int32_t* __restrict__ cand, int* __restrict__ status) {
    __shared__ int32_t keys[kHashSlots];
    __shared__ double vals[kHashSlots];
    const int I = blockIdx.x;
    for (int h = threadIdx.x; h < kHashSlots; h += kThreads) {
        keys[h] = -1;
        vals[h] = 0.0;
    }
    __syncthreads();
    bool overflow = false;
    // term 1: K in {I} + nbr(I), weight G^N_IK, row K of G^D
    const int deg = nrp[I + 1] - nrp[I];
    for (int q = -1; q < deg; ++q) {
        const int K = q < 0 ? I : ncl[nrp[I] + q];
        const double wn = q < 0 ? 1.0 : gn_weight(pos, I, K, L, iL, alpha);
        const int s = sub_of[K];
        const SubDesc d = desc[s];
        const double* row = gd + gbase[s] + (int64_t)loc_of[K] * d.natoms;
        for (int j = threadIdx.x; j < d.natoms; j += kThreads) {
            double v = row[j];
            if (v == 0.0) continue;
            int slot = hash_slot(keys, atoms[d.atom0 + j]);
            if (slot < 0) {
                overflow = true;
                continue;
            }
            vals[slot] += wn * v;
        }
        __syncthreads();
    }
    // term 2: K in row I of G^D, weight G^D_IK, then J in {K} + nbr(K)
    {
        const int s = sub_of[I];
        const SubDesc d = desc[s];
        const double* row = gd + gbase[s] + (int64_t)loc_of[I] * d.natoms;
        for (int j0 = 0; j0 < d.natoms; ++j0) {
            const double v = row[j0];
            if (v == 0.0) continue;
            const int K = atoms[d.atom0 + j0];
            const int kd = nrp[K + 1] - nrp[K];
            for (int q = (int)threadIdx.x - 1; q < kd; q += kThreads) {
                const int J = q < 0 ? K : ncl[nrp[K] + q];
                const double wn = q < 0 ? 1.0 : gn_weight(pos, K, J, L, iL, alpha);
                int slot = hash_slot(keys, J);
                if (slot < 0) {
                    overflow = true;
                    continue;
                }
                vals[slot] += v * wn;
            }
            __syncthreads();
        }
    }
    if (overflow) gdm_raise(status, GDM_STATUS_CAPACITY);
    for (int h = threadIdx.x; h < kHashSlots; h += kThreads) {
        int J = keys[h];
        if (J < 0 || J == I || !(vals[h] > tau)) continue;
        if (FILL) {
            cand[atomicAdd(&cursor[I], 1)] = J;
            cand[atomicAdd(&cursor[J], 1)] = I;
        } else {
            atomicAdd(&cnt[I], 1);
            atomicAdd(&cnt[J], 1);
        }
    }
}

// Sort + unique each candidate row (one workgroup per row, bitonic sort in LDS).
template <bool WRITE>
__global__ void __launch_bounds__(kThreads) k_row_unique(int n, const int32_t* __restrict__ off,
                                                  const int32_t* __restrict__ cand, int32_t* __restrict__ ucnt,
                                                  const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                                                  int* __restrict__ status) {
    __shared__ int32_t buf[kRowSortMax];
    __shared__ int tmp[8];
    const int I = blockIdx.x;
    const int b = off[I], len = off[I + 1] - b;
    if (len > kRowSortMax) {
        if (threadIdx.x == 0) gdm_raise(status, GDM_STATUS_CAPACITY);
        return;
    }
    int p2 = 1;
    while (p2 < len) p2 <<= 1;
    for (int k = threadIdx.x; k < p2; k += kThreads) buf[k] = k < len ? cand[b + k] : 0x7fffffff;
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int k = threadIdx.x; k < p2; k += kThreads) {
                int partner = k ^ stride;
                if (partner > k) {
                    bool up = (k & size) == 0;
                    int x = buf[k], y = buf[partner];
                    if ((x > y) == up) {
                        buf[k] = y;
                        buf[partner] = x;
                    }
                }
            }
            __syncthreads();
        }
    // unique
    int written = 0;
    const int out0 = WRITE ? row_ptr[I] : 0;
    for (int base = 0; base < len; base += kThreads) {
        int k = base + threadIdx.x;
        int keep = (k < len && (k == 0 || buf[k] != buf[k - 1])) ? 1 : 0;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        int incl = keep;
        for (int o = 1; o < 64; o <<= 1) {
            int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) tmp[wave] = incl;
        __syncthreads();
        int pre = 0, tot = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wave) pre += tmp[w];
            tot += tmp[w];
        }
        if (WRITE && keep) col[out0 + written + pre + incl - keep] = buf[k];
        written += tot;
        __syncthreads();
    }
    if (!WRITE && threadIdx.x == 0) ucnt[I] = written;
}

}  // namespace

int gdm_scan_i32(gdm_ctx* ctx, const int32_t* in, int32_t* out, int64_t n);
int gdm_fill_i32(gdm_ctx* ctx, int32_t* p, int64_t n, int32_t v);

int gdm_dm_graph(gdm_ctx* ctx, const gdm_system* sys, int mode, double alpha, double tau, const gdm_subgraphs* prev,
                 const double* D_core, const int32_t* nbr_row_ptr, const int32_t* nbr_col,
                 const int32_t* union_row_ptr, const int32_t* union_col, int32_t* row_ptr, int32_t* col, int64_t cap,
                 int64_t* nnz_out) {
    Plan& P = ctx->plan;
    if (prev->n_sub != P.n_sub || P.n_sub <= 0)
        return gdm_fail(ctx, GDM_E_STATE, "gdm_build_graph: prev must be the planned subgraph set");
    if (P.max_natoms > kMaxSubAtoms)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_build_graph: subgraph with %d atoms exceeds %d", P.max_natoms,
                        kMaxSubAtoms);
    const int n = sys->n_atoms;
    const int ns = P.n_sub;
    std::vector<int64_t> gb(ns + 1, 0);
    for (int s = 0; s < ns; ++s) gb[s + 1] = gb[s] + (int64_t)P.desc[s].ncore_atoms * P.desc[s].natoms;
    bool ok = true;
    int64_t* gbase = (int64_t*)gdm_buf(ctx, BUF_G_W, sizeof(int64_t) * (ns + 1), &ok);
    double* gd = (double*)gdm_buf(ctx, BUF_G_TMP, sizeof(double) * (size_t)gb[ns], &ok);
    int32_t* sub_of = (int32_t*)gdm_buf(ctx, BUF_G_CELL, sizeof(int32_t) * (size_t)n, &ok);
    int32_t* loc_of = (int32_t*)gdm_buf(ctx, BUF_G_CELLATOMS, sizeof(int32_t) * (size_t)n, &ok);
    int32_t* cnt = (int32_t*)gdm_buf(ctx, BUF_G_CNT, sizeof(int32_t) * (size_t)(n + 1), &ok);
    int32_t* off = (int32_t*)gdm_buf(ctx, BUF_G_CELLSTART, sizeof(int32_t) * (size_t)(n + 1), &ok);
    int32_t* cursor = (int32_t*)gdm_buf(ctx, BUF_G_CELLCNT, sizeof(int32_t) * (size_t)(n + 1), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "workspace allocation failed (graph from D)");
    GDM_HIP(ctx, hipMemcpyAsync(gbase, gb.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, ctx->stream));
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    int rc;
    if ((rc = gdm_fill_i32(ctx, sub_of, n, -1))) return rc;
    hipLaunchKernelGGL(k_atom_map, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, prev->atoms, sub_of, loc_of);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_gd_rows, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, gbase, prev->atoms, sys->orb_ptr, D_core,
                       gd);
    GDM_LAUNCH_CHECK(ctx);
    double3 L = make_double3(sys->box[0], sys->box[1], sys->box[2]);
    double3 iL = make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]);
    auto candidates = [&](bool fill, int32_t* cand) {
        if (mode == GDM_GRAPH_DM) {
            if (fill)
                hipLaunchKernelGGL(k_cand_dm<true>, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, gbase, prev->atoms, gd,
                                   tau, cnt, cursor, cand);
            else
                hipLaunchKernelGGL(k_cand_dm<false>, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, gbase, prev->atoms,
                                   gd, tau, cnt, cursor, cand);
        } else {
            if (fill)
                hipLaunchKernelGGL(k_cand_adaptive<true>, dim3(n), dim3(kThreads), 0, ctx->stream, n, sys->pos, L, iL,
                                   alpha, tau, nbr_row_ptr, nbr_col, desc, gbase, prev->atoms, sub_of, loc_of, gd,
                                   cnt, cursor, cand, ctx->d_status);
            else
                hipLaunchKernelGGL(k_cand_adaptive<false>, dim3(n), dim3(kThreads), 0, ctx->stream, n, sys->pos, L, iL,
                                   alpha, tau, nbr_row_ptr, nbr_col, desc, gbase, prev->atoms, sub_of, loc_of, gd,
                                   cnt, cursor, cand, ctx->d_status);
        }
        if (union_row_ptr) {
            if (fill)
                hipLaunchKernelGGL(k_cand_union<true>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n,
                                   union_row_ptr, union_col, cnt, cursor, cand);
            else
                hipLaunchKernelGGL(k_cand_union<false>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n,
                                   union_row_ptr, union_col, cnt, cursor, cand);
        }
    };
    if ((rc = gdm_fill_i32(ctx, cnt, n + 1, 0))) return rc;
    candidates(false, nullptr);
    GDM_LAUNCH_CHECK(ctx);
    if ((rc = gdm_scan_i32(ctx, cnt, off, n))) return rc;
    int32_t ncand = 0;
    GDM_HIP(ctx, hipMemcpyAsync(&ncand, off + n, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    int32_t* cand = (int32_t*)gdm_buf(ctx, BUF_G_FLAGS, sizeof(int32_t) * (size_t)(ncand + 1), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "workspace allocation failed (graph candidates)");
    GDM_HIP(ctx, hipMemcpyAsync(cursor, off, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
    candidates(true, cand);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_row_unique<false>, dim3(n), dim3(kThreads), 0, ctx->stream, n, off, cand, cnt, nullptr, nullptr,
                       ctx->d_status);
    GDM_LAUNCH_CHECK(ctx);
    if ((rc = gdm_scan_i32(ctx, cnt, row_ptr, n))) return rc;
    int32_t total = 0;
    GDM_HIP(ctx, hipMemcpyAsync(&total, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *nnz_out = total;
    if (total > cap)
        return gdm_fail(ctx, GDM_E_CAPACITY, "graph needs %lld edges, capacity %lld", (long long)total,
                        (long long)cap);
    hipLaunchKernelGGL(k_row_unique<true>, dim3(n), dim3(kThreads), 0, ctx->stream, n, off, cand, cnt, row_ptr, col,
                       ctx->d_status);
    GDM_LAUNCH_CHECK(ctx);
    return gdm_check(ctx);
}
