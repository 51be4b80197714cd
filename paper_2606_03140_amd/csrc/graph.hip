// Neighbour graph (cell list), spatial-grid cores and core+halo subgraphs.
//
// The neighbour test must reproduce the reference minimum-image arithmetic
// bit for bit (integer outputs are compared exactly), so the distance code
// below is compiled without floating-point contraction.
#include "gdm_internal.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int kScanThreads = 1024;

template <typename T>
__global__ void k_scan_single(const T* in, T* out, int64_t n) {
    __shared__ T sums[kScanThreads];
    const int t = threadIdx.x;
    const int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
    const int64_t b = (int64_t)t * chunk;
    const int64_t e = b + chunk < n ? b + chunk : n;
    T s = 0;
    for (int64_t i = b; i < e; ++i) s += in[i];
    sums[t] = s;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        T v = t >= o ? sums[t - o] : T(0);
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    T run = t ? sums[t - 1] : T(0);
    for (int64_t i = b; i < e; ++i) {
        T v = in[i];
        out[i] = run;
        run += v;
    }
    if (t == kScanThreads - 1) out[n] = sums[kScanThreads - 1];
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Minimum-image squared distance, evaluated exactly as
//   d = x_j - x_i ; d = d - L * rint(d * inv_L) ; r2 = (dx*dx + dy*dy) + dz*dz
__device__ __forceinline__ double min_image_r2(const double* __restrict__ pos, int i, int j,
                                               double3 L, double3 iL, double3* dout) {
#pragma clang fp contract(off)
    double dx = pos[3 * j + 0] - pos[3 * i + 0];
    double dy = pos[3 * j + 1] - pos[3 * i + 1];
    double dz = pos[3 * j + 2] - pos[3 * i + 2];
    double tx = rint(dx * iL.x), ty = rint(dy * iL.y), tz = rint(dz * iL.z);
    double px = L.x * tx, py = L.y * ty, pz = L.z * tz;
    dx = dx - px;
    dy = dy - py;
    dz = dz - pz;
    double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    double s = xx + yy;
    if (dout) *dout = make_double3(dx, dy, dz);
    return s + zz;
}

struct Grid3 {
    int g[3];
    double gi[3];   // g / L: maps a wrapped coordinate to a cell index
};

__device__ __forceinline__ int cell_coord(double x, double gi, int g) {
    int c = (int)floor(x * gi);
    return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

__global__ void k_cell_assign(const double* __restrict__ pos, int n, Grid3 G, int32_t* __restrict__ cell,
                              int32_t* __restrict__ cellcnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(pos[3 * i], G.gi[0], G.g[0]);
    int cy = cell_coord(pos[3 * i + 1], G.gi[1], G.g[1]);
    int cz = cell_coord(pos[3 * i + 2], G.gi[2], G.g[2]);
    int c = (cx * G.g[1] + cy) * G.g[2] + cz;
    cell[i] = c;
    atomicAdd(&cellcnt[c], 1);
}

__global__ void k_cell_scatter(int n, const int32_t* __restrict__ cell, int32_t* __restrict__ cursor,
                               int32_t* __restrict__ cellatoms) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int slot = atomicAdd(&cursor[cell[i]], 1);
    cellatoms[slot] = i;
}

constexpr int kShortRow = 64;
constexpr int kSortMax = 8192;

template <bool FILL>
__global__ void k_cell_pairs(const double* __restrict__ pos, int n, Grid3 G, double3 L, double3 iL,
                             double c2, const int32_t* __restrict__ cell,
                             const int32_t* __restrict__ cellstart, const int32_t* __restrict__ cellatoms,
                             int32_t* __restrict__ cnt, const int32_t* __restrict__ row_ptr,
                             int32_t* __restrict__ col) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell[i];
    int cz = c % G.g[2], cy = (c / G.g[2]) % G.g[1], cx = c / (G.g[1] * G.g[2]);
    int count = 0;
    int out = FILL ? row_ptr[i] : 0;
    int rx = G.g[0] >= 3 ? 1 : 0, ry = G.g[1] >= 3 ? 1 : 0, rz = G.g[2] >= 3 ? 1 : 0;
    for (int ox = -rx; ox <= rx; ++ox)
        for (int oy = -ry; oy <= ry; ++oy)
            for (int oz = -rz; oz <= rz; ++oz) {
                int nx = (cx + ox + G.g[0]) % G.g[0];
                int ny = (cy + oy + G.g[1]) % G.g[1];
                int nz = (cz + oz + G.g[2]) % G.g[2];
                int nc = (nx * G.g[1] + ny) * G.g[2] + nz;
                for (int k = cellstart[nc]; k < cellstart[nc + 1]; ++k) {
                    int j = cellatoms[k];
                    if (j == i) continue;
                    double r2 = min_image_r2(pos, i, j, L, iL, nullptr);
                    if (r2 < c2) {
                        if (FILL) col[out + count] = j;
                        ++count;
                    }
                }
            }
    if (!FILL) {
        cnt[i] = count;
    } else if (count <= kShortRow || count > kSortMax) {
        // ascending columns: insertion sort of a short row (rows of
        // kShortRow..kSortMax entries are sorted by k_sort_long_rows)
        int b = row_ptr[i];
        for (int a = 1; a < count; ++a) {
            int v = col[b + a];
            int p = a - 1;
            while (p >= 0 && col[b + p] > v) {
                col[b + p + 1] = col[b + p];
                --p;
            }
            col[b + p + 1] = v;
        }
    }
}

// Bitonic sort in LDS of every row with kShortRow < length <= kSortMax (one
// workgroup per row; shorter and longer rows were sorted by k_cell_pairs).
__global__ void __launch_bounds__(256) k_sort_long_rows(const int32_t* __restrict__ row_ptr,
                                                       int32_t* __restrict__ col) {
    __shared__ int32_t s[kSortMax];
    const int i = blockIdx.x;
    const int b = row_ptr[i], cnt = row_ptr[i + 1] - b;
    if (cnt <= kShortRow || cnt > kSortMax) return;
    int P = 1;
    while (P < cnt) P <<= 1;
    for (int e = threadIdx.x; e < P; e += 256) s[e] = e < cnt ? col[b + e] : INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int e = threadIdx.x; e < P; e += 256) {
                const int x = e ^ j;
                if (x > e) {
                    const int a = s[e], c = s[x];
                    if ((a > c) == ((e & k) == 0)) {
                        s[e] = c;
                        s[x] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int e = threadIdx.x; e < cnt; e += 256) col[b + e] = s[e];
}

// ---------------------------------------------------------------- cores

__global__ void k_core_cells(const double* __restrict__ pos, const int32_t* __restrict__ anchor, int n,
                             int gx, int gy, int gz, double3 iL, int32_t* __restrict__ cid,
                             int32_t* __restrict__ flags) {
#pragma clang fp contract(off)
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = anchor[i];
    double px = pos[3 * a], py = pos[3 * a + 1], pz = pos[3 * a + 2];
    double fx = floor((px * iL.x) * (double)gx);
    double fy = floor((py * iL.y) * (double)gy);
    double fz = floor((pz * iL.z) * (double)gz);
    int cx = (int)fx, cy = (int)fy, cz = (int)fz;
    cx = cx > gx - 1 ? gx - 1 : cx;
    cy = cy > gy - 1 ? gy - 1 : cy;
    cz = cz > gz - 1 ? gz - 1 : cz;
    int c = (cx * gy + cy) * gz + cz;
    cid[i] = c;
    flags[c] = 1;
}

__global__ void k_core_remap(int n, const int32_t* __restrict__ cid, const int32_t* __restrict__ remap,
                             int32_t* __restrict__ core_of_atom) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    core_of_atom[i] = remap[cid[i]];
}

// ------------------------------------------------------------ subgraphs

constexpr int kExtractThreads = 256;

// exclusive prefix over the 256 threads of a block; returns the block total in *total
__device__ __forceinline__ int block_excl_scan256(int v, int* tmp, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wave) base += tmp[w];
        tot += tmp[w];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

template <bool FILL>
__global__ void __launch_bounds__(kExtractThreads)
k_extract(int n_atoms, const int32_t* __restrict__ species, const int32_t* __restrict__ row_ptr,
          const int32_t* __restrict__ col, const int32_t* __restrict__ core_of_atom, int n_orb0, int n_orb1,
          int32_t* __restrict__ counts /* [4*n_cores]: natoms, ncore, norb, ncore_orb */,
          const int32_t* __restrict__ atom_ptr, int32_t* __restrict__ atoms_out) {
    extern __shared__ uint32_t bm[];
    __shared__ int tmp[8];
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    const int words = (n_atoms + 31) >> 5;
    for (int w = t; w < words; w += kExtractThreads) bm[w] = 0u;
    __syncthreads();
    int my_core = 0, my_core_orb = 0;
    int out_base = FILL ? atom_ptr[c] : 0;
    int written = 0;
    for (int base = 0; base < n_atoms; base += kExtractThreads) {
        int i = base + t;
        int is_core = (i < n_atoms && core_of_atom[i] == c) ? 1 : 0;
        if (is_core) {
            ++my_core;
            my_core_orb += species[i] == 0 ? n_orb0 : n_orb1;
            for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                int j = col[k];
                atomicOr(&bm[j >> 5], 1u << (j & 31));
            }
        }
        if (FILL) {
            int tot;
            int pos = block_excl_scan256(is_core, tmp, &tot);
            if (is_core) atoms_out[out_base + written + pos] = i;
            written += tot;
        }
    }
    __syncthreads();
    // drop the core atoms from the halo bitmap
    for (int base = 0; base < n_atoms; base += kExtractThreads) {
        int i = base + t;
        if (i < n_atoms && core_of_atom[i] == c) atomicAnd(&bm[i >> 5], ~(1u << (i & 31)));
    }
    __syncthreads();
    // halo: contiguous word ranges per thread keep ascending order
    const int per = (words + kExtractThreads - 1) / kExtractThreads;
    const int w0 = t * per, w1 = min(words, w0 + per);
    int my_halo = 0, my_halo_orb = 0;
    for (int w = w0; w < w1; ++w) {
        uint32_t m = bm[w];
        my_halo += __popc(m);
        while (m) {
            int b = __ffs(m) - 1;
            m &= m - 1;
            int j = (w << 5) + b;
            my_halo_orb += species[j] == 0 ? n_orb0 : n_orb1;
        }
    }
    if (FILL) {
        int tot;
        int pos = block_excl_scan256(my_halo, tmp, &tot);
        int o = out_base + written + pos;
        for (int w = w0; w < w1; ++w) {
            uint32_t m = bm[w];
            while (m) {
                int b = __ffs(m) - 1;
                m &= m - 1;
                atoms_out[o++] = (w << 5) + b;
            }
        }
    } else {
        int tot_core, tot_core_orb, tot_halo, tot_halo_orb;
        block_excl_scan256(my_core, tmp, &tot_core);
        block_excl_scan256(my_core_orb, tmp, &tot_core_orb);
        block_excl_scan256(my_halo, tmp, &tot_halo);
        block_excl_scan256(my_halo_orb, tmp, &tot_halo_orb);
        if (t == 0) {
            counts[4 * c + 0] = tot_core + tot_halo;
            counts[4 * c + 1] = tot_core;
            counts[4 * c + 2] = tot_core_orb + tot_halo_orb;
            counts[4 * c + 3] = tot_core_orb;
        }
    }
}

__global__ void k_extract_split(int n_cores, const int32_t* __restrict__ counts, int32_t* __restrict__ natoms,
                                int32_t* __restrict__ n_core) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cores) return;
    natoms[c] = counts[4 * c];
    n_core[c] = counts[4 * c + 1];
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

// ----------------------------------------------------------------- host

int gdm_scan_i32(gdm_ctx* ctx, const int32_t* in, int32_t* out, int64_t n) {
    hipLaunchKernelGGL(k_scan_single<int32_t>, dim3(1), dim3(kScanThreads), 0, ctx->stream, in, out, n);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

int gdm_scan_i64(gdm_ctx* ctx, const int64_t* in, int64_t* out, int64_t n) {
    hipLaunchKernelGGL(k_scan_single<int64_t>, dim3(1), dim3(kScanThreads), 0, ctx->stream, in, out, n);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

template <typename T>
static int fill(gdm_ctx* ctx, T* p, int64_t n, T v) {
    if (n <= 0) return GDM_OK;
    int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, ctx->stream, p, n, v);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

int gdm_fill_i32(gdm_ctx* ctx, int32_t* p, int64_t n, int32_t v) { return fill(ctx, p, n, v); }
int gdm_fill_f64(gdm_ctx* ctx, double* p, int64_t n, double v) { return fill(ctx, p, n, v); }

int gdm_cutoff_graph(gdm_ctx* ctx, const gdm_system* sys, double cutoff, int32_t* row_ptr, int32_t* col,
                     int64_t cap, int64_t* nnz_out) {
    const int n = sys->n_atoms;
    Grid3 G;
    for (int a = 0; a < 3; ++a) {
        int g = (int)std::floor(sys->box[a] / (cutoff * (1.0 + 1e-9)));
        if (g < 3) g = 1;
        G.g[a] = g;
        G.gi[a] = (double)g * sys->inv_box[a];
    }
    const int64_t ncell = (int64_t)G.g[0] * G.g[1] * G.g[2];
    bool ok = true;
    int32_t* cell = (int32_t*)gdm_buf(ctx, BUF_G_CELL, sizeof(int32_t) * (size_t)n, &ok);
    int32_t* cellcnt = (int32_t*)gdm_buf(ctx, BUF_G_CELLCNT, sizeof(int32_t) * (size_t)(ncell + 1), &ok);
    int32_t* cellstart = (int32_t*)gdm_buf(ctx, BUF_G_CELLSTART, sizeof(int32_t) * (size_t)(ncell + 1), &ok);
    int32_t* cellatoms = (int32_t*)gdm_buf(ctx, BUF_G_CELLATOMS, sizeof(int32_t) * (size_t)n, &ok);
    int32_t* cnt = (int32_t*)gdm_buf(ctx, BUF_G_CNT, sizeof(int32_t) * (size_t)(n + 1), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "workspace allocation failed (cell list)");
    int rc;
    if ((rc = fill<int32_t>(ctx, cellcnt, ncell + 1, 0))) return rc;
    hipLaunchKernelGGL(k_cell_assign, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, sys->pos, n, G, cell,
                       cellcnt);
    GDM_LAUNCH_CHECK(ctx);
    if ((rc = gdm_scan_i32(ctx, cellcnt, cellstart, ncell))) return rc;
    // cursor copy: cellcnt <- cellstart
    GDM_HIP(ctx, hipMemcpyAsync(cellcnt, cellstart, sizeof(int32_t) * (size_t)ncell, hipMemcpyDeviceToDevice,
                                ctx->stream));
    hipLaunchKernelGGL(k_cell_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, n, cell, cellcnt,
                       cellatoms);
    GDM_LAUNCH_CHECK(ctx);
    double3 L = make_double3(sys->box[0], sys->box[1], sys->box[2]);
    double3 iL = make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]);
    const double c2 = cutoff * cutoff;
    hipLaunchKernelGGL(k_cell_pairs<false>, dim3(blocks_for(n, 128)), dim3(128), 0, ctx->stream, sys->pos, n, G, L,
                       iL, c2, cell, cellstart, cellatoms, cnt, nullptr, nullptr);
    GDM_LAUNCH_CHECK(ctx);
    if ((rc = gdm_scan_i32(ctx, cnt, row_ptr, n))) return rc;
    int32_t total = 0;
    GDM_HIP(ctx, hipMemcpyAsync(&total, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *nnz_out = total;
    if (total > cap) return gdm_fail(ctx, GDM_E_CAPACITY, "neighbour graph needs %lld edges, capacity %lld",
                                     (long long)total, (long long)cap);
    hipLaunchKernelGGL(k_cell_pairs<true>, dim3(blocks_for(n, 128)), dim3(128), 0, ctx->stream, sys->pos, n, G, L,
                       iL, c2, cell, cellstart, cellatoms, nullptr, row_ptr, col);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_sort_long_rows, dim3(n), dim3(256), 0, ctx->stream, row_ptr, col);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_grid_cores(gdm_ctx* ctx, const gdm_system* sys, const int32_t grid[3], int32_t* core_of_atom,
                              int32_t* n_cores_out) {
    if (!ctx) return GDM_E_ARG;
    if (!sys || !grid || !core_of_atom || !n_cores_out || !sys->pos || !sys->anchor || sys->n_atoms <= 0)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_grid_cores: null argument or empty system");
    if (grid[0] < 1 || grid[1] < 1 || grid[2] < 1 || (int64_t)grid[0] * grid[1] * grid[2] > (1 << 26))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_grid_cores: bad grid %d x %d x %d", grid[0], grid[1], grid[2]);
    const int n = sys->n_atoms;
    const int64_t ncell = (int64_t)grid[0] * grid[1] * grid[2];
    bool ok = true;
    int32_t* cid = (int32_t*)gdm_buf(ctx, BUF_G_CELL, sizeof(int32_t) * (size_t)n, &ok);
    int32_t* flags = (int32_t*)gdm_buf(ctx, BUF_G_FLAGS, sizeof(int32_t) * (size_t)(ncell + 1), &ok);
    int32_t* remap = (int32_t*)gdm_buf(ctx, BUF_G_SCAN, sizeof(int32_t) * (size_t)(ncell + 1), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "workspace allocation failed (cores)");
    int rc;
    if ((rc = fill<int32_t>(ctx, flags, ncell + 1, 0))) return rc;
    double3 iL = make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]);
    hipLaunchKernelGGL(k_core_cells, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, sys->pos, sys->anchor, n,
                       grid[0], grid[1], grid[2], iL, cid, flags);
    GDM_LAUNCH_CHECK(ctx);
    if ((rc = gdm_scan_i32(ctx, flags, remap, ncell))) return rc;
    hipLaunchKernelGGL(k_core_remap, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, n, cid, remap,
                       core_of_atom);
    GDM_LAUNCH_CHECK(ctx);
    int32_t nc = 0;
    GDM_HIP(ctx, hipMemcpyAsync(&nc, remap + ncell, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *n_cores_out = nc;
    return GDM_OK;
}

extern "C" int gdm_extract_subgraphs(gdm_ctx* ctx, const gdm_system* sys, const gdm_tb_params* tb,
                                     const int32_t* row_ptr, const int32_t* col, const int32_t* core_of_atom,
                                     int32_t n_cores, int32_t* atom_ptr, int32_t* atoms, int64_t cap_atoms,
                                     int32_t* n_core, int32_t* h_norb, int32_t* h_ncore_orb,
                                     int64_t* total_atoms_out) {
    if (!ctx) return GDM_E_ARG;
    if (!sys || !tb || !row_ptr || !col || !core_of_atom || !atom_ptr || !atoms || !n_core || !total_atoms_out ||
        !sys->species)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_extract_subgraphs: null argument");
    if (n_cores <= 0 || sys->n_atoms <= 0 || sys->n_atoms > 1000000)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_extract_subgraphs: n_cores=%d n_atoms=%d out of range", n_cores,
                        sys->n_atoms);
    const int n = sys->n_atoms;
    const size_t lds = sizeof(uint32_t) * (size_t)((n + 31) / 32);
    if (lds > 64 * 1024) {
        GDM_HIP(ctx, hipFuncSetAttribute((const void*)k_extract<false>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        GDM_HIP(ctx, hipFuncSetAttribute((const void*)k_extract<true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    bool ok = true;
    int32_t* counts = (int32_t*)gdm_buf(ctx, BUF_G_COUNTS, sizeof(int32_t) * 4 * (size_t)n_cores, &ok);
    int32_t* natoms = (int32_t*)gdm_buf(ctx, BUF_G_TMP, sizeof(int32_t) * (size_t)(n_cores + 1), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "workspace allocation failed (extract)");
    hipLaunchKernelGGL(k_extract<false>, dim3(n_cores), dim3(kExtractThreads), lds, ctx->stream, n, sys->species,
                       row_ptr, col, core_of_atom, tb->n_orb[0], tb->n_orb[1], counts, nullptr, nullptr);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_extract_split, dim3(blocks_for(n_cores, 256)), dim3(256), 0, ctx->stream, n_cores, counts,
                       natoms, n_core);
    GDM_LAUNCH_CHECK(ctx);
    int rc;
    if ((rc = gdm_scan_i32(ctx, natoms, atom_ptr, n_cores))) return rc;
    std::vector<int32_t> hc(4 * (size_t)n_cores);
    int32_t total = 0;
    GDM_HIP(ctx, hipMemcpyAsync(hc.data(), counts, sizeof(int32_t) * hc.size(), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipMemcpyAsync(&total, atom_ptr + n_cores, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *total_atoms_out = total;
    for (int c = 0; c < n_cores; ++c) {
        if (h_norb) h_norb[c] = hc[4 * c + 2];
        if (h_ncore_orb) h_ncore_orb[c] = hc[4 * c + 3];
    }
    if (total > cap_atoms)
        return gdm_fail(ctx, GDM_E_CAPACITY, "subgraph atom list needs %lld entries, capacity %lld",
                        (long long)total, (long long)cap_atoms);
    hipLaunchKernelGGL(k_extract<true>, dim3(n_cores), dim3(kExtractThreads), lds, ctx->stream, n, sys->species,
                       row_ptr, col, core_of_atom, tb->n_orb[0], tb->n_orb[1], counts, atom_ptr, atoms);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}
