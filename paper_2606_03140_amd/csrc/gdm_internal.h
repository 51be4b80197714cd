// Internal declarations shared by the HIP translation units of libgdm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/gdm.h"

#define GDM_STATUS_NOT_PD 1
#define GDM_STATUS_NOT_CONVERGED 2
#define GDM_STATUS_NAN 4
#define GDM_STATUS_CAPACITY 8
#define GDM_STATUS_NO_BRACKET 16
#define GDM_STATUS_PARTITION 32

__host__ __device__ inline bool gdm_is_mixed(int precision) {
    return precision == GDM_MIXED_F16 || precision == GDM_MIXED_BF16;
}

// Per-subgraph descriptor for the dense solve (device resident).
struct SubDesc {
    int32_t n;        // orbitals
    int32_t nc;       // core orbitals
    int32_t ld;       // leading dimension of the dense n x n tiles
    int32_t natoms;   // atoms (core + halo)
    int32_t ncore_atoms;
    int32_t atom0;    // offset into the packed atom list
    int32_t dc_depth; // FP64 path: levels of the divide-and-conquer tree (leaves at this level)
    int32_t pad_;
    int64_t off2;     // offset of the ld*ld tiles
    int64_t offv;     // offset of length-ld vectors
    int64_t offc;     // offset of nc*ld core blocks
    int64_t offd;     // offset of the packed D core rows (nc*n)
    int64_t offe;     // offset of packed eigenvalues (n)
    int64_t offt;     // FP64 path: offset of the 64 x 64 T factors of the reflector blocks
};

// FP64 path, tridiagonal divide and conquer: a leaf or merge block [lo, hi)
// of one subgraph at one tree level (merge: children [lo, mid), [mid, hi)),
// and one 64 x 64 tile of the products with its factor.
struct DcNode {
    int32_t sub, lo, mid, hi, level, pad_;
    int64_t offu;     // offset of the block's k x k factor
};
struct DcTile {
    int32_t sub, lo, k, level, r0, c0;
    int64_t offu;
};
constexpr int kDcMaxRows = 2048;   // largest subgraph of the FP64 path (LDS of one merge)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Plan {
    int precision = -1;
    int n_sub = 0;
    std::vector<int32_t> n, nc;
    std::vector<SubDesc> desc;
    std::vector<int32_t> order;     // subgraph processing order (largest first)
    int64_t tot2 = 0, totv = 0, totc = 0, totd = 0, tote = 0, tott = 0;
    int32_t max_n = 0, max_nc = 0, max_natoms = 0;
    int generation = 0;
    // FP64 path: divide-and-conquer work lists (leaves, then merges by round;
    // product tiles forward and reverse by round)
    std::vector<DcNode> dc_nodes;
    std::vector<DcTile> dc_tiles;
    std::vector<int> dc_round, dc_fwd, dc_rev;
    int dc_max_depth = 0;
    int64_t dc_totu = 0;
    size_t dc_merge_lds = 0, dc_tiles_off = 0;
};

struct ProfRec {
    const char* name;
    hipEvent_t start, stop;
};

struct gdm_ctx {
    int device = 0;
    int n_cu = 256;             // compute units of the device
    hipStream_t stream = nullptr;
    int* d_status = nullptr;
    std::string err;
    Plan plan;
    // named device buffers (grown on demand at plan / graph time)
    DevBuf b[64];
    bool solved = false;        // find_mu has run on the current plan
    int solved_precision = -1;
    double mu_solved = 0.0;
    double kT_solved = 0.0;
    // mixed path: options and the state of the last find_mu
    int mixed_ns_z = 3;          // coupled Newton-Schulz iterations for s^-1/2 (first try)
    int mixed_ns_z_extra = 8;    // iterations that may be added while the residual is too large
    int mixed_ns_z_used = 0;     // iterations the last find_mu took
    int mu_out_device = 0;       // gdm_find_mu writes mu and N to device scalars (FP64 path)
    int fp64_leaf = 64;          // FP64 path: largest leaf of the divide-and-conquer tree (gdm_set_fp64_options)
    int mixed_packed = 1;        // expansion matrices stored as upper tiles (gdm_set_mixed_storage)
    int mixed_ns_inv = 1;        // Newton-Schulz iterations per inverse after its minimax start
    int mixed_inv_deg = 4;       // degree of that start: 4 (two products) or 2 (one product)
    int mixed_max_passes = 16;   // expansion passes allowed for mu
    int mixed_dev_passes = 3;    // passes launched by the device-side search (gdm_set_mixed_capture)
    int mixed_nd_launch = 12;    // doublings launched per pass by the device-side search
    bool mixed_dev_state = false;   // the last mixed search ran on the device (its state is there)
    int64_t mixed_tiles = 0, mixed_tiles_sym = 0, mixed_tiles_core = 0;
    int64_t mixed_upper_elems = 0;   // elements of the upper tiles of all subgraphs (packed storage)
    double mixed_flops_full = 0, mixed_flops_sym = 0;  // one product per launch
    double mixed_flops = 0;      // summed over the launches of the last find_mu
    double mixed_bytes = 0;      // algorithmic HBM bytes of those launches
    int64_t mixed_gemms = 0;
    int mixed_passes = 0;
    int mixed_nd = 0;
    double mixed_mu_pass = 0.0;
    double mixed_slope = 0.0;
    double mixed_beta = 0.0;
    // charge response: doubling history of the last expansion pass
    int mixed_rec_cap = 0;       // doublings that fit the history buffer (0: not recorded)
    int mixed_rec_nd = -1;       // doublings recorded by the last pass (-1: none)
    double mixed_x0_slope = 0.0; // dX_0 / dh_perp of that pass (X_0 = I/2 - q (h_perp - mu I))
    bool resp_v_ready = false;   // s[core,:] Z of the last find_mu is in the response buffer
    // tracing
    bool prof_on = false;
    std::vector<hipEvent_t> prof_pool;
    std::vector<ProfRec> prof;
};

// Record events around one launch when tracing is on.
struct GdmTimed {
    gdm_ctx* ctx;
    int idx = -1;
    GdmTimed(gdm_ctx* c, const char* name) : ctx(c) {
        if (!c->prof_on || 2 * (c->prof.size() + 1) > c->prof_pool.size()) return;
        idx = (int)c->prof.size();
        ProfRec r{name, c->prof_pool[2 * idx], c->prof_pool[2 * idx + 1]};
        c->prof.push_back(r);
        (void)hipEventRecord(r.start, c->stream);
    }
    ~GdmTimed() {
        if (idx >= 0) (void)hipEventRecord(ctx->prof[idx].stop, ctx->stream);
    }
};
#define GDM_TIMED(ctx, name) GdmTimed gdm_timed_scope_(ctx, name)

// Buffer slots.
enum {
    BUF_DESC = 0, BUF_ORDER, BUF_A, BUF_S, BUF_L, BUF_TAU, BUF_D, BUF_E, BUF_LAM, BUF_W,
    BUF_DCU, BUF_DCAUX, BUF_DCIDX, BUF_DCLIST, BUF_QC, BUF_QC2, BUF_HT, BUF_CC, BUF_MU, BUF_MUPART,
    BUF_G_CELL, BUF_G_CELLCNT, BUF_G_CELLSTART, BUF_G_CELLATOMS, BUF_G_CNT, BUF_G_TMP,
    BUF_G_FLAGS, BUF_G_COUNTS, BUF_G_SCAN, BUF_G_TOTAL, BUF_G_W,
    BUF_X_HI, BUF_X_LO, BUF_X_F, BUF_Y_HI, BUF_Y_LO, BUF_Y_F, BUF_T_HI, BUF_T_LO, BUF_T_F,
    BUF_Z_HI, BUF_Z_LO, BUF_Z_F, BUF_H_HI, BUF_H_LO, BUF_H_F, BUF_TR, BUF_GERSH, BUF_NDBL,
    BUF_TILES, BUF_PASS, BUF_EWALD, BUF_MIXPART,
    BUF_HIST_HI, BUF_HIST_LO, BUF_RESP, BUF_KRYLOV, BUF_MSTATE, BUF_FPAIR, BUF_FMAP, BUF_ESUM, BUF_TRDP,
    BUF_COUNT_
};

int gdm_fail(gdm_ctx* ctx, int code, const char* fmt, ...);
int gdm_hip(gdm_ctx* ctx, hipError_t e, const char* what);
void* gdm_buf(gdm_ctx* ctx, int slot, size_t bytes, bool* ok);
void gdm_buf_release(gdm_ctx* ctx, int slot);

#define GDM_HIP(ctx, call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return gdm_hip((ctx), e_, #call); \
    } while (0)

#define GDM_STR2_(x) #x
#define GDM_STR_(x) GDM_STR2_(x)
#define GDM_LAUNCH_CHECK(ctx)                                                         \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess) return gdm_hip((ctx), e_, "launch at " __FILE__ ":" GDM_STR_(__LINE__)); \
    } while (0)

// exclusive scan over n int32 (out has n+1 entries, out[n] = total) on stream
int gdm_scan_i32(gdm_ctx* ctx, const int32_t* in, int32_t* out, int64_t n);
int gdm_scan_i64(gdm_ctx* ctx, const int64_t* in, int64_t* out, int64_t n);
// fill n entries with v on the stream (a kernel, no memset node)
int gdm_fill_i32(gdm_ctx* ctx, int32_t* p, int64_t n, int32_t v);
int gdm_fill_f64(gdm_ctx* ctx, double* p, int64_t n, double v);

// solve paths
int gdm_fp64_find_mu(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                     const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                     const double* H, const double* S, double n_e, double kT,
                     double* mu_out, double* n_out);
// mu_dev: when non-null, the kernel reads mu from this device scalar instead
// energy != 0: the energy-weighted rows C[core,:] diag(f lam) C^T instead of D
int gdm_fp64_density(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, const double* mu_dev, double kT,
                     double* D_core, double* eig_out, int energy);
// electronic free energy 2 sum_s sum_k w_k [f lam + kT s(f)] of the last FP64 solve (device scalar out)
int gdm_fp64_band_energy(gdm_ctx* ctx, double mu, double kT, double* out_dev);
// raise the dynamic-LDS attributes the FP64 kernels need for the current plan
int gdm_fp64_plan_lds(gdm_ctx* ctx);
// tridiagonal divide and conquer (FP64 path): work lists and workspace at
// plan time; eigenvalues and factors from the tridiagonal (BUF_D, BUF_E);
// products of the core rows with the eigenvector matrix (reverse: with its
// transpose)
int gdm_dc_depth(int n, int leaf);
int gdm_dc_plan(gdm_ctx* ctx);
int gdm_dc_solve(gdm_ctx* ctx);
int gdm_dc_apply(gdm_ctx* ctx, int reverse);
int gdm_mixed_find_mu(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                      const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                      const double* H, const double* S, double n_e, double kT,
                      double mu_guess, double tol_N, double* mu_out, double* n_out);
int gdm_mixed_plan(gdm_ctx* ctx);
int gdm_mixed_density(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, const double* mu_dev, double kT,
                      double* D_core);
int gdm_mixed_pass_mu(gdm_ctx* ctx, double* mu_pass);
int gdm_mixed_response_alloc(gdm_ctx* ctx);
int gdm_mixed_response(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                       const int32_t* row_ptr, const int32_t* col, int64_t nnz, const double* S,
                       const double* dV, double* dq, double* dmu);
int gdm_launch_mulliken(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                        const int32_t* row_ptr, const int32_t* col, int64_t nnz, const double* S,
                        const double* D_core, const double n0[2], double* q_out);

// gather of principal submatrices (shared by both solvers)
int gdm_launch_gather(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                      const int32_t* row_ptr, const int32_t* col, int64_t nnz,
                      const double* H, const double* S, double* A, double* Sd, int orthogonal);

// ---- device helpers
__device__ __forceinline__ int gdm_lower_bound(const int32_t* a, int n, int32_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double gdm_wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float gdm_wave_sumf(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int gdm_wave_sumi(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Taper of the radial functions: 1 below r_on, 1 - x^3 (10 - 15 x + 6 x^2)
// with x = (r - r_on)/(r_c - r_on) up to r_c; *dt (nullable) = dt/dr
__host__ __device__ inline double gdm_taper(double r, double r_on, double r_c, double* dt) {
    if (r <= r_on) {
        if (dt) *dt = 0.0;
        return 1.0;
    }
    const double w = r_c - r_on, x = (r - r_on) / w;
    if (x >= 1.0) {
        if (dt) *dt = 0.0;
        return 0.0;
    }
    if (dt) *dt = -30.0 * x * x * (1.0 - x) * (1.0 - x) / w;
    return 1.0 - x * x * x * (10.0 - 15.0 * x + 6.0 * x * x);
}

__device__ __forceinline__ void gdm_raise(int* status, int flag) {
    atomicOr(status, flag);
}
