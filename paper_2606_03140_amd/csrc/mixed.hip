// Mixed-precision recursive Fermi-operator expansion (the "recursive
// Fermi-operator expansion" option of the paper's subgraph step, run on the
// matrix cores as the paper's accelerator library does for FOE and the
// inverse overlap).  Per subgraph, padded to P = 64 * ceil(n / 64):
//
//   Z = s^-1/2 by coupled Newton-Schulz (Y0 = s/c, Z0 = I,
//       T = (3I - Z Y)/2, Y <- Y T, Z <- T Z; then Z /= sqrt(c)),
//   h_perp = Z h Z,  W = Z s,
//   X0 = I/2 - (b/4)(h_perp - mu I),  b = beta / 2^n_d,
//   n_d times:  X2 = X X,  A = 2 X2 - 2 X + I = X^2 + (I - X)^2,
//               Y = A^-1 by Newton-Schulz from the minimax start
//               Y0 = 48/17 I - 32/17 A (|I - A Y0| <= 1/17 on [1/2, 1]),
//               X <- X2 Y            (f_b -> f_2b),
//   N(mu) = 2 sum_core (Z X W)_aa,  N'(mu) = 2 beta sum_core (Z (X - X^2) W)_aa
//   in FP64, Newton steps on mu with a bisection bracket, and the final
//   collected core rows D = Z[core,:] (X + dmu beta (X - X^2)) Z in FP64.
//
// Every GEMM uses split FP16 operands x = hi + 2^-11 lo with FP32
// accumulation: AB = Ah Bh + 2^-11 (Ah Bl + Al Bh) on v_mfma_f32_16x16x32_f16.
// All products are of symmetric matrices, so B[k][n] = B[n][k] and both
// operands are read row-major (C = A B^T form).
#include "gdm_internal.h"

#include <algorithm>
#include <cmath>

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

namespace {

constexpr int kTile = 64;       // output tile edge per workgroup
constexpr int kK = 32;          // k-step (one MFMA k)
constexpr int kLdsRow = kK + 8; // padded LDS row (halves)
constexpr int kGemmThreads = 256;
constexpr float kLoScale = 2048.0f;            // 2^11
constexpr float kLoInv = 1.0f / 2048.0f;

struct SplitMat {
    float* f;
    _Float16* hi;
    _Float16* lo;
};

struct GemmArgs {
    SplitMat A, B;       // operands (hi/lo used)
    SplitMat O1;         // raw product (nullable members)
    SplitMat O2;         // alpha*AB + beta*E + gamma*I
    const float* E;
    float alpha, beta, gamma;
    int sym;             // tiles cover i <= j only; results mirrored (exactly symmetric output)
};

__device__ __forceinline__ void store_split(const SplitMat& m, int64_t idx, float v) {
    if (m.f) m.f[idx] = v;
    if (m.hi) {
        _Float16 h = (_Float16)v;
        m.hi[idx] = h;
        m.lo[idx] = (_Float16)((v - (float)h) * kLoScale);
    }
}

// Tile list entries: (subgraph, tile row, tile col)
__global__ void __launch_bounds__(kGemmThreads) k_gemm_split(const SubDesc* __restrict__ desc,
                                                            const int4* __restrict__ tiles, GemmArgs g) {
    __shared__ __attribute__((aligned(16))) _Float16 sAh[kTile * kLdsRow];
    __shared__ __attribute__((aligned(16))) _Float16 sAl[kTile * kLdsRow];
    __shared__ __attribute__((aligned(16))) _Float16 sBh[kTile * kLdsRow];
    __shared__ __attribute__((aligned(16))) _Float16 sBl[kTile * kLdsRow];
    const int4 tl = tiles[blockIdx.x];
    const SubDesc d = desc[tl.x];
    const int P = d.ld;
    const int64_t base = d.off2;
    const int m0 = tl.y * kTile, n0 = tl.z * kTile;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // global -> LDS assignment: thread t loads 16 B (8 halves) of row t/4, chunk t%4
    const int lr = t >> 2, lc = (t & 3) * 8;
    const _Float16* gAh = g.A.hi + base + (int64_t)(m0 + lr) * P + lc;
    const _Float16* gAl = g.A.lo + base + (int64_t)(m0 + lr) * P + lc;
    const _Float16* gBh = g.B.hi + base + (int64_t)(n0 + lr) * P + lc;
    const _Float16* gBl = g.B.lo + base + (int64_t)(n0 + lr) * P + lc;
    float4v acc_hh[2][2], acc_x[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            acc_hh[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
            acc_x[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
        }
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int k0 = 0; k0 < P; k0 += kK) {
        uint4 va = *(const uint4*)(gAh + k0);
        uint4 vb = *(const uint4*)(gAl + k0);
        uint4 vc = *(const uint4*)(gBh + k0);
        uint4 vd = *(const uint4*)(gBl + k0);
        __syncthreads();
        *(uint4*)(sAh + lr * kLdsRow + lc) = va;
        *(uint4*)(sAl + lr * kLdsRow + lc) = vb;
        *(uint4*)(sBh + lr * kLdsRow + lc) = vc;
        *(uint4*)(sBl + lr * kLdsRow + lc) = vd;
        __syncthreads();
        half8 ah[2], al[2], bh[2], bl[2];
        for (int i = 0; i < 2; ++i) {
            const int r = wm * 32 + i * 16 + fr;
            ah[i] = *(const half8*)(sAh + r * kLdsRow + fk);
            al[i] = *(const half8*)(sAl + r * kLdsRow + fk);
        }
        for (int j = 0; j < 2; ++j) {
            const int c = wn * 32 + j * 16 + fr;
            bh[j] = *(const half8*)(sBh + c * kLdsRow + fk);
            bl[j] = *(const half8*)(sBl + c * kLdsRow + fk);
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                acc_hh[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc_hh[i][j], 0, 0, 0);
                acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc_x[i][j], 0, 0, 0);
                acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc_x[i][j], 0, 0, 0);
            }
    }
    // epilogue.  In symmetric mode the tile list holds tile rows <= tile
    // columns; every value is written at (m, n) and mirrored to (n, m), and in
    // a diagonal tile only m <= n is taken, so the output is exactly symmetric.
    const bool diag_tile = tl.y == tl.z;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn * 32 + j * 16 + (lane & 15);
                if (g.sym && diag_tile && m > n) continue;
                const int64_t idx = base + (int64_t)m * P + n;
                const int64_t tdx = base + (int64_t)n * P + m;
                const bool mirror = g.sym && m != n;
                const float v = acc_hh[i][j][r] + kLoInv * acc_x[i][j][r];
                if (g.O1.f || g.O1.hi) {
                    store_split(g.O1, idx, v);
                    if (mirror) store_split(g.O1, tdx, v);
                }
                if (g.O2.f || g.O2.hi) {
                    float o = g.alpha * v;
                    if (g.E) o += g.beta * g.E[idx];
                    if (m == n) o += g.gamma;
                    store_split(g.O2, idx, o);
                    if (mirror) store_split(g.O2, tdx, o);
                }
            }
}


// ------------------------------------------------------------ FP64 GEMM
// C = alpha A B + beta Cin + gamma I on the padded P x P tiles, true product
// (no symmetry assumed), FP64 FMA.  64 x 64 output tile per workgroup, each
// thread a 4 x 4 block, k-steps of 16 staged in LDS.  TA / TB: double or float.
template <typename TA, typename TB>
__global__ void __launch_bounds__(256) k_gemm64(const SubDesc* __restrict__ desc, const int4* __restrict__ tiles,
                                               const TA* __restrict__ A, const TB* __restrict__ B,
                                               const double* __restrict__ Cin, double* __restrict__ C,
                                               double alpha, double beta, double gamma) {
    __shared__ double sA[16][64 + 1];   // sA[k][m]
    __shared__ double sB[16][64 + 1];   // sB[k][n]
    const int4 tl = tiles[blockIdx.x];
    const SubDesc d = desc[tl.x];
    const int P = d.ld;
    const int64_t base = d.off2;
    const int m0 = tl.y * 64, n0 = tl.z * 64;
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    double acc[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < P; k0 += 16) {
        __syncthreads();
        for (int e = t; e < 16 * 64; e += 256) {
            const int r = e >> 4, k = e & 15;             // A: row m0+r, col k0+k
            sA[k][r] = (double)A[base + (int64_t)(m0 + r) * P + k0 + k];
            const int kb = e >> 6, c = e & 63;            // B: row k0+kb, col n0+c
            sB[kb][c] = (double)B[base + (int64_t)(k0 + kb) * P + n0 + c];
        }
        __syncthreads();
        for (int k = 0; k < 16; ++k) {
            double a[4], b[4];
            for (int i = 0; i < 4; ++i) a[i] = sA[k][ty * 4 + i];
            for (int j = 0; j < 4; ++j) b[j] = sB[k][tx * 4 + j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
            const int64_t idx = base + (int64_t)m * P + n;
            double v = alpha * acc[i][j];
            if (Cin) v += beta * Cin[idx];
            if (m == n) v += gamma;
            C[idx] = v;
        }
}

// Z64 (FP64) <- its FP32 split copy for the expansion
__global__ void __launch_bounds__(256) k_z64_to_split(const SubDesc* __restrict__ desc, const double* __restrict__ Z64,
                                                     SplitMat Z) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld;
    for (int64_t e = threadIdx.x; e < (int64_t)P * P; e += 256) store_split(Z, d.off2 + e, (float)Z64[d.off2 + e]);
}

// FP32 -> FP64 copy (the Newton-Schulz Z before refinement)
__global__ void __launch_bounds__(256) k_f32_to_f64(const SubDesc* __restrict__ desc, const float* __restrict__ src,
                                                   double* __restrict__ dst) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld;
    for (int64_t e = threadIdx.x; e < (int64_t)P * P; e += 256) dst[d.off2 + e] = (double)src[d.off2 + e];
}

// ------------------------------------------------------- elementwise kernels
constexpr int kEw = 256;

__device__ __forceinline__ double block_reduce_max(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < kEw / 64; ++w) r = fmax(r, red[w]);
    return r;
}

__device__ __forceinline__ double block_reduce_min(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < kEw / 64; ++w) r = fmin(r, red[w]);
    return r;
}

__device__ __forceinline__ double block_reduce_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < kEw / 64; ++w) r += red[w];
    return r;
}

// From the gathered FP64 h, s (leading dimension P): the Gershgorin upper
// bound c of s, then S = s, H = h, Y0 = s / c, Z0 = I (padding: identity for
// S, Y, Z and zero for H).
__global__ void __launch_bounds__(kEw) k_prep(const SubDesc* __restrict__ desc, double* __restrict__ h64,
                                             double* __restrict__ s64, SplitMat S, SplitMat H, SplitMat Y,
                                             SplitMat Z, double* __restrict__ scale, int orthogonal) {
    __shared__ double red[kEw / 64];
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld;
    const int64_t base = d.off2;
    double rmax = 0.0;
    if (!orthogonal)
        for (int i = threadIdx.x; i < n; i += kEw) {
            const double* row = s64 + base + (int64_t)i * P;
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += fabs(row[j]);
            rmax = fmax(rmax, acc);
        }
    const double c = orthogonal ? 1.0 : block_reduce_max(rmax, red);
    if (threadIdx.x == 0) scale[blockIdx.x] = c;
    const float ic = (float)(1.0 / c);
    for (int64_t e = threadIdx.x; e < (int64_t)P * P; e += kEw) {
        const int i = (int)(e / P), j = (int)(e - (int64_t)i * P);
        const int64_t idx = base + e;
        const bool in = i < n && j < n;
        float sv = in ? (orthogonal ? (i == j ? 1.f : 0.f) : (float)s64[idx]) : (i == j ? 1.f : 0.f);
        float hv = in ? (float)h64[idx] : 0.f;
        store_split(S, idx, sv);
        store_split(H, idx, hv);
        store_split(Y, idx, in ? sv * ic : (i == j ? 1.f : 0.f));
        store_split(Z, idx, i == j ? 1.f : 0.f);
        if (!in) {     // padding of the FP64 tiles: h = 0, s = I
            h64[idx] = 0.0;
            s64[idx] = i == j ? 1.0 : 0.0;
        }
    }
}

// Z <- Z / sqrt(c) on the n x n block (padding stays identity)
__global__ void __launch_bounds__(kEw) k_scale_z(const SubDesc* __restrict__ desc, SplitMat Z,
                                                const double* __restrict__ scale) {
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld;
    const float f = (float)(1.0 / sqrt(scale[blockIdx.x]));
    for (int64_t e = threadIdx.x; e < (int64_t)P * P; e += kEw) {
        const int i = (int)(e / P), j = (int)(e - (int64_t)i * P);
        if (i >= n || j >= n) continue;
        const int64_t idx = d.off2 + e;
        store_split(Z, idx, Z.f[idx] * f);
    }
}

// H <- (H + H^T)/2 on the n x n block; Gershgorin bounds in FP64 -> bounds[2s], bounds[2s+1]
__global__ void __launch_bounds__(kEw) k_sym_bounds(const SubDesc* __restrict__ desc, SplitMat H,
                                                   double* __restrict__ bounds) {
    __shared__ double red[kEw / 64];
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld;
    const int64_t base = d.off2;
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kEw) {
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        if (j <= i) continue;
        const float v = 0.5f * (H.f[base + (int64_t)i * P + j] + H.f[base + (int64_t)j * P + i]);
        store_split(H, base + (int64_t)i * P + j, v);
        store_split(H, base + (int64_t)j * P + i, v);
    }
    __syncthreads();
    double lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < n; i += kEw) {
        const float* row = H.f + base + (int64_t)i * P;
        double r = 0.0;
        for (int j = 0; j < n; ++j)
            if (j != i) r += fabs((double)row[j]);
        lo = fmin(lo, (double)row[i] - r);
        hi = fmax(hi, (double)row[i] + r);
    }
    lo = block_reduce_min(lo, red);
    hi = block_reduce_max(hi, red);
    if (threadIdx.x == 0) {
        bounds[2 * blockIdx.x] = lo;
        bounds[2 * blockIdx.x + 1] = hi;
    }
}

// X0 = I/2 - (b/4)(H - mu I) on the n x n block, zero padding
__global__ void __launch_bounds__(kEw) k_x0(const SubDesc* __restrict__ desc, const float* __restrict__ Hf,
                                           SplitMat X, double mu, double b) {
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld;
    const double q = b / 4.0;
    for (int64_t e = threadIdx.x; e < (int64_t)P * P; e += kEw) {
        const int i = (int)(e / P), j = (int)(e - (int64_t)i * P);
        const int64_t idx = d.off2 + e;
        float v = 0.f;
        if (i < n && j < n) {
            double hv = (double)Hf[idx];
            v = (float)((i == j ? 0.5 : 0.0) - q * (hv - (i == j ? mu : 0.0)));
        }
        store_split(X, idx, v);
    }
}

// Per subgraph (FP64, refined Z):
//   N_s = 2 sum_{a<nc} sum_c G_ac W_ca,  M_s = 2 sum_{a<nc} sum_c Gp_ac W_ca
//   G = Z[core,:] X, Gp = Z[core,:] (X - X2), W[:, a] = Z s[:, a] (core columns).
__global__ void __launch_bounds__(kEw) k_traces(const SubDesc* __restrict__ desc, const double* __restrict__ Z64,
                                               const float* __restrict__ Xf, const float* __restrict__ X2f,
                                               const double* __restrict__ s64, double* __restrict__ part) {
    __shared__ double red[kEw / 64];
    extern __shared__ double sm[];
    double* zrow = sm;           // [n]
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld, nc = d.nc;
    const int64_t base = d.off2;
    double accN = 0.0, accM = 0.0;
    for (int a = 0; a < nc; ++a) {
        __syncthreads();
        for (int b = threadIdx.x; b < n; b += kEw) zrow[b] = Z64[base + (int64_t)a * P + b];
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += kEw) {
            double gx = 0.0, gp = 0.0, w = 0.0;
            const double* zc = Z64 + base + (int64_t)c * P;
            for (int b = 0; b < n; ++b) {
                const double x = (double)Xf[base + (int64_t)b * P + c];
                const double x2 = (double)X2f[base + (int64_t)b * P + c];
                gx += zrow[b] * x;
                gp += zrow[b] * (x - x2);
                w += zc[b] * s64[base + (int64_t)b * P + a];
            }
            accN += gx * w;
            accM += gp * w;
        }
    }
    accN = block_reduce_sum(accN, red);
    accM = block_reduce_sum(accM, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = 2.0 * accN;
        part[2 * blockIdx.x + 1] = 2.0 * accM;
    }
}

__global__ void k_sum_parts(int n_sub, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[kEw / 64];
    double a = 0.0, b = 0.0;
    for (int s = threadIdx.x; s < n_sub; s += kEw) {
        a += part[2 * s];
        b += part[2 * s + 1];
    }
    a = block_reduce_sum(a, red);
    b = block_reduce_sum(b, red);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// D_core[a][j] = sum_c G[a][c] Z[c][j],  G[a][c] = sum_b Z[a][b] (X + kappa (X - X2))[b][c]   (FP64)
__global__ void __launch_bounds__(kEw) k_dcore_mixed(const SubDesc* __restrict__ desc, const double* __restrict__ Zf,
                                                    const float* __restrict__ Xf, const float* __restrict__ X2f,
                                                    double kappa, double* __restrict__ Gbuf,
                                                    double* __restrict__ Dout) {
    extern __shared__ double zrow[];
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld, nc = d.nc;
    const int64_t base = d.off2;
    double* G = Gbuf + d.offc;                // nc x n (ld = n)
    for (int a = 0; a < nc; ++a) {
        __syncthreads();
        for (int b = threadIdx.x; b < n; b += kEw) zrow[b] = Zf[base + (int64_t)a * P + b];
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += kEw) {
            double g = 0.0;
            for (int b = 0; b < n; ++b) {
                const double x = (double)Xf[base + (int64_t)b * P + c];
                const double x2 = (double)X2f[base + (int64_t)b * P + c];
                g += zrow[b] * (x + kappa * (x - x2));
            }
            G[(int64_t)a * n + c] = g;
        }
    }
    __syncthreads();
    double* out = Dout + d.offd;
    for (int a = 0; a < nc; ++a) {
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += kEw) zrow[c] = G[(int64_t)a * n + c];
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += kEw) {
            double acc = 0.0;
            for (int c = 0; c < n; ++c) acc += zrow[c] * Zf[base + (int64_t)c * P + j];
            out[(int64_t)a * n + j] = acc;
        }
    }
}

}  // namespace

// --------------------------------------------------------------------- host

enum { SL_S = 0, SL_H, SL_Y, SL_Z, SL_T, SL_Y2, SL_Z2, SL_HP, SL_W, SL_X, SL_X2, SL_A, SL_R, SL_YI, SL_COUNT };

static SplitMat slot(gdm_ctx* ctx, int k) {
    const int64_t tot = ctx->plan.tot2;
    float* f = (float*)ctx->b[BUF_X_F].p + (int64_t)k * tot;
    _Float16* hi = (_Float16*)ctx->b[BUF_X_HI].p + (int64_t)k * tot;
    _Float16* lo = (_Float16*)ctx->b[BUF_X_LO].p + (int64_t)k * tot;
    return SplitMat{f, hi, lo};
}

static SplitMat none() { return SplitMat{nullptr, nullptr, nullptr}; }

int gdm_mixed_plan(gdm_ctx* ctx) {
    Plan& P = ctx->plan;
    // tiles in decreasing subgraph size order (long subgraphs first)
    std::vector<int> order(P.n_sub);
    for (int s = 0; s < P.n_sub; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.n[a] > P.n[b]; });
    std::vector<int4> tiles, utiles;
    double ffull = 0.0, fsym = 0.0;
    for (int s : order) {
        const int nt = P.desc[s].ld / kTile;
        const double pt = 2.0 * kTile * kTile * (double)P.desc[s].ld;   // flops of one output tile
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < nt; ++j) {
                tiles.push_back(make_int4(s, i, j, 0));
                ffull += pt;
                if (i <= j) {
                    utiles.push_back(make_int4(s, i, j, 0));
                    fsym += pt;
                }
            }
    }
    const size_t nfull = tiles.size();
    tiles.insert(tiles.end(), utiles.begin(), utiles.end());
    bool ok = true;
    int4* dt = (int4*)gdm_buf(ctx, BUF_TILES, sizeof(int4) * tiles.size(), &ok);
    gdm_buf(ctx, BUF_A, sizeof(double) * P.tot2, &ok);
    gdm_buf(ctx, BUF_S, sizeof(double) * P.tot2, &ok);
    gdm_buf(ctx, BUF_X_F, sizeof(float) * P.tot2 * SL_COUNT, &ok);
    gdm_buf(ctx, BUF_X_HI, sizeof(_Float16) * P.tot2 * SL_COUNT, &ok);
    gdm_buf(ctx, BUF_X_LO, sizeof(_Float16) * P.tot2 * SL_COUNT, &ok);
    gdm_buf(ctx, BUF_GERSH, sizeof(double) * 2 * (size_t)P.n_sub, &ok);
    gdm_buf(ctx, BUF_TR, sizeof(double) * (2 * (size_t)P.n_sub + 8), &ok);
    gdm_buf(ctx, BUF_NDBL, sizeof(double) * (size_t)P.n_sub, &ok);
    gdm_buf(ctx, BUF_CC, sizeof(double) * (size_t)P.totc, &ok);
    gdm_buf(ctx, BUF_L, sizeof(double) * P.tot2 * 3, &ok);     // F, E, Z64 of the FP64 refinement
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_plan: mixed workspace allocation failed");
    GDM_HIP(ctx, hipMemcpyAsync(dt, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, ctx->stream));
    ctx->mixed_tiles = (int64_t)nfull;
    ctx->mixed_tiles_sym = (int64_t)utiles.size();
    ctx->mixed_flops_full = ffull;
    ctx->mixed_flops_sym = fsym;
    return GDM_OK;
}

// C = A B for symmetric B (read row-major as B^T).  sym = 1 when A and B
// commute (products of polynomials in the same matrix): only upper tiles are
// computed and mirrored.
static int gemm(gdm_ctx* ctx, SplitMat A, SplitMat B, SplitMat O1, SplitMat O2, const float* E, float alpha,
                float beta, float gamma, const char* tag, int sym = 1) {
    GemmArgs g{A, B, O1, O2, E, alpha, beta, gamma, sym};
    const int4* tl = (const int4*)ctx->b[BUF_TILES].p + (sym ? ctx->mixed_tiles : 0);
    const int64_t nt = sym ? ctx->mixed_tiles_sym : ctx->mixed_tiles;
    GDM_TIMED(ctx, tag);
    hipLaunchKernelGGL(k_gemm_split, dim3((unsigned)nt), dim3(kGemmThreads), 0, ctx->stream,
                       (const SubDesc*)ctx->b[BUF_DESC].p, tl, g);
    GDM_LAUNCH_CHECK(ctx);
    ctx->mixed_gemms += 1;
    ctx->mixed_flops += sym ? ctx->mixed_flops_sym : ctx->mixed_flops_full;
    return GDM_OK;
}

#define GDM_TRY(x)          \
    do {                    \
        int rc_ = (x);      \
        if (rc_) return rc_; \
    } while (0)

// One full recursive expansion at chemical potential mu; leaves X in SL_X and X^2 in SL_X2.
static int foe_pass(gdm_ctx* ctx, double mu, double beta, double lo, double hi, int* nd_out) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const double R = std::max(std::fabs(lo - mu), std::fabs(hi - mu));
    int nd = (int)std::ceil(std::log2(beta * R));
    nd = std::max(1, std::min(nd, 40));
    const double b = beta / std::ldexp(1.0, nd);
    *nd_out = nd;
    {
        GDM_TIMED(ctx, "mixed_misc");
        hipLaunchKernelGGL(k_x0, dim3(P.n_sub), dim3(kEw), 0, ctx->stream, desc, slot(ctx, SL_HP).f, slot(ctx, SL_X),
                           mu, b);
    }
    GDM_LAUNCH_CHECK(ctx);
    const float c0 = 48.0f / 17.0f, c1 = -32.0f / 17.0f;
    SplitMat X = slot(ctx, SL_X), X2 = slot(ctx, SL_X2), A = slot(ctx, SL_A), Rm = slot(ctx, SL_R);
    SplitMat Y = slot(ctx, SL_Y), Yn = slot(ctx, SL_YI);
    for (int it = 0; it < nd; ++it) {
        // X2 = X X ; A = 2 X2 - 2 X + I
        GDM_TRY(gemm(ctx, X, X, X2, A, X.f, 2.0f, -2.0f, 1.0f, "foe_gemm"));
        // Newton-Schulz inverse of A from Y0 = c0 I + c1 A:
        //   R = 2I - A Y0 = 2I - c0 A - c1 A A ;  Y1 = Y0 R = c0 R + c1 A R
        GDM_TRY(gemm(ctx, A, A, none(), Rm, A.f, -c1, -c0, 2.0f, "foe_gemm"));
        GDM_TRY(gemm(ctx, A, Rm, none(), Y, Rm.f, c1, c0, 0.0f, "foe_gemm"));
        for (int k = 1; k < ctx->mixed_ns_inv; ++k) {
            GDM_TRY(gemm(ctx, A, Y, none(), Rm, nullptr, -1.0f, 0.0f, 2.0f, "foe_gemm"));
            GDM_TRY(gemm(ctx, Y, Rm, Yn, none(), nullptr, 1.0f, 0.0f, 0.0f, "foe_gemm"));
            std::swap(Y, Yn);
        }
        // X <- X2 Y
        GDM_TRY(gemm(ctx, X2, Y, X, none(), nullptr, 1.0f, 0.0f, 0.0f, "foe_gemm"));
    }
    // X^2 of the final X (for N'(mu) and the first-order mu correction)
    GDM_TRY(gemm(ctx, X, X, X2, none(), nullptr, 1.0f, 0.0f, 0.0f, "foe_gemm"));
    return GDM_OK;
}

static double* z64(gdm_ctx* ctx) { return (double*)ctx->b[BUF_L].p + 2 * ctx->plan.tot2; }

static int gemm64_ff(gdm_ctx* ctx, const double* A, const float* B, const double* Cin, double* C, double alpha,
                     double beta, double gamma) {
    GDM_TIMED(ctx, "refine64");
    hipLaunchKernelGGL((k_gemm64<double, float>), dim3((unsigned)ctx->mixed_tiles), dim3(256), 0, ctx->stream,
                       (const SubDesc*)ctx->b[BUF_DESC].p, (const int4*)ctx->b[BUF_TILES].p, A, B, Cin, C, alpha,
                       beta, gamma);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

static int gemm64_dd(gdm_ctx* ctx, const double* A, const double* B, const double* Cin, double* C, double alpha,
                     double beta, double gamma) {
    GDM_TIMED(ctx, "refine64");
    hipLaunchKernelGGL((k_gemm64<double, double>), dim3((unsigned)ctx->mixed_tiles), dim3(256), 0, ctx->stream,
                       (const SubDesc*)ctx->b[BUF_DESC].p, (const int4*)ctx->b[BUF_TILES].p, A, B, Cin, C, alpha,
                       beta, gamma);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

static int traces(gdm_ctx* ctx, double* N, double* M) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    double* part = (double*)ctx->b[BUF_TR].p;
    {
        GDM_TIMED(ctx, "traces");
        hipLaunchKernelGGL(k_traces, dim3(P.n_sub), dim3(kEw), sizeof(double) * P.max_n, ctx->stream, desc,
                           z64(ctx), slot(ctx, SL_X).f, slot(ctx, SL_X2).f, (const double*)ctx->b[BUF_S].p, part);
        GDM_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kEw), 0, ctx->stream, P.n_sub, part,
                           part + 2 * (size_t)P.n_sub);
        GDM_LAUNCH_CHECK(ctx);
    }
    double h[2];
    GDM_HIP(ctx, hipMemcpyAsync(h, part + 2 * (size_t)P.n_sub, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *N = h[0];
    *M = h[1];
    return GDM_OK;
}

int gdm_mixed_find_mu(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg, const int32_t* row_ptr,
                      const int32_t* col, int64_t nnz, const double* H, const double* S, double n_e, double kT,
                      double mu_guess, double tol_N, double* mu_out, double* n_out) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const double beta = 1.0 / kT;
    const int orth = S == nullptr;
    double* h64 = (double*)ctx->b[BUF_A].p;
    double* s64 = (double*)ctx->b[BUF_S].p;
    double* scale = (double*)ctx->b[BUF_NDBL].p;
    double* bounds = (double*)ctx->b[BUF_GERSH].p;
    ctx->mixed_gemms = 0;
    ctx->mixed_flops = 0.0;
    GDM_TRY(gdm_launch_gather(ctx, sys, sg, row_ptr, col, nnz, H, S, h64, s64, orth));
    {
        GDM_TIMED(ctx, "mixed_misc");
        hipLaunchKernelGGL(k_prep, dim3(P.n_sub), dim3(kEw), 0, ctx->stream, desc, h64, s64, slot(ctx, SL_S),
                           slot(ctx, SL_H), slot(ctx, SL_Y), slot(ctx, SL_Z), scale, orth);
    }
    GDM_LAUNCH_CHECK(ctx);
    // coupled Newton-Schulz: Z -> (s/c)^-1/2
    SplitMat Y = slot(ctx, SL_Y), Z = slot(ctx, SL_Z), T = slot(ctx, SL_T), Y2 = slot(ctx, SL_Y2),
             Z2 = slot(ctx, SL_Z2);
    if (!orth) {
        for (int it = 0; it < ctx->mixed_ns_z; ++it) {
            GDM_TRY(gemm(ctx, Z, Y, none(), T, nullptr, -0.5f, 0.0f, 1.5f, "ns_gemm"));
            GDM_TRY(gemm(ctx, Y, T, Y2, none(), nullptr, 1.0f, 0.0f, 0.0f, "ns_gemm"));
            GDM_TRY(gemm(ctx, T, Z, Z2, none(), nullptr, 1.0f, 0.0f, 0.0f, "ns_gemm"));
            std::swap(Y, Y2);
            std::swap(Z, Z2);
        }
        {
            GDM_TIMED(ctx, "mixed_misc");
            hipLaunchKernelGGL(k_scale_z, dim3(P.n_sub), dim3(kEw), 0, ctx->stream, desc, Z, scale);
        }
        GDM_LAUNCH_CHECK(ctx);
    }
    // keep the final Z in SL_Z
    if (Z.f != slot(ctx, SL_Z).f) {
        const int64_t tot = P.tot2;
        GDM_HIP(ctx, hipMemcpyAsync(slot(ctx, SL_Z).f, Z.f, sizeof(float) * tot, hipMemcpyDeviceToDevice, ctx->stream));
        GDM_HIP(ctx, hipMemcpyAsync(slot(ctx, SL_Z).hi, Z.hi, sizeof(_Float16) * tot, hipMemcpyDeviceToDevice,
                                    ctx->stream));
        GDM_HIP(ctx, hipMemcpyAsync(slot(ctx, SL_Z).lo, Z.lo, sizeof(_Float16) * tot, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    }
    Z = slot(ctx, SL_Z);
    // FP64 residual refinement of Z (Z s Z = I): F = s Z, E = Z F - I,
    // Z64 = Z - Z E / 2 (error O(E^2)); Z64 serves the traces and the final
    // step, its FP32 split copy the expansion.
    {
        double* F = (double*)ctx->b[BUF_L].p;
        double* E = F + P.tot2;
        double* Z64 = E + P.tot2;
        {
            GDM_TIMED(ctx, "refine64");
            hipLaunchKernelGGL(k_f32_to_f64, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, Z.f, Z64);
        }
        GDM_LAUNCH_CHECK(ctx);
        GDM_TRY(gemm64_ff(ctx, s64, Z.f, nullptr, F, 1.0, 0.0, 0.0));
        GDM_TRY(gemm64_dd(ctx, Z64, F, nullptr, E, 1.0, 0.0, -1.0));     // E = Z (s Z) - I
        GDM_TRY(gemm64_dd(ctx, Z64, E, Z64, F, -0.5, 1.0, 0.0));        // F <- Z - Z E / 2
        GDM_HIP(ctx, hipMemcpyAsync(Z64, F, sizeof(double) * P.tot2, hipMemcpyDeviceToDevice, ctx->stream));
        {
            GDM_TIMED(ctx, "refine64");
            hipLaunchKernelGGL(k_z64_to_split, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, Z64, Z);
        }
        GDM_LAUNCH_CHECK(ctx);
    }
    // h_perp = Z h Z (T = Z h, then T Z)
    GDM_TRY(gemm(ctx, Z, slot(ctx, SL_H), T, none(), nullptr, 1.0f, 0.0f, 0.0f, "ns_gemm", 0));
    GDM_TRY(gemm(ctx, T, Z, slot(ctx, SL_HP), none(), nullptr, 1.0f, 0.0f, 0.0f, "ns_gemm"));
    {
        GDM_TIMED(ctx, "mixed_misc");
        hipLaunchKernelGGL(k_sym_bounds, dim3(P.n_sub), dim3(kEw), 0, ctx->stream, desc, slot(ctx, SL_HP), bounds);
    }
    GDM_LAUNCH_CHECK(ctx);
    std::vector<double> hb(2 * (size_t)P.n_sub);
    GDM_HIP(ctx, hipMemcpyAsync(hb.data(), bounds, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double lo = INFINITY, hi = -INFINITY;
    for (int s = 0; s < P.n_sub; ++s) {
        lo = std::min(lo, hb[2 * s]);
        hi = std::max(hi, hb[2 * s + 1]);
    }
    if (!std::isfinite(lo) || !std::isfinite(hi)) return gdm_fail(ctx, GDM_E_NAN, "mixed: non-finite spectral bounds");
    // mu: safeguarded Newton steps on the FP64 traces (refined Z, count error
    // ~1e-7 N_e) until |N - N_e| <= max(tol_N, 1e-7 N_e).  Within that
    // resolution the count cannot place mu any better (inside a gap N'(mu) is
    // tiny), so the first-order correction mu* = mu + (N_e - N)/N'(mu) is only
    // applied when the pass budget ran out, and only within kT.
    double mu = std::isfinite(mu_guess) && mu_guess > lo && mu_guess < hi ? mu_guess : 0.5 * (lo + hi);
    double blo = lo, bhi = hi, N = 0.0, M = 0.0;
    int passes = 0, nd = 0;
    const double tol = std::max(tol_N, 1e-7 * n_e);
    for (;;) {
        GDM_TRY(foe_pass(ctx, mu, beta, lo, hi, &nd));
        GDM_TRY(traces(ctx, &N, &M));
        ++passes;
        const double dN = n_e - N;
        const double slope = beta * M;
        if (std::fabs(dN) <= tol || passes >= ctx->mixed_max_passes) break;
        if (dN > 0) blo = mu; else bhi = mu;
        // safeguarded Newton: the Newton point if it stays in the bracket and
        // shrinks it by at least half, else bisection
        double next = slope > 0.0 ? mu + dN / slope : 0.5 * (blo + bhi);
        if (!(next > blo && next < bhi) || std::fabs(next - mu) > 0.5 * (bhi - blo)) next = 0.5 * (blo + bhi);
        mu = next;
    }
    ctx->mixed_passes = passes;
    ctx->mixed_nd = nd;
    ctx->mixed_mu_pass = mu;
    ctx->mixed_slope = beta * M;
    // first-order correction mu* = mu + dmu, used only inside its linear range (|dmu| <= kT)
    double dmu = 0.0;
    if (std::fabs(n_e - N) > tol && beta * M > 0.0) {
        dmu = (n_e - N) / (beta * M);
        if (std::fabs(dmu) > kT) dmu = 0.0;
    }
    *mu_out = mu + dmu;
    *n_out = N + beta * M * dmu;
    return GDM_OK;
}

int gdm_mixed_density(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, double kT, double* D_core) {
    const Plan& P = ctx->plan;
    const double beta = 1.0 / kT;
    const double kappa = (mu - ctx->mixed_mu_pass) * beta;
    GDM_TIMED(ctx, "dcore");
    hipLaunchKernelGGL(k_dcore_mixed, dim3(P.n_sub), dim3(kEw), sizeof(double) * P.max_n, ctx->stream,
                       (const SubDesc*)ctx->b[BUF_DESC].p, z64(ctx), slot(ctx, SL_X).f, slot(ctx, SL_X2).f,
                       kappa, (double*)ctx->b[BUF_CC].p, D_core);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_set_mixed_options(gdm_ctx* ctx, int ns_z, int ns_inv, int max_passes) {
    if (!ctx) return GDM_E_ARG;
    if (ns_z > 64 || ns_inv > 16 || max_passes > 64)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_set_mixed_options: values out of range");
    if (ns_z > 0) ctx->mixed_ns_z = ns_z;
    if (ns_inv > 0) ctx->mixed_ns_inv = ns_inv;
    if (max_passes > 0) ctx->mixed_max_passes = max_passes;
    return GDM_OK;
}

extern "C" int gdm_mixed_stats(gdm_ctx* ctx, int* passes, int* n_doublings, int64_t* gemm_launches,
                               double* flops_per_launch) {
    if (!ctx) return GDM_E_ARG;
    if (passes) *passes = ctx->mixed_passes;
    if (n_doublings) *n_doublings = ctx->mixed_nd;
    if (gemm_launches) *gemm_launches = ctx->mixed_gemms;
    if (flops_per_launch) *flops_per_launch = ctx->mixed_gemms ? ctx->mixed_flops / (double)ctx->mixed_gemms : 0.0;
    return GDM_OK;
}

extern "C" int gdm_debug_slot(gdm_ctx* ctx, int which, int sub, float* out) {
    if (!ctx) return GDM_E_ARG;
    const Plan& P = ctx->plan;
    if (P.precision != GDM_MIXED_F16 || which < 0 || which >= SL_COUNT || sub < 0 || sub >= P.n_sub || !out)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_debug_slot: bad argument");
    const SubDesc& d = P.desc[sub];
    GDM_HIP(ctx, hipMemcpyAsync(out, slot(ctx, which).f + d.off2, sizeof(float) * (size_t)d.ld * d.ld,
                                hipMemcpyDeviceToDevice, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GDM_OK;
}
