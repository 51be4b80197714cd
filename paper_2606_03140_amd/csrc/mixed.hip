// Mixed-precision recursive Fermi-operator expansion (the "recursive
// Fermi-operator expansion" option of the paper's subgraph step, run on the
// matrix cores as the paper's accelerator library does for FOE and the
// inverse overlap).  Per subgraph, padded to P = 64 * ceil(n / 64):
//
//   Z = s^-1/2 by coupled Newton-Schulz on s/c (c the largest absolute row
//       sum of s): Z0 = kZ0a I + kZ0b s/c (linear minimax start), Y0 = (s/c) Z0,
//       T = (3I - Z Y)/2, Y <- Y T, Z <- T Z; then Z64 = Z / sqrt(c) in FP64
//       and one FP64 residual step Z64 <- Z64 - Z64 (Z64 s Z64 - I) / 2,
//   h_perp = Z h Z,
//   K = b (h_perp - mu I), b = beta / 2^n_d, and the start X0 = f_b(K) to
//       high order: the degree-7 odd polynomial of kStart7 (n_d >= 5), else
//       the cubic I/2 - K/4 + K^3/108, or the linear I/2 - K/4 when the pass is
//       recorded for the charge response,
//   n_d times:  X2 = X X,  A = 2 X2 - 2 X + I = X^2 + (I - X)^2,
//               Y = A^-1 by Newton-Schulz from the minimax quadratic start
//               Y0 = (420 I - 576 A + 256 A^2) / 99 (|I - A Y0| <= 1/99 on
//               [1/2, 1]), then ns_inv iterations,
//               X <- X2 Y            (f_b -> f_2b),
//   N(mu) = 2 sum_core (Z X Z s)_aa,  N'(mu) = 2 beta sum_core (Z (X - X^2) Z s)_aa
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
constexpr int kK = 64;          // k-step per LDS stage (two MFMA k-steps of 32)
constexpr int kLdsRow = kK + 8; // padded LDS row (halves): 144 B, conflict-free MFMA operand reads
constexpr int kGemmThreads = 256;
constexpr int kXcds = 8;        // workgroup b is dispatched to XCD b mod 8
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
    SplitMat E;          // read as f32 if present, else as hi + 2^-11 lo
    float alpha, beta, gamma;
    int sym;             // tiles cover i <= j only; results mirrored (the mirror is written from
                         // registers, so it can differ from the upper tile in the last bit)
    int packed;          // sym only.  Bit 0: the operands hold valid upper tiles only (a lower
                         // tile is read as its stored mirror, transposed into LDS).  Bit 1: the
                         // outputs are written on the upper tiles only (no mirror); E is then
                         // read on upper tiles only too, so it may be packed as well
};

__device__ __forceinline__ void store_split(SplitMat m, int64_t idx, float v) {
    if (m.f) m.f[idx] = v;
    if (m.hi) {
        _Float16 h = (_Float16)v;
        m.hi[idx] = h;
        m.lo[idx] = (_Float16)((v - (float)h) * kLoScale);
    }
}

// Tile list entries: (subgraph, tile row, tile col).  Each workgroup forms a
// 64 x 64 output tile with four waves (2 x 2 blocks of 32 x 32, each 2 x 2
// MFMA 16x16x32 tiles, three products per k-step).  Operands move through
// LDS in k-slabs of 64 (each thread carries two 16-byte row segments per
// operand array; a row segment of 128 B is read by 8 consecutive lanes); the
// next slab is prefetched into registers while the current one is
// multiplied.  The accumulator register r of lane l holds row 4 r + l / 16,
// column l % 16 of its 16 x 16 tile.  Epilogue: the tile is staged in LDS
// (row stride 68 floats: conflict-free writes from the accumulator layout and
// 16-byte row reads) and written as coalesced rows; in symmetric mode the
// mirror image of an off-diagonal tile is written straight from registers,
// where the accumulator layout already holds four consecutive elements of a
// mirrored row per lane.
constexpr int kOperandLds = 4 * kTile * kLdsRow * 2;        // bytes of the four operand tiles
constexpr int kOutRow = kTile + 4;                           // staged output row stride (floats)
constexpr int kOutLds = kTile * kOutRow * 4;                 // bytes of the staged output tile
constexpr int kGemmLds = kOperandLds > kOutLds ? kOperandLds : kOutLds;

typedef _Float16 half4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store4(SplitMat m, int64_t idx, float4 v) {
    if (m.f) *(float4*)(m.f + idx) = v;
    if (m.hi) {
        half4 h, l;
        const float x[4] = {v.x, v.y, v.z, v.w};
        for (int q = 0; q < 4; ++q) {
            const _Float16 hh = (_Float16)x[q];
            h[q] = hh;
            l[q] = (_Float16)((x[q] - (float)hh) * kLoScale);
        }
        *(half4*)(m.hi + idx) = h;
        *(half4*)(m.lo + idx) = l;
    }
}

// x = hi + 2^-11 lo for four consecutive elements
__device__ __forceinline__ float4 load4(SplitMat m, int64_t idx) {
    if (m.f) return *(const float4*)(m.f + idx);
    const half4 h = *(const half4*)(m.hi + idx);
    const half4 l = *(const half4*)(m.lo + idx);
    return make_float4((float)h[0] + kLoInv * (float)l[0], (float)h[1] + kLoInv * (float)l[1],
                       (float)h[2] + kLoInv * (float)l[2], (float)h[3] + kLoInv * (float)l[3]);
}

// Four waves per SIMD (four workgroups per CU, as the LDS allows): the
// register budget is held to 128 per lane (no spills).
__global__ void __launch_bounds__(kGemmThreads) __attribute__((amdgpu_waves_per_eu(4))) k_gemm_split(const SubDesc* __restrict__ desc,
                                                            const int4* __restrict__ tiles, GemmArgs g) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[kGemmLds];
    _Float16* sAh = (_Float16*)lds;
    _Float16* sAl = sAh + kTile * kLdsRow;
    _Float16* sBh = sAl + kTile * kLdsRow;
    _Float16* sBl = sBh + kTile * kLdsRow;
    float* sC = (float*)lds;                    // reused after the k loop: [64][kOutRow]
    const int4 tl = tiles[blockIdx.x];
    if (tl.x < 0) return;
    const SubDesc d = desc[tl.x];
    const int P = d.ld;
    const int64_t base = d.off2;
    const int m0 = tl.y * kTile, n0 = tl.z * kTile;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // global -> LDS: rows lr and lr + 32 of the slab, columns lc .. lc + 7
    const int lr = t >> 3, lc = (t & 7) * 8;
    const int64_t rA = base + (int64_t)(m0 + lr) * P + lc;
    const int64_t rB = base + (int64_t)(n0 + lr) * P + lc;
    const int64_t r32 = (int64_t)32 * P;
    float4v acc_hh[2][2], acc_x[2][2];
    #pragma unroll
    for (int i = 0; i < 2; ++i)
        #pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc_hh[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
            acc_x[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
        }
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    // LDS layout of an operand slab: element (r, c) (row r of the tile, k
    // column c) at r * kLdsRow + (c ^ sw(r)), sw(r) = 8 ((r / 8) mod 8): an
    // XOR of the 16-byte chunk index by the row's 8-row group.  Row-wise
    // 16-byte stores and the MFMA fragment reads (8 consecutive k of one row)
    // stay aligned and conflict-free, and the column-wise 2-byte stores of a
    // transposed slab spread over all banks instead of four.
    //
    // Slab k0 of the A panel (rows m0.., columns k0..) is a lower tile when
    // k0 < m0; in packed storage it is read from the stored upper tile (k0, m0)
    // instead: the thread's rows lr, lr + 32 of that tile hold columns lr,
    // lr + 32 of the wanted block, so its eight halves go to LDS column-wise.
    // The same for the B panel with n0.  Both choices are uniform per
    // workgroup, and every address stays inside the subgraph's P x P matrix.
    auto addr_a = [&](int k0) -> int64_t {
        return ((g.packed & 1) && k0 < m0) ? base + (int64_t)(k0 + lr) * P + m0 + lc : rA + k0;
    };
    auto addr_b = [&](int k0) -> int64_t {
        return ((g.packed & 1) && k0 < n0) ? base + (int64_t)(k0 + lr) * P + n0 + lc : rB + k0;
    };
    // row-wise stores: rows lr and lr + 32, chunk lc
    const int w0 = lr * kLdsRow + (lc ^ ((lr & 56))), w1 = (lr + 32) * kLdsRow + (lc ^ ((lr + 32) & 56));
    // column-wise stores: rows lc + q (one 8-row group, sw = lc), columns lr, lr + 32
    const int t0 = lc * kLdsRow + (lr ^ lc), t1 = lc * kLdsRow + ((lr + 32) ^ lc);
    auto store_t = [&](_Float16* dst, uint4 lo32, uint4 hi32) {
        unsigned short* d = (unsigned short*)dst;
        const unsigned a[4] = {lo32.x, lo32.y, lo32.z, lo32.w};
        const unsigned b[4] = {hi32.x, hi32.y, hi32.z, hi32.w};
        #pragma unroll
        for (int q = 0; q < 8; ++q) {
            const unsigned sh = (q & 1) * 16;
            d[t0 + q * kLdsRow] = (unsigned short)(a[q >> 1] >> sh);
            d[t1 + q * kLdsRow] = (unsigned short)(b[q >> 1] >> sh);
        }
    };
    uint4 v0, v1, v2, v3, v4, v5, v6, v7;
    {
        const int64_t a0 = addr_a(0), b0 = addr_b(0);
        v0 = *(const uint4*)(g.A.hi + a0);
        v1 = *(const uint4*)(g.A.hi + a0 + r32);
        v2 = *(const uint4*)(g.A.lo + a0);
        v3 = *(const uint4*)(g.A.lo + a0 + r32);
        v4 = *(const uint4*)(g.B.hi + b0);
        v5 = *(const uint4*)(g.B.hi + b0 + r32);
        v6 = *(const uint4*)(g.B.lo + b0);
        v7 = *(const uint4*)(g.B.lo + b0 + r32);
    }
    for (int k0 = 0; k0 < P; k0 += kK) {
        __syncthreads();
        if ((g.packed & 1) && k0 < m0) {
            store_t(sAh, v0, v1);
            store_t(sAl, v2, v3);
        } else {
            *(uint4*)(sAh + w0) = v0;
            *(uint4*)(sAh + w1) = v1;
            *(uint4*)(sAl + w0) = v2;
            *(uint4*)(sAl + w1) = v3;
        }
        if ((g.packed & 1) && k0 < n0) {
            store_t(sBh, v4, v5);
            store_t(sBl, v6, v7);
        } else {
            *(uint4*)(sBh + w0) = v4;
            *(uint4*)(sBh + w1) = v5;
            *(uint4*)(sBl + w0) = v6;
            *(uint4*)(sBl + w1) = v7;
        }
        __syncthreads();
        if (k0 + kK < P) {
            const int64_t a1 = addr_a(k0 + kK), b1 = addr_b(k0 + kK);
            v0 = *(const uint4*)(g.A.hi + a1);
            v1 = *(const uint4*)(g.A.hi + a1 + r32);
            v2 = *(const uint4*)(g.A.lo + a1);
            v3 = *(const uint4*)(g.A.lo + a1 + r32);
            v4 = *(const uint4*)(g.B.hi + b1);
            v5 = *(const uint4*)(g.B.hi + b1 + r32);
            v6 = *(const uint4*)(g.B.lo + b1);
            v7 = *(const uint4*)(g.B.lo + b1 + r32);
        }
        #pragma unroll
        for (int ks = 0; ks < kK; ks += 32) {
            half8 ah[2], al[2], bh[2], bl[2];
            #pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int r = wm * 32 + i * 16 + fr;
                ah[i] = *(const half8*)(sAh + r * kLdsRow + ((ks + fk) ^ (r & 56)));
                al[i] = *(const half8*)(sAl + r * kLdsRow + ((ks + fk) ^ (r & 56)));
            }
            #pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int c = wn * 32 + j * 16 + fr;
                bh[j] = *(const half8*)(sBh + c * kLdsRow + ((ks + fk) ^ (c & 56)));
                bl[j] = *(const half8*)(sBl + c * kLdsRow + ((ks + fk) ^ (c & 56)));
            }
            #pragma unroll
            for (int i = 0; i < 2; ++i)
                #pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc_hh[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc_hh[i][j], 0, 0, 0);
                    acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc_x[i][j], 0, 0, 0);
                    acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc_x[i][j], 0, 0, 0);
                }
        }
    }
    __syncthreads();
    const int gq = lane >> 4;                   // accumulator row group
    #pragma unroll
    for (int i = 0; i < 2; ++i)
        #pragma unroll
        for (int j = 0; j < 2; ++j)
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ml = wm * 32 + i * 16 + 4 * gq + r;
                const int nl = wn * 32 + j * 16 + fr;
                sC[ml * kOutRow + nl] = acc_hh[i][j][r] + kLoInv * acc_x[i][j][r];
            }
    __syncthreads();
    const bool diag_tile = tl.y == tl.z;
    const bool has_e = g.E.f || g.E.hi;
    const bool out1 = g.O1.f || g.O1.hi, out2 = g.O2.f || g.O2.hi;
    // rows of the tile, four floats per lane, 16 lanes per 64-wide row; in a
    // diagonal symmetric tile, (m, n) with m > n takes the value of (n, m)
    const int c4 = (t & 15) * 4;
    for (int rb = 0; rb < kTile; rb += kGemmThreads / 16) {
        const int rl = rb + (t >> 4);
        const float4 xv = *(const float4*)(sC + rl * kOutRow + c4);
        float x[4] = {xv.x, xv.y, xv.z, xv.w};
        if (g.sym && diag_tile)
            #pragma unroll
            for (int q = 0; q < 4; ++q)
                if (rl > c4 + q) x[q] = sC[(c4 + q) * kOutRow + rl];
        const int gm = m0 + rl, gn = n0 + c4;
        const int64_t idx = base + (int64_t)gm * P + gn;
        if (out1) store4(g.O1, idx, make_float4(x[0], x[1], x[2], x[3]));
        if (out2) {
            const float4 e = has_e ? load4(g.E, idx) : make_float4(0.f, 0.f, 0.f, 0.f);
            const float ev[4] = {e.x, e.y, e.z, e.w};
            float o[4];
            #pragma unroll
            for (int q = 0; q < 4; ++q) {
                o[q] = g.alpha * x[q] + g.beta * ev[q];
                if (gm == gn + q) o[q] += g.gamma;
            }
            store4(g.O2, idx, make_float4(o[0], o[1], o[2], o[3]));
        }
    }
    if (!g.sym || diag_tile || (g.packed & 2)) return;
    // mirror image of an off-diagonal tile from registers: register r of lane
    // l is element (4 gq + r, fr) of its 16 x 16 block, i.e. element
    // (fr, 4 gq + r) of the mirrored block: four consecutive columns of row fr
    #pragma unroll
    for (int i = 0; i < 2; ++i)
        #pragma unroll
        for (int j = 0; j < 2; ++j) {
            float x[4];
            #pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = acc_hh[i][j][r] + kLoInv * acc_x[i][j][r];
            const int gm = n0 + wn * 32 + j * 16 + fr;
            const int gn = m0 + wm * 32 + i * 16 + 4 * gq;
            const int64_t idx = base + (int64_t)gm * P + gn;
            if (out1) store4(g.O1, idx, make_float4(x[0], x[1], x[2], x[3]));
            if (out2) {
                const float4 e = has_e ? load4(g.E, idx) : make_float4(0.f, 0.f, 0.f, 0.f);
                store4(g.O2, idx, make_float4(g.alpha * x[0] + g.beta * e.x, g.alpha * x[1] + g.beta * e.y,
                                              g.alpha * x[2] + g.beta * e.z, g.alpha * x[3] + g.beta * e.w));
            }
        }
}

// ------------------------------------------------------------ FP64 GEMM
// C = alpha A B + beta Cin + gamma I on the padded P x P tiles, true product,
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  64 x 64 output tile per
// workgroup: four waves, each a 32 x 32 block of 2 x 2 MFMA tiles; k-steps of
// 16 staged in LDS (A row-major [m][k], B [k][n]).  Lane layout of the
// instruction (checked on the device): A lane l holds A[l % 16][l / 16], B
// lane l holds B[l / 16][l % 16], accumulator register r of lane l holds
// D[4 r + l / 16][l % 16].  TA / TB: double or float (converted when staged).
// SYM: the product is symmetric (Z s Z, and Z E of commuting factors):
// launched on the upper tiles only and written with its mirror, the lower
// half of a diagonal tile taken from its upper half, so C is exactly
// symmetric (Cin must then be symmetric too).
typedef double double4v __attribute__((ext_vector_type(4)));
// FP64 MFMA GEMM C = alpha A B + beta Cin + gamma I on 64 x 64 output tiles
// (four waves of 32 x 32, each 2 x 2 v_mfma_f64_16x16x4f64 blocks).  Operands
// stream through LDS in k-slabs of 32: each thread loads 8 consecutive
// elements of A and of B with 16-byte loads, and the next slab is held in
// registers while the current one is multiplied.  LDS rows are padded to 36
// (A) and 80 (B) doubles, so the operand reads of a wave (rows fr, k fk of
// A; k fk, columns fr of B) hit every bank exactly twice.  The tile is staged
// in LDS (row stride 65) and written as coalesced rows; SYM (products of
// commuting symmetric matrices, upper tiles only) also writes the mirror
// tile from the transposed LDS read, and on a diagonal tile takes both
// halves from the upper triangle, so C is exactly symmetric.
constexpr int kK64 = 32;
constexpr int kA64Row = kK64 + 4;        // doubles per LDS row of the A slab
constexpr int kB64Row = 64 + 16;         // doubles per LDS row of the B slab
constexpr int kC64Row = 64 + 1;          // doubles per LDS row of the staged tile
constexpr int kG64Lds = 64 * kA64Row + kK64 * kB64Row;    // doubles

__device__ __forceinline__ void load8(const double* p, double* v) {
    const double4 x = *(const double4*)p, y = *(const double4*)(p + 4);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w; v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
}
__device__ __forceinline__ void load8(const float* p, double* v) {
    const float4 x = *(const float4*)p, y = *(const float4*)(p + 4);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w; v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
}

template <typename TA, typename TB, bool SYM>
__global__ void __launch_bounds__(256) k_gemm64(const SubDesc* __restrict__ desc, const int4* __restrict__ tiles,
                                               const TA* __restrict__ A, const TB* __restrict__ B,
                                               const double* __restrict__ Cin, double* __restrict__ C,
                                               double alpha, double beta, double gamma) {
    __shared__ double lds[kG64Lds];
    double* sA = lds;                        // [64][kA64Row]
    double* sB = lds + 64 * kA64Row;         // [kK64][kB64Row]
    const int4 tl = tiles[blockIdx.x];
    if (tl.x < 0) return;
    const SubDesc d = desc[tl.x];
    const int P = d.ld;
    const int64_t base = d.off2;
    const int m0 = tl.y * 64, n0 = tl.z * 64;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int fr = lane & 15, fk = lane >> 4;
    // this thread's share of a slab: A row ra, columns ca..ca+7; B row rb, columns cb..cb+7
    const int ra = t >> 2, ca = (t & 3) * 8;
    const int rb = t >> 3, cb = (t & 7) * 8;
    const TA* pa = A + base + (int64_t)(m0 + ra) * P + ca;
    const TB* pb = B + base + (int64_t)rb * P + n0 + cb;
    double va[8], vb[8];
    load8(pa, va);
    load8(pb, vb);
    double4v acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = double4v{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < P; k0 += kK64) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            sA[ra * kA64Row + ca + q] = va[q];
            sB[rb * kB64Row + cb + q] = vb[q];
        }
        __syncthreads();
        if (k0 + kK64 < P) {
            load8(pa + k0 + kK64, va);
            load8(pb + (int64_t)(k0 + kK64) * P, vb);
        }
#pragma unroll
        for (int kk = 0; kk < kK64; kk += 4) {
            double a[2], b[2];
            for (int i = 0; i < 2; ++i) a[i] = sA[(wm * 32 + i * 16 + fr) * kA64Row + kk + fk];
            for (int j = 0; j < 2; ++j) b[j] = sB[(kk + fk) * kB64Row + wn * 32 + j * 16 + fr];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // stage the tile: accumulator register r of lane l is element (4 r + fk, fr)
    // of its 16 x 16 block
    __syncthreads();
    double* sC = lds;                        // [64][kC64Row]
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sC[(wm * 32 + i * 16 + 4 * r + fk) * kC64Row + wn * 32 + j * 16 + fr] = acc[i][j][r];
    __syncthreads();
    const bool diag = SYM && tl.y == tl.z;
    for (int e = t; e < 64 * 64; e += 256) {
        const int m = e >> 6, n = e & 63;
        // on a diagonal tile of a symmetric product both halves come from m <= n
        const double x = (diag && m > n) ? sC[n * kC64Row + m] : sC[m * kC64Row + n];
        const int64_t idx = base + (int64_t)(m0 + m) * P + n0 + n;
        double v = alpha * x;
        if (Cin) v += beta * Cin[idx];
        if (m0 + m == n0 + n) v += gamma;
        C[idx] = v;
    }
    if (SYM && !diag)
        for (int e = t; e < 64 * 64; e += 256) {
            const int nn = e >> 6, mm = e & 63;      // mirror tile row n0 + nn, column m0 + mm
            const int64_t idx = base + (int64_t)(n0 + nn) * P + m0 + mm;
            double v = alpha * sC[mm * kC64Row + nn];
            if (Cin) v += beta * Cin[idx];
            C[idx] = v;
        }
}

// Z (FP16 hi/lo split) <- Z64, flat over every packed tile (padding included)
__global__ void __launch_bounds__(256) k_z64_to_split(int64_t n4, const double* __restrict__ Z64, SplitMat Z) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n4; e += (int64_t)gridDim.x * 256) {
        const double4 v = *(const double4*)(Z64 + 4 * e);
        store4(Z, 4 * e, make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w));
    }
}

// N_s = 2 sum_{a<nc, c<n} G_ac V_ac,  M_s = 2 sum (G - G2)_ac V_ac   (FP64)
// with G = Z[core,:] X, G2 = Z[core,:] X^2, V = s[core,:] Z, so that
// sum_c G_ac V_ac = (Z X Z s)_aa, the core diagonal of D s.
__global__ void __launch_bounds__(256) k_trace_dot(const SubDesc* __restrict__ desc, const double* __restrict__ G,
                                                  const double* __restrict__ G2, const double* __restrict__ V,
                                                  double* __restrict__ part) {
    __shared__ double red[4];
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld, nc = d.nc;
    double an = 0.0, am = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)nc * n; e += 256) {
        const int a = (int)(e / n), c = (int)(e - (int64_t)a * n);
        const int64_t idx = d.off2 + (int64_t)a * P + c;
        const double g = G[idx], v = V[idx];
        an += g * v;
        am += (g - G2[idx]) * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        an += __shfl_xor(an, o, 64);
        am += __shfl_xor(am, o, 64);
    }
    __shared__ double red2[4];
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = an;
        red2[threadIdx.x >> 6] = am;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = 2.0 * (red[0] + red[1] + red[2] + red[3]);
        part[2 * blockIdx.x + 1] = 2.0 * (red2[0] + red2[1] + red2[2] + red2[3]);
    }
}

// Gk <- Base + kappa (G - G2) on the core rows: the first-order mu
// correction of Z X (Base = G), or the chemical-potential term of the
// canonical response (Base = Z dX); Gk may alias Base
__global__ void __launch_bounds__(256) k_combine(const SubDesc* __restrict__ desc, const double* Base,
                                                const double* __restrict__ G, const double* __restrict__ G2,
                                                double* Gk, double kappa) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld, nc = d.nc;
    const int rows = (nc + 63) / 64 * 64;
    for (int64_t e = threadIdx.x; e < (int64_t)rows * P; e += 256) {
        const int64_t idx = d.off2 + e;
        Gk[idx] = Base[idx] + kappa * (G[idx] - G2[idx]);
    }
}

// D_core (packed nc x n) <- rows of the P-strided product
__global__ void __launch_bounds__(256) k_pack_core(const SubDesc* __restrict__ desc, const double* __restrict__ Dp,
                                                  double* __restrict__ Dout) {
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld, nc = d.nc;
    for (int64_t e = threadIdx.x; e < (int64_t)nc * n; e += 256) {
        const int a = (int)(e / n), c = (int)(e - (int64_t)a * n);
        Dout[d.offd + e] = Dp[d.off2 + (int64_t)a * P + c];
    }
}

// ------------------------------------------------------- elementwise kernels
constexpr int kEw = 256;
constexpr double kZResidMax = 3e-3;   // largest |Z s Z - I| entry accepted before refinement

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

// The elementwise kernels below run on a (subgraph, 64-row strip) grid: block
// (x, y) covers rows 64y .. 64y+63 of subgraph x's padded P x P tile, four
// consecutive columns per thread and step (P is a multiple of 64).

// Gershgorin upper bound of s: max_i sum_j |s_ij| per subgraph, one wave per
// row; the maximum is combined with an unsigned atomic max on the bit pattern
// (order-preserving for non-negative doubles) into cbits, zeroed beforehand.
__global__ void __launch_bounds__(kEw) k_rowabs_max(const SubDesc* __restrict__ desc, const double* __restrict__ s64,
                                                   unsigned long long* __restrict__ cbits) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld, n = d.n, r0 = blockIdx.y * 64;
    if (r0 >= n) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r1 = min(r0 + 64, n);
    double m = 0.0;
    for (int r = r0 + wave; r < r1; r += kEw / 64) {
        const double* row = s64 + d.off2 + (int64_t)r * P;
        double acc = 0.0;
        for (int j = lane; j < n; j += 64) acc += fabs(row[j]);
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        m = fmax(m, acc);
    }
    if (lane == 0 && m > 0.0) atomicMax(&cbits[blockIdx.x], (unsigned long long)__double_as_longlong(m));
}

// Start of the coupled Newton-Schulz iteration for (s/c)^-1/2: Z0 = a I + b
// (s/c), the linear minimax approximation of x^-1/2 in the error measure
// |1 - x z(x)^2| on [0.1, 1] (error <= 0.417 there, against 1 - x for Z0 =
// I; x z^2 <= 1.42 on [0, 1], inside the iteration's convergence region).
constexpr float kZ0a = 2.598551f, kZ0b = -1.834840f;

// H = h, Y = s / c, Z0 = a I + b s / c as split operands (padding: identity
// for Y, a + b on Z's diagonal, zero for H; the FP64 tiles get h = 0, s = I
// there).  c = scale[sub] (the Gershgorin bound of s; 1 when s = I).  When
// s = I, Z0 = I with its FP32 copy, since Newton-Schulz is skipped then.
__global__ void __launch_bounds__(kEw) k_prep(const SubDesc* __restrict__ desc, double* __restrict__ h64,
                                             double* __restrict__ s64, SplitMat H, SplitMat Y, SplitMat Z,
                                             const double* __restrict__ scale, int orthogonal) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld, n = d.n, r0 = blockIdx.y * 64;
    if (r0 >= P) return;
    const float ic = orthogonal ? 1.f : (float)(1.0 / scale[blockIdx.x]);
    const int q4 = P >> 2;
    for (int e = threadIdx.x; e < 64 * q4; e += kEw) {
        const int i = r0 + e / q4, j0 = (e % q4) * 4;
        const int64_t idx = d.off2 + (int64_t)i * P + j0;
        float hv[4], yv[4], zv[4];
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + q;
            const bool in = i < n && j < n;
            const float id = i == j ? 1.f : 0.f;
            const float sv = in ? (orthogonal ? id : (float)s64[idx + q]) : id;
            hv[q] = in ? (float)h64[idx + q] : 0.f;
            yv[q] = in ? sv * ic : id;
            zv[q] = orthogonal ? id : kZ0a * id + kZ0b * yv[q];
            if (!in) {
                h64[idx + q] = 0.0;
                s64[idx + q] = id;
            }
        }
        store4(H, idx, make_float4(hv[0], hv[1], hv[2], hv[3]));
        store4(Y, idx, make_float4(yv[0], yv[1], yv[2], yv[3]));
        store4(Z, idx, make_float4(zv[0], zv[1], zv[2], zv[3]));
    }
}

// Z64 <- the Newton-Schulz Z / sqrt(c) in FP64 on the n x n block (padding
// copied: it stays the identity through the iteration)
__global__ void __launch_bounds__(kEw) k_scale_to_f64(const SubDesc* __restrict__ desc, const float* __restrict__ Zf,
                                                     const double* __restrict__ scale, int orthogonal,
                                                     double* __restrict__ Z64) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld, n = d.n, r0 = blockIdx.y * 64;
    if (r0 >= P) return;
    const double f = orthogonal ? 1.0 : 1.0 / sqrt(scale[blockIdx.x]);
    const int q4 = P >> 2;
    for (int e = threadIdx.x; e < 64 * q4; e += kEw) {
        const int i = r0 + e / q4, j0 = (e % q4) * 4;
        const int64_t idx = d.off2 + (int64_t)i * P + j0;
        const float4 z = *(const float4*)(Zf + idx);
        const double zs[4] = {z.x, z.y, z.z, z.w};
        double o[4];
        for (int q = 0; q < 4; ++q) o[q] = (i < n && j0 + q < n) ? zs[q] * f : zs[q];
        *(double4*)(Z64 + idx) = make_double4(o[0], o[1], o[2], o[3]);
    }
}

// Gershgorin bounds of h_perp in FP64 over the rows of one 64-row strip of
// one subgraph -> bounds[2 (s strips + strip) + {0, 1}] (+inf / -inf for a
// strip past the last row); h_perp comes out of the symmetric-mode product
// exactly symmetric.  One wave per row.
__global__ void __launch_bounds__(kEw) k_sym_bounds(const SubDesc* __restrict__ desc, SplitMat H, int strips,
                                                   double* __restrict__ bounds) {
    __shared__ double red[kEw / 64];
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld, r0 = blockIdx.y * 64;
    const int r1 = min(r0 + 64, n);
    const int64_t base = d.off2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double lo = INFINITY, hi = -INFINITY;
    for (int i = r0 + wave; i < r1; i += kEw / 64) {
        const float* row = H.f + base + (int64_t)i * P;
        double r = 0.0;
        for (int j = lane; j < n; j += 64)
            if (j != i) r += fabs((double)row[j]);
        for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
        const double dii = (double)row[i];
        lo = fmin(lo, dii - r);
        hi = fmax(hi, dii + r);
    }
    lo = block_reduce_min(lo, red);
    hi = block_reduce_max(hi, red);
    if (threadIdx.x == 0) {
        const int64_t k = 2 * ((int64_t)blockIdx.x * strips + blockIdx.y);
        bounds[k] = lo;
        bounds[k + 1] = hi;
    }
}

// X <- c0 I - q (H - mu I) on the n x n block, zero padding (the linear start
// X0 = I/2 - (b/4)(H - mu I), or K = b (H - mu I) for the cubic start)
__global__ void __launch_bounds__(kEw) k_x0(const SubDesc* __restrict__ desc, const float* __restrict__ Hf,
                                           SplitMat X, double mu, double q, double c0) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld, n = d.n, r0 = blockIdx.y * 64;
    if (r0 >= P) return;
    const int q4 = P >> 2;
    for (int e = threadIdx.x; e < 64 * q4; e += kEw) {
        const int i = r0 + e / q4, j0 = (e % q4) * 4;
        const int64_t idx = d.off2 + (int64_t)i * P + j0;
        const float4 h = *(const float4*)(Hf + idx);
        const float hs[4] = {h.x, h.y, h.z, h.w};
        float v[4];
        for (int k = 0; k < 4; ++k) {
            const int j = j0 + k;
            v[k] = (i < n && j < n) ? (float)((i == j ? c0 : 0.0) - q * ((double)hs[k] - (i == j ? mu : 0.0))) : 0.f;
        }
        store4(X, idx, make_float4(v[0], v[1], v[2], v[3]));
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

// Largest |E_ij| = |(Z s Z - I)_ij| over every subgraph's n x n block, as an
// atomic max on the bit pattern (non-negative doubles order as integers; NaN
// counts as infinite).
__global__ void __launch_bounds__(kEw) k_resid_max(const SubDesc* __restrict__ desc, const double* __restrict__ E,
                                                  unsigned long long* __restrict__ out) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld, n = d.n, r0 = blockIdx.y * 64;
    if (r0 >= n) return;
    double m = 0.0;
    for (int e = threadIdx.x; e < 64 * P; e += kEw) {
        const int i = r0 + e / P, j = e % P;
        if (i < n && j < n) {
            const double v = fabs(E[d.off2 + (int64_t)i * P + j]);
            m = v == v ? fmax(m, v) : INFINITY;
        }
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// ------------------------------------------------------- charge response
// Potential change of every subgraph orbital, dv[offv + a] = dV[atom of a]
// (atoms in subgraph order, orbital counts from orb_ptr); 0 on the padding.
__global__ void __launch_bounds__(64) k_orb_dv(const SubDesc* __restrict__ desc, const int32_t* __restrict__ atoms_all,
                                               const int32_t* __restrict__ orb_ptr, const double* __restrict__ dV,
                                               double* __restrict__ dv) {
    const SubDesc d = desc[blockIdx.x];
    const int lane = threadIdx.x;
    double* out = dv + d.offv;
    int run = 0;
    for (int base = 0; base < d.natoms; base += 64) {
        const int i = base + lane;
        const int g = i < d.natoms ? atoms_all[d.atom0 + i] : 0;
        const int no = i < d.natoms ? orb_ptr[g + 1] - orb_ptr[g] : 0;
        int incl = no;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        const double v = i < d.natoms ? dV[g] : 0.0;
        for (int t = 0; t < no; ++t) {
            const int a = run + incl - no + t;
            if (a < d.ld) out[a] = v;
        }
        run += __shfl(incl, 63, 64);
    }
    for (int a = d.n + lane; a < d.ld; a += 64) out[a] = 0.0;
}

// dh_ab = 1/2 s_ab (dv_a + dv_b), the change of the SCC shift (s is the
// identity for an orthogonal model); 0 on the padding
__global__ void __launch_bounds__(kEw) k_dh(const SubDesc* __restrict__ desc, const double* __restrict__ S64,
                                           const double* __restrict__ dv, SplitMat out) {
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld, n = d.n, r0 = blockIdx.y * 64;
    if (r0 >= P) return;
    const double* v = dv + d.offv;
    const int q4 = P >> 2;
    for (int e = threadIdx.x; e < 64 * q4; e += kEw) {
        const int i = r0 + e / q4, j0 = (e % q4) * 4;
        const int64_t idx = d.off2 + (int64_t)i * P + j0;
        float w[4];
        for (int k = 0; k < 4; ++k) {
            const int j = j0 + k;
            w[k] = (i < n && j < n) ? (float)(0.5 * S64[idx + k] * (v[i] + v[j])) : 0.f;
        }
        store4(out, idx, make_float4(w[0], w[1], w[2], w[3]));
    }
}

// On the tile pair (I, J), (J, I) of an upper-tile list entry (I <= J):
// dX2 = Pm + Pm^T and Dl = dX - dX2, both tiles of Pm staged in LDS
// (row stride 65 floats: the transposed reads hit distinct banks).
__global__ void __launch_bounds__(256) k_sym_pair(const SubDesc* __restrict__ desc, const int4* __restrict__ tiles,
                                                 SplitMat Pm, SplitMat dX, SplitMat dX2, SplitMat Dl) {
    __shared__ float a[64][65];
    __shared__ float b[64][65];
    const int4 tl = tiles[blockIdx.x];
    if (tl.x < 0) return;
    const SubDesc d = desc[tl.x];
    const int P = d.ld;
    const int I0 = tl.y * 64, J0 = tl.z * 64;
    const int t = threadIdx.x;
    for (int e = t; e < 64 * 16; e += 256) {
        const int r = e >> 4, c = (e & 15) * 4;
        const float4 x = load4(Pm, d.off2 + (int64_t)(I0 + r) * P + J0 + c);
        const float4 y = load4(Pm, d.off2 + (int64_t)(J0 + r) * P + I0 + c);
        a[r][c] = x.x; a[r][c + 1] = x.y; a[r][c + 2] = x.z; a[r][c + 3] = x.w;
        b[r][c] = y.x; b[r][c + 1] = y.y; b[r][c + 2] = y.z; b[r][c + 3] = y.w;
    }
    __syncthreads();
    for (int e = t; e < 64 * 16; e += 256) {
        const int r = e >> 4, c = (e & 15) * 4;
        float s1[4], s2[4];
        for (int k = 0; k < 4; ++k) {
            s1[k] = a[r][c + k] + b[c + k][r];
            s2[k] = b[r][c + k] + a[c + k][r];
        }
        const int64_t i1 = d.off2 + (int64_t)(I0 + r) * P + J0 + c;
        const float4 x1 = load4(dX, i1);
        store4(dX2, i1, make_float4(s1[0], s1[1], s1[2], s1[3]));
        store4(Dl, i1, make_float4(x1.x - s1[0], x1.y - s1[1], x1.z - s1[2], x1.w - s1[3]));
        if (I0 != J0) {
            const int64_t i2 = d.off2 + (int64_t)(J0 + r) * P + I0 + c;
            const float4 x2 = load4(dX, i2);
            store4(dX2, i2, make_float4(s2[0], s2[1], s2[2], s2[3]));
            store4(Dl, i2, make_float4(x2.x - s2[0], x2.y - s2[1], x2.z - s2[2], x2.w - s2[3]));
        }
    }
}

}  // namespace

// --------------------------------------------------------------------- host

enum { SL_H = 0, SL_Y, SL_Z, SL_T, SL_Y2, SL_Z2, SL_HP, SL_X, SL_X2, SL_A, SL_R, SL_YI, SL_COUNT };

// Every slot holds the FP16 hi/lo split; only the matrices read back in FP32
// (the inverse-overlap factor and its Newton-Schulz partner, h_perp and X)
// also keep an FP32 copy.  Slots without one have f = nullptr, which every
// writer skips.
constexpr int kF32Slots = 4;
static int f32_index(int k) {
    switch (k) {
        case SL_Z: return 0;
        case SL_Z2: return 1;
        case SL_HP: return 2;
        case SL_X: return 3;
        default: return -1;
    }
}

static SplitMat slot(gdm_ctx* ctx, int k) {
    const int64_t tot = ctx->plan.tot2;
    const int fi = f32_index(k);
    float* f = fi < 0 ? nullptr : (float*)ctx->b[BUF_X_F].p + (int64_t)fi * tot;
    _Float16* hi = (_Float16*)ctx->b[BUF_X_HI].p + (int64_t)k * tot;
    _Float16* lo = (_Float16*)ctx->b[BUF_X_LO].p + (int64_t)k * tot;
    return SplitMat{f, hi, lo};
}

static SplitMat none() { return SplitMat{nullptr, nullptr, nullptr}; }

#define GDM_TRY(x)          \
    do {                    \
        int rc_ = (x);      \
        if (rc_) return rc_; \
    } while (0)

// (subgraph, 64-row strip) grid of the elementwise kernels
static dim3 strip_grid(const Plan& P) { return dim3((unsigned)P.n_sub, (unsigned)((P.max_n + 63) / 64)); }

int gdm_mixed_plan(gdm_ctx* ctx) {
    Plan& P = ctx->plan;
    // tiles in decreasing subgraph size order (long subgraphs first)
    std::vector<int> order(P.n_sub);
    for (int s = 0; s < P.n_sub; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.n[a] > P.n[b]; });
    // XCD-aware tile lists: workgroup b runs on XCD b mod 8, so each subgraph is
    // assigned to one of 8 queues (largest first, to the least loaded queue) and
    // position 8k + x of a list holds the k-th tile of queue x.  All tiles of a
    // subgraph then share one XCD's L2 and reuse its panels; queues are padded
    // with empty entries (x = -1) that exit at once.
    auto build = [&](int mode, double* flops) {
        std::vector<std::vector<int4>> q(kXcds);
        std::vector<double> load(kXcds, 0.0);
        *flops = 0.0;
        for (int s : order) {
            const int nt = P.desc[s].ld / kTile;
            const int nr = mode == 2 ? (P.desc[s].nc + kTile - 1) / kTile : nt;
            const double pt = 2.0 * kTile * kTile * (double)P.desc[s].ld;
            int x = 0;
            for (int k = 1; k < kXcds; ++k)
                if (load[k] < load[x]) x = k;
            for (int i = 0; i < nr; ++i)
                for (int j = 0; j < nt; ++j) {
                    if (mode == 1 && i > j) continue;
                    q[x].push_back(make_int4(s, i, j, 0));
                    load[x] += pt;
                    *flops += pt;
                }
        }
        size_t len = 0;
        for (auto& v : q) len = std::max(len, v.size());
        std::vector<int4> out(len * kXcds, make_int4(-1, 0, 0, 0));
        for (int x = 0; x < kXcds; ++x)
            for (size_t k = 0; k < q[x].size(); ++k) out[k * kXcds + x] = q[x][k];
        return out;
    };
    double ffull, fsym, fcore;
    std::vector<int4> tiles = build(0, &ffull);
    std::vector<int4> utiles = build(1, &fsym);
    std::vector<int4> ctiles = build(2, &fcore);
    const size_t nfull = tiles.size();
    tiles.insert(tiles.end(), utiles.begin(), utiles.end());
    tiles.insert(tiles.end(), ctiles.begin(), ctiles.end());
    bool ok = true;
    int4* dt = (int4*)gdm_buf(ctx, BUF_TILES, sizeof(int4) * tiles.size(), &ok);
    gdm_buf(ctx, BUF_A, sizeof(double) * P.tot2, &ok);
    gdm_buf(ctx, BUF_S, sizeof(double) * P.tot2, &ok);
    gdm_buf(ctx, BUF_X_F, sizeof(float) * P.tot2 * kF32Slots, &ok);
    gdm_buf(ctx, BUF_X_HI, sizeof(_Float16) * P.tot2 * SL_COUNT, &ok);
    gdm_buf(ctx, BUF_X_LO, sizeof(_Float16) * P.tot2 * SL_COUNT, &ok);
    gdm_buf(ctx, BUF_GERSH, sizeof(double) * 2 * (size_t)P.n_sub * strip_grid(P).y, &ok);
    gdm_buf(ctx, BUF_TR, sizeof(double) * (2 * (size_t)P.n_sub + 8), &ok);
    gdm_buf(ctx, BUF_NDBL, sizeof(double) * (size_t)P.n_sub, &ok);
    gdm_buf(ctx, BUF_CC, sizeof(double) * (size_t)P.totc, &ok);
    gdm_buf(ctx, BUF_L, sizeof(double) * P.tot2 * 5, &ok);     // F/V, E/G, Z64, G2, D (FP64)
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_plan: mixed workspace allocation failed");
    GDM_TRY(gdm_mixed_response_alloc(ctx));
    GDM_HIP(ctx, hipMemcpyAsync(dt, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, ctx->stream));
    ctx->mixed_tiles = (int64_t)nfull;
    ctx->mixed_tiles_sym = (int64_t)utiles.size();
    ctx->mixed_tiles_core = (int64_t)ctiles.size();
    ctx->mixed_upper_elems = 0;
    for (const SubDesc& d : P.desc) {
        const int64_t t = d.ld / kTile;
        ctx->mixed_upper_elems += t * (t + 1) / 2 * kTile * kTile;
    }
    ctx->mixed_flops_full = ffull;
    ctx->mixed_flops_sym = fsym;
    return GDM_OK;
}

// C = A B for symmetric B (read row-major as B^T).  sym = 1 when A and B
// commute (products of polynomials in the same matrix): only upper tiles are
// computed and mirrored.
static SplitMat hl(SplitMat m) { return SplitMat{nullptr, m.hi, m.lo}; }

static int gemm(gdm_ctx* ctx, SplitMat A, SplitMat B, SplitMat O1, SplitMat O2, SplitMat E, float alpha,
                float beta, float gamma, const char* tag, int sym = 1, int packed = 0) {
    // packed: bit 0 operands in upper-tile storage, bit 1 outputs (and E) on
    // upper tiles only; symmetric products only
    if (!sym) packed = 0;
    GemmArgs g{A, B, O1, O2, E, alpha, beta, gamma, sym, packed};
    const int4* tl = (const int4*)ctx->b[BUF_TILES].p + (sym ? ctx->mixed_tiles : 0);
    const int64_t nt = sym ? ctx->mixed_tiles_sym : ctx->mixed_tiles;
    GDM_TIMED(ctx, tag);
    hipLaunchKernelGGL(k_gemm_split, dim3((unsigned)nt), dim3(kGemmThreads), 0, ctx->stream,
                       (const SubDesc*)ctx->b[BUF_DESC].p, tl, g);
    GDM_LAUNCH_CHECK(ctx);
    ctx->mixed_gemms += 1;
    ctx->mixed_flops += sym ? ctx->mixed_flops_sym : ctx->mixed_flops_full;
    // algorithmic HBM bytes: each operand and E read once, each output written
    // once, over all elements, or over the upper tiles only in packed storage
    const double full = (double)ctx->plan.tot2, upper = (double)ctx->mixed_upper_elems;
    const double ein = (packed & 1) ? upper : full, eout = (packed & 2) ? upper : full;
    double bytes = 8.0 * ein;                           // A and B as FP16 hi + lo
    if (E.f || E.hi) bytes += 4.0 * eout;
    for (const SplitMat* o : {&O1, &O2}) {
        if (o->f) bytes += 4.0 * eout;
        if (o->hi) bytes += 4.0 * eout;
    }
    ctx->mixed_bytes += bytes;
    return GDM_OK;
}

// Coefficients a3, a5, a7 of the degree-7 start X0 = 1/2 - K/4 + a3 K^3 +
// a5 K^5 + a7 K^7 of the expansion, K = b (h - mu I) with |K| <= 8: chosen
// (minimax, numerically) so that after n_d >= 5 doublings the occupations
// f(2^n_d u0(K)), u0 = log((1 - X0) / X0), differ from f(2^n_d K) by at most
// 6.1e-8 over the whole range, with X0 in (0, 1/2) for K in (0, 8] (odd
// about 1/2).  a3 is close to the Taylor value 1/48 of the Fermi function,
// which keeps the states near mu exact to high order; the start is not
// monotone in K, which the doublings do not need.
static constexpr float kStart7[3] = {0.0208103713f, -0.000615022611f, 5.41684949e-06f};

// Doubling history for the charge response: X_k (which = 0), the input of
// doubling k, and Y_k (which = 1), its inverse (2 X_k^2 - 2 X_k + I)^-1, as
// FP16 hi/lo pairs.
static SplitMat hist(gdm_ctx* ctx, int k, int which) {
    const int64_t off = (int64_t)(2 * k + which) * ctx->plan.tot2;
    return SplitMat{nullptr, (_Float16*)ctx->b[BUF_HIST_HI].p + off, (_Float16*)ctx->b[BUF_HIST_LO].p + off};
}

// One full recursive expansion at chemical potential mu; leaves X (with its
// FP32 copy) in SL_X.  With a history buffer large enough for the nd doublings,
// every X_k and Y_k is kept there (the products write into the history in
// place of the working slots, so recording adds no traffic).
static int foe_pass(gdm_ctx* ctx, double mu, double beta, double lo, double hi, int* nd_out) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    // Each doubling maps X = f(u) to f(2u) (f the Fermi function), so n_d
    // doublings from X0 = f(u0) give f(2^n_d u0), and u0 must be b (h - mu),
    // b = beta / 2^n_d, to first order near mu, with X0's spectrum in [0, 1].
    // The linear start X0 = I/2 - (b/4)(h - mu I) needs b R <= 2 (R the
    // spectral half-width about mu); the cubic start with K = b (h - mu I),
    // X0 = I/2 - K/4 + K^3/108, stays in [0, 1] for b R <= 4 (its minimum, 0,
    // is at K = +-3), which saves one doubling (7 products) for 2.  The
    // response differentiates the linear start, so a recorded pass uses it.
    const double R = std::max(std::fabs(lo - mu), std::fabs(hi - mu));
    const bool rec_wanted = ctx->mixed_rec_cap > 0;
    // The degree-7 start of kStart7 reaches b R <= 8 (one doubling fewer than
    // the cubic for two more products) but is tuned for at least 5 doublings:
    // states near |K| = 8 start well inside (0, 1/2) and need them to settle.
    const int nd7 = (int)std::ceil(std::log2(0.125 * beta * R));
    const bool septic = !rec_wanted && nd7 >= 5;
    const bool cubic = !rec_wanted && !septic;
    int nd = septic ? nd7 : (int)std::ceil(std::log2((cubic ? 0.25 : 0.5) * beta * R));
    nd = std::max(1, std::min(nd, 40));
    const double b = beta / std::ldexp(1.0, nd);
    *nd_out = nd;
    const bool rec = ctx->mixed_rec_cap >= nd;
    ctx->mixed_rec_nd = -1;
    ctx->mixed_x0_slope = b / 4.0;
    SplitMat X = slot(ctx, SL_X), X2 = slot(ctx, SL_X2), A = slot(ctx, SL_A), Rm = slot(ctx, SL_R);
    const SplitMat Ya = slot(ctx, SL_Y), Yb = slot(ctx, SL_YI);
    // upper-tile storage of the pass's symmetric matrices (not when recording:
    // the response reads the recorded X_k, Y_k whole)
    const int pk = (!rec && ctx->mixed_packed) ? 3 : 0;
    if (septic || cubic) {
        const SplitMat K = slot(ctx, SL_T);
        {
            GDM_TIMED(ctx, "mixed_misc");
            hipLaunchKernelGGL(k_x0, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, slot(ctx, SL_HP).f, hl(K), mu, -b,
                               0.0);
        }
        GDM_LAUNCH_CHECK(ctx);
        if (septic) {
            // X0 = I/2 - K/4 + K (K^2 (K^2 (a7 K^2 + a5 I) + a3 I)), four products
            GDM_TRY(gemm(ctx, K, K, hl(Rm), hl(A), none(), kStart7[2], 0.0f, kStart7[1], "foe_gemm", 1, pk));
            GDM_TRY(gemm(ctx, Rm, A, none(), hl(Ya), none(), 1.0f, 0.0f, kStart7[0], "foe_gemm", 1, pk));
            GDM_TRY(gemm(ctx, Rm, Ya, hl(Yb), none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, pk));
            GDM_TRY(gemm(ctx, K, Yb, none(), hl(X), hl(K), 1.0f, -0.25f, 0.5f, "foe_gemm", 1, pk));
        } else {
            GDM_TRY(gemm(ctx, K, K, hl(Rm), none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, pk));
            GDM_TRY(gemm(ctx, K, Rm, none(), hl(X), hl(K), 1.0f / 108.0f, -0.25f, 0.5f, "foe_gemm", 1, pk));
        }
    } else {
        GDM_TIMED(ctx, "mixed_misc");
        hipLaunchKernelGGL(k_x0, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, slot(ctx, SL_HP).f,
                           rec ? hist(ctx, 0, 0) : X, mu, b / 4.0, 0.5);
    }
    GDM_LAUNCH_CHECK(ctx);
    const int ns = ctx->mixed_ns_inv;
    for (int it = 0; it < nd; ++it) {
        const SplitMat Xk = rec ? hist(ctx, it, 0) : X;
        // X2 = X X ; A = 2 X2 - 2 X + I
        GDM_TRY(gemm(ctx, Xk, Xk, hl(X2), hl(A), hl(Xk), 2.0f, -2.0f, 1.0f, "foe_gemm", 1, pk));
        // Newton-Schulz inverse of A (eigenvalues in [1/2, 1]) from the minimax
        // quadratic start Y0 = (420 I - 576 A + 256 A^2) / 99: 1 - a y0(a) is the
        // Chebyshev T3 on [1/2, 1] scaled to 1 at a = 0, so |1 - a y0| <= 1/99;
        // each iteration R = 2I - A Y, Y <- Y R squares the error
        SplitMat Y = (rec && ns == 0) ? hist(ctx, it, 1) : Ya;
        GDM_TRY(gemm(ctx, A, A, none(), hl(Y), hl(A), 256.0f / 99.0f, -576.0f / 99.0f, 420.0f / 99.0f, "foe_gemm", 1,
                     pk));
        for (int k = 0; k < ns; ++k) {
            GDM_TRY(gemm(ctx, A, Y, none(), hl(Rm), none(), -1.0f, 0.0f, 2.0f, "foe_gemm", 1, pk));
            const SplitMat Yn = (rec && k == ns - 1) ? hist(ctx, it, 1) : (Y.hi == Ya.hi ? Yb : Ya);
            GDM_TRY(gemm(ctx, Y, Rm, hl(Yn), none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, pk));
            Y = Yn;
        }
        // X <- X2 Y
        const SplitMat Xn = it + 1 == nd ? X : (rec ? hist(ctx, it + 1, 0) : hl(X));
        // the last product writes X whole (its FP32 copy is read by full rows)
        GDM_TRY(gemm(ctx, X2, Y, Xn, none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, it + 1 == nd ? (pk & 1) : pk));
    }
    if (rec) ctx->mixed_rec_nd = nd;
    return GDM_OK;
}

static double* z64(gdm_ctx* ctx) { return (double*)ctx->b[BUF_L].p + 2 * ctx->plan.tot2; }

// FP64 products on all tiles (sym = 0) or on the upper tiles with mirrored
// output (sym = 1, symmetric products only)
static int gemm64_dd(gdm_ctx* ctx, const double* A, const double* B, const double* Cin, double* C, double alpha,
                     double beta, double gamma, int sym) {
    GDM_TIMED(ctx, "refine64");
    const int4* tl = (const int4*)ctx->b[BUF_TILES].p + (sym ? ctx->mixed_tiles : 0);
    const unsigned nt = (unsigned)(sym ? ctx->mixed_tiles_sym : ctx->mixed_tiles);
    if (sym)
        hipLaunchKernelGGL((k_gemm64<double, double, true>), dim3(nt), dim3(256), 0, ctx->stream,
                           (const SubDesc*)ctx->b[BUF_DESC].p, tl, A, B, Cin, C, alpha, beta, gamma);
    else
        hipLaunchKernelGGL((k_gemm64<double, double, false>), dim3(nt), dim3(256), 0, ctx->stream,
                           (const SubDesc*)ctx->b[BUF_DESC].p, tl, A, B, Cin, C, alpha, beta, gamma);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

template <typename TB>
static int gemm64_core(gdm_ctx* ctx, const double* A, const TB* B, double* C, const char* tag) {
    GDM_TIMED(ctx, tag);
    const int4* tl = (const int4*)ctx->b[BUF_TILES].p + ctx->mixed_tiles + ctx->mixed_tiles_sym;
    hipLaunchKernelGGL((k_gemm64<double, TB, false>), dim3((unsigned)ctx->mixed_tiles_core), dim3(256), 0, ctx->stream,
                       (const SubDesc*)ctx->b[BUF_DESC].p, tl, A, B, (const double*)nullptr, C, 1.0, 0.0, 0.0);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

static double* fp64_region(gdm_ctx* ctx, int k) { return (double*)ctx->b[BUF_L].p + (int64_t)k * ctx->plan.tot2; }

static int traces(gdm_ctx* ctx, double* N, double* M) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    double* part = (double*)ctx->b[BUF_TR].p;
    double* G = fp64_region(ctx, 1);
    double* G2 = fp64_region(ctx, 3);
    double* V = fp64_region(ctx, 0);
    GDM_TRY(gemm64_core<float>(ctx, z64(ctx), slot(ctx, SL_X).f, G, "traces"));
    GDM_TRY(gemm64_core<float>(ctx, G, slot(ctx, SL_X).f, G2, "traces"));     // Z[core,:] X^2 = G X
    {
        GDM_TIMED(ctx, "traces");
        hipLaunchKernelGGL(k_trace_dot, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, G, G2, V, part);
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
    ctx->mixed_bytes = 0.0;
    ctx->mixed_rec_nd = -1;
    ctx->resp_v_ready = false;
    GDM_TRY(gdm_launch_gather(ctx, sys, sg, row_ptr, col, nnz, H, S, h64, s64, orth));
    {
        GDM_TIMED(ctx, "mixed_misc");
        GDM_TRY(gdm_fill_f64(ctx, scale, P.n_sub, 0.0));
        if (!orth) {
            hipLaunchKernelGGL(k_rowabs_max, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, s64,
                               (unsigned long long*)scale);
            GDM_LAUNCH_CHECK(ctx);
        }
        hipLaunchKernelGGL(k_prep, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, h64, s64, hl(slot(ctx, SL_H)),
                           hl(slot(ctx, SL_Y)), orth ? slot(ctx, SL_Z) : hl(slot(ctx, SL_Z)), scale, orth);
    }
    GDM_LAUNCH_CHECK(ctx);
    // coupled Newton-Schulz: Z -> (s/c)^-1/2, ns_z iterations, then more (at
    // most mixed_ns_z_extra) while the residual before refinement is too large
    // for one refinement step to remove
    SplitMat Y = slot(ctx, SL_Y), Z = slot(ctx, SL_Z), T = slot(ctx, SL_T), Y2 = slot(ctx, SL_Y2),
             Z2 = slot(ctx, SL_Z2);
    // upper-tile storage for these symmetric products too, except the Z that
    // the FP64 refinement reads whole (with its FP32 copy)
    const int pkz = ctx->mixed_packed ? 3 : 0;
    auto ns_step = [&](bool full_z) -> int {
        GDM_TRY(gemm(ctx, Z, Y, none(), hl(T), none(), -0.5f, 0.0f, 1.5f, "ns_gemm", 1, pkz));
        GDM_TRY(gemm(ctx, Y, T, hl(Y2), none(), none(), 1.0f, 0.0f, 0.0f, "ns_gemm", 1, pkz));
        GDM_TRY(gemm(ctx, T, Z, full_z ? Z2 : hl(Z2), none(), none(), 1.0f, 0.0f, 0.0f, "ns_gemm", 1,
                     full_z ? (pkz & 1) : pkz));
        std::swap(Y, Y2);
        std::swap(Z, Z2);
        return GDM_OK;
    };
    if (!orth) {
        // Y0 = (s/c) Z0 = a (s/c) + b (s/c)^2 (Z0 from k_prep)
        GDM_TRY(gemm(ctx, Y, Y, none(), hl(Y2), hl(Y), kZ0b, kZ0a, 0.0f, "ns_gemm", 1, pkz));
        std::swap(Y, Y2);
        for (int it = 0; it < ctx->mixed_ns_z; ++it) GDM_TRY(ns_step(it + 1 == ctx->mixed_ns_z));
    }
    ctx->mixed_ns_z_used = orth ? 0 : ctx->mixed_ns_z;
    // FP64 residual refinement of Z (Z s Z = I): Z64 = Z / sqrt(c) in FP64,
    // F = s Z64, E = Z64 F - I, Z64 <- Z64 - Z64 E / 2 (error O(E^2)); E and
    // the update are symmetric products (upper tiles, mirrored).  The
    // refinement also removes any systematic bias of the split products from
    // Z64, which the electron count (and so mu) depends on.  While max |E_ij|
    // is too large for one step, the coupled iteration continues first.
    // Z64 serves the traces and the final step, its split copy (in SL_Z) the
    // expansion.
    {
        double* F = fp64_region(ctx, 0);
        double* E = fp64_region(ctx, 1);
        double* Z64 = z64(ctx);
        double* emax_d = (double*)ctx->b[BUF_TR].p + 2 * (size_t)P.n_sub + 4;
        for (int extra = 0;; ++extra) {
            {
                GDM_TIMED(ctx, "refine64");
                hipLaunchKernelGGL(k_scale_to_f64, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, Z.f, scale, orth,
                                   Z64);
            }
            GDM_LAUNCH_CHECK(ctx);
            if (orth) break;                                                  // Z = I exactly
            GDM_TRY(gemm64_dd(ctx, s64, Z64, nullptr, F, 1.0, 0.0, 0.0, 0));     // F = s Z
            GDM_TRY(gemm64_dd(ctx, Z64, F, nullptr, E, 1.0, 0.0, -1.0, 1));     // E = Z (s Z) - I
            double emax = 0.0;
            {
                GDM_TIMED(ctx, "refine64");
                GDM_TRY(gdm_fill_f64(ctx, emax_d, 1, 0.0));
                hipLaunchKernelGGL(k_resid_max, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, E,
                                   (unsigned long long*)emax_d);
            }
            GDM_LAUNCH_CHECK(ctx);
            GDM_HIP(ctx, hipMemcpyAsync(&emax, emax_d, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (emax <= kZResidMax) {
                GDM_TRY(gemm64_dd(ctx, Z64, E, Z64, F, -0.5, 1.0, 0.0, 1));        // F <- Z - Z E / 2
                GDM_HIP(ctx, hipMemcpyAsync(Z64, F, sizeof(double) * P.tot2, hipMemcpyDeviceToDevice, ctx->stream));
                break;
            }
            if (extra >= ctx->mixed_ns_z_extra || !std::isfinite(emax))
                return gdm_fail(ctx, GDM_E_NOT_CONVERGED,
                                "mixed: inverse-overlap factor residual %.3g after %d Newton-Schulz iterations "
                                "(overlap too ill-conditioned)", emax, ctx->mixed_ns_z_used);
            GDM_TRY(ns_step(true));
            ++ctx->mixed_ns_z_used;
        }
        Z = slot(ctx, SL_Z);
        {
            GDM_TIMED(ctx, "refine64");
            hipLaunchKernelGGL(k_z64_to_split, dim3(4096), dim3(256), 0, ctx->stream, P.tot2 / 4, Z64, hl(Z));
        }
        GDM_LAUNCH_CHECK(ctx);
        GDM_TRY(gemm64_core<double>(ctx, s64, Z64, F, "refine64"));   // V = s[core,:] Z
    }
    // h_perp = Z h Z (T = Z h, then T Z)
    GDM_TRY(gemm(ctx, Z, slot(ctx, SL_H), hl(T), none(), none(), 1.0f, 0.0f, 0.0f, "ns_gemm", 0));
    GDM_TRY(gemm(ctx, T, Z, slot(ctx, SL_HP), none(), none(), 1.0f, 0.0f, 0.0f, "ns_gemm"));
    {
        GDM_TIMED(ctx, "mixed_misc");
        hipLaunchKernelGGL(k_sym_bounds, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, slot(ctx, SL_HP),
                           (int)strip_grid(P).y, bounds);
    }
    GDM_LAUNCH_CHECK(ctx);
    std::vector<double> hb(2 * (size_t)P.n_sub * strip_grid(P).y);
    GDM_HIP(ctx, hipMemcpyAsync(hb.data(), bounds, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double lo = INFINITY, hi = -INFINITY;
    for (size_t k = 0; k < hb.size(); k += 2) {
        lo = std::min(lo, hb[k]);
        hi = std::max(hi, hb[k + 1]);
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
    ctx->mixed_beta = beta;
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
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const double beta = 1.0 / kT;
    const double kappa = (mu - ctx->mixed_mu_pass) * beta;
    double* G = fp64_region(ctx, 1);
    double* G2 = fp64_region(ctx, 3);
    double* Gk = fp64_region(ctx, 0);
    double* Dp = fp64_region(ctx, 4);
    // D[core,:] = (G + kappa (G - G2)) Z,  G = Z[core,:] X, G2 = Z[core,:] X^2 of the last pass
    {
        GDM_TIMED(ctx, "dcore");
        hipLaunchKernelGGL(k_combine, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, G, G, G2, Gk, kappa);
    }
    GDM_LAUNCH_CHECK(ctx);
    GDM_TRY(gemm64_core<double>(ctx, Gk, z64(ctx), Dp, "dcore"));
    {
        GDM_TIMED(ctx, "dcore");
        hipLaunchKernelGGL(k_pack_core, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, Dp, D_core);
    }
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

// ---------------------------------------------------------- charge response

// History buffers for up to mixed_rec_cap doublings (X_k, Y_k: 8 B per padded
// element each doubling) and the FP64 work of the response: s[core,:] Z and
// the padded response rows (tot2 each), the packed response rows (totd) and
// the orbital potentials (totv).  Released when recording is off.
int gdm_mixed_response_alloc(gdm_ctx* ctx) {
    const Plan& P = ctx->plan;
    if (ctx->mixed_rec_cap <= 0 || P.precision != GDM_MIXED_F16 || P.n_sub <= 0) {
        GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int b : {BUF_HIST_HI, BUF_HIST_LO, BUF_RESP}) gdm_buf_release(ctx, b);
        return GDM_OK;
    }
    bool ok = true;
    const size_t halves = (size_t)2 * ctx->mixed_rec_cap * (size_t)P.tot2;
    gdm_buf(ctx, BUF_HIST_HI, sizeof(_Float16) * halves, &ok);
    gdm_buf(ctx, BUF_HIST_LO, sizeof(_Float16) * halves, &ok);
    gdm_buf(ctx, BUF_RESP, sizeof(double) * (size_t)(2 * P.tot2 + P.totd + P.totv), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "charge response: history allocation failed");
    return GDM_OK;
}

// Canonical first-order response of the collected charges to a change dV of
// the atomic potentials, by differentiating the recorded expansion:
//   dh = 1/2 s o (dv 1^T + 1 dv^T),  dh_perp = Z dh Z,  dX_0 = -q dh_perp,
//   per doubling (X_{k+1} = X_k^2 Y_k, Y_k = (2 X_k^2 - 2 X_k + I)^-1):
//     dX2 = X_k dX_k + dX_k X_k,
//     dX_{k+1} = (dX2 - X_{k+1} dA_k) Y_k with dA_k = 2 dX2 - 2 dX_k,
//              = (2 X_{k+1} (dX_k - dX2) + dX2) Y_k   (X_{k+1}, Y_k commute),
// then dD[core,:] = Z[core,:] (dX + beta dmu (X - X^2)) Z with dmu from a
// constant electron count, and dq = 2 diag(dD S) per atom.
int gdm_mixed_response(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg, const int32_t* row_ptr,
                       const int32_t* col, int64_t nnz, const double* S, const double* dV, double* dq, double* dmu) {
    const Plan& P = ctx->plan;
    const int nd = ctx->mixed_rec_nd;
    if (nd < 1)
        return gdm_fail(ctx, GDM_E_STATE,
                        "gdm_density_response: the last expansion (%d doublings) was not recorded; call "
                        "gdm_set_response with room for it before gdm_find_mu", ctx->mixed_nd);
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    double* s64 = (double*)ctx->b[BUF_S].p;
    double* R0 = (double*)ctx->b[BUF_RESP].p;   // s[core,:] Z
    double* R1 = R0 + P.tot2;                    // padded response rows
    double* dDp = R1 + P.tot2;                   // packed response rows
    double* dv = dDp + P.totd;                   // orbital potentials
    double* Gd = fp64_region(ctx, 4);
    double* G = fp64_region(ctx, 1);
    double* G2 = fp64_region(ctx, 3);
    // the response GEMMs are not part of the expansion statistics
    const int64_t gemms0 = ctx->mixed_gemms;
    const double flops0 = ctx->mixed_flops, bytes0 = ctx->mixed_bytes;
    if (!ctx->resp_v_ready) {
        GDM_TRY(gemm64_core<double>(ctx, s64, z64(ctx), R0, "response"));
        ctx->resp_v_ready = true;
    }
    {
        GDM_TIMED(ctx, "response");
        hipLaunchKernelGGL(k_orb_dv, dim3(P.n_sub), dim3(64), 0, ctx->stream, desc, sg->atoms, sys->orb_ptr, dV, dv);
        GDM_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_dh, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, s64, dv, hl(slot(ctx, SL_H)));
        GDM_LAUNCH_CHECK(ctx);
    }
    const SplitMat Z = slot(ctx, SL_Z), T = slot(ctx, SL_T), Pm = slot(ctx, SL_R), dX2 = slot(ctx, SL_Y2),
                   Dl = slot(ctx, SL_Y);
    SplitMat dX = slot(ctx, SL_A), dXn = slot(ctx, SL_YI);
    GDM_TRY(gemm(ctx, Z, slot(ctx, SL_H), hl(T), none(), none(), 1.0f, 0.0f, 0.0f, "response", 0));
    GDM_TRY(gemm(ctx, T, Z, none(), hl(dX), none(), (float)-ctx->mixed_x0_slope, 0.0f, 0.0f, "response"));
    const int4* sym_tiles = (const int4*)ctx->b[BUF_TILES].p + ctx->mixed_tiles;
    for (int k = 0; k < nd; ++k) {
        const SplitMat Xk = hist(ctx, k, 0), Yk = hist(ctx, k, 1);
        const SplitMat Xn = k + 1 == nd ? slot(ctx, SL_X) : hist(ctx, k + 1, 0);
        GDM_TRY(gemm(ctx, Xk, dX, hl(Pm), none(), none(), 1.0f, 0.0f, 0.0f, "response", 0));
        {
            GDM_TIMED(ctx, "response");
            hipLaunchKernelGGL(k_sym_pair, dim3((unsigned)ctx->mixed_tiles_sym), dim3(256), 0, ctx->stream, desc,
                               sym_tiles, hl(Pm), hl(dX), hl(dX2), hl(Dl));
        }
        GDM_LAUNCH_CHECK(ctx);
        GDM_TRY(gemm(ctx, Xn, Dl, none(), hl(T), hl(dX2), 2.0f, 1.0f, 0.0f, "response", 0));
        GDM_TRY(gemm(ctx, T, Yk, k + 1 == nd ? slot(ctx, SL_Z2) : hl(dXn), none(), none(), 1.0f, 0.0f, 0.0f,
                     "response", 0));
        std::swap(dX, dXn);
    }
    ctx->mixed_gemms = gemms0;
    ctx->mixed_flops = flops0;
    ctx->mixed_bytes = bytes0;
    // Gd = Z[core,:] dX at fixed mu, its electron count, and the canonical shift
    GDM_TRY(gemm64_core<float>(ctx, z64(ctx), slot(ctx, SL_Z2).f, Gd, "response"));
    double* part = (double*)ctx->b[BUF_TR].p;
    {
        GDM_TIMED(ctx, "response");
        hipLaunchKernelGGL(k_trace_dot, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, Gd, Gd, R0, part);
        GDM_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kEw), 0, ctx->stream, P.n_sub, part,
                           part + 2 * (size_t)P.n_sub);
        GDM_LAUNCH_CHECK(ctx);
    }
    double h[2];
    GDM_HIP(ctx, hipMemcpyAsync(h, part + 2 * (size_t)P.n_sub, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    // N'(mu) = beta M (slope of the last pass): dmu = -dN0 / (beta M), and the
    // shift adds beta dmu Z(X - X^2)Z^T, i.e. kappa = beta dmu = -dN0 / M
    const double slope = ctx->mixed_slope;
    const double dm = slope > 0.0 ? -h[0] / slope : 0.0;
    const double kappa = slope > 0.0 ? dm * ctx->mixed_beta : 0.0;
    {
        GDM_TIMED(ctx, "response");
        hipLaunchKernelGGL(k_combine, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, Gd, G, G2, Gd, kappa);
    }
    GDM_LAUNCH_CHECK(ctx);
    GDM_TRY(gemm64_core<double>(ctx, Gd, z64(ctx), R1, "response"));
    {
        GDM_TIMED(ctx, "response");
        hipLaunchKernelGGL(k_pack_core, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, R1, dDp);
    }
    GDM_LAUNCH_CHECK(ctx);
    const double zero[2] = {0.0, 0.0};
    GDM_TRY(gdm_launch_mulliken(ctx, sys, sg, row_ptr, col, nnz, S, dDp, zero, dq));
    if (dmu) *dmu = dm;
    return GDM_OK;
}

extern "C" int gdm_set_mixed_storage(gdm_ctx* ctx, int upper_tiles) {
    if (!ctx) return GDM_E_ARG;
    if (upper_tiles != 0 && upper_tiles != 1)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_set_mixed_storage: upper_tiles must be 0 or 1");
    ctx->mixed_packed = upper_tiles;
    return GDM_OK;
}

extern "C" int gdm_set_mixed_options(gdm_ctx* ctx, int ns_z, int ns_inv, int max_passes, int ns_z_extra) {
    if (!ctx) return GDM_E_ARG;
    if (ns_z > 64 || ns_inv > 16 || max_passes > 64 || ns_z_extra > 32)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_set_mixed_options: values out of range");
    if (ns_z > 0) ctx->mixed_ns_z = ns_z;
    if (ns_inv > 0) ctx->mixed_ns_inv = ns_inv;
    if (max_passes > 0) ctx->mixed_max_passes = max_passes;
    if (ns_z_extra >= 0) ctx->mixed_ns_z_extra = ns_z_extra;
    return GDM_OK;
}

extern "C" int gdm_mixed_stats(gdm_ctx* ctx, int* passes, int* n_doublings, int64_t* gemm_launches,
                               double* flops_per_launch, double* bytes_per_launch, int* ns_z_used) {
    if (!ctx) return GDM_E_ARG;
    if (passes) *passes = ctx->mixed_passes;
    if (n_doublings) *n_doublings = ctx->mixed_nd;
    if (gemm_launches) *gemm_launches = ctx->mixed_gemms;
    if (flops_per_launch) *flops_per_launch = ctx->mixed_gemms ? ctx->mixed_flops / (double)ctx->mixed_gemms : 0.0;
    if (bytes_per_launch) *bytes_per_launch = ctx->mixed_gemms ? ctx->mixed_bytes / (double)ctx->mixed_gemms : 0.0;
    if (ns_z_used) *ns_z_used = ctx->mixed_ns_z_used;
    return GDM_OK;
}

extern "C" int gdm_debug_slot(gdm_ctx* ctx, int which, int sub, float* out) {
    if (!ctx) return GDM_E_ARG;
    const Plan& P = ctx->plan;
    static const int kDebugSlots[3] = {SL_Z, SL_HP, SL_X};
    if (P.precision != GDM_MIXED_F16 || which < 0 || which >= 3 || sub < 0 || sub >= P.n_sub || !out)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_debug_slot: bad argument");
    const SubDesc& d = P.desc[sub];
    GDM_HIP(ctx, hipMemcpyAsync(out, slot(ctx, kDebugSlots[which]).f + d.off2, sizeof(float) * (size_t)d.ld * d.ld,
                                hipMemcpyDeviceToDevice, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GDM_OK;
}
