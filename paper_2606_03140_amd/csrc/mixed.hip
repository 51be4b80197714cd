// Mixed-precision recursive Fermi-operator expansion (the "recursive
// Fermi-operator expansion" option of the paper's subgraph step, run on the
// matrix cores as the paper's accelerator library does for FOE and the
// inverse overlap).  Per subgraph, padded to P = 64 * ceil(n / 64):
//
//   Z = s^-1/2 by coupled Newton-Schulz on s/c (c the largest absolute row
//       sum of s): Z0 = kZ0a I + kZ0b s/c (linear minimax start), Y0 = (s/c) Z0,
//       T = (3I - Z Y)/2, Y <- Y T, Z <- T Z; then Z64 = Z / sqrt(c) in FP64
//       and one third-order FP64 residual step with E = Z64 s Z64 - I,
//       Z64 <- Z64 (I - E/2 + 3/8 E^2),
//   h_perp = Z h Z,
//   K = b (h_perp - mu I), b = beta / 2^n_d, and the start X0 = f_b(K) to
//       high order: the degree-7 odd polynomial of kStart7 (n_d >= 5), else
//       the cubic I/2 - K/4 + K^3/108, or the linear I/2 - K/4 when the pass is
//       recorded for the charge response,
//   n_d times:  X2 = X X,  A = 2 X2 - 2 X + I = X^2 + (I - X)^2,
//               Y = A^-1 by Newton-Schulz from a minimax start on [1/2, 1]:
//               the quartic y4 of kInvStart4 (two products, |I - A Y0| <=
//               1/3363) and ns_inv = 1 iteration by default, or the
//               quadratic (420 I - 576 A + 256 A^2) / 99 (one product, <= 1/99)
//               and ns_inv = 2,
//               X <- X2 Y            (f_b -> f_2b);
//   the last of them with X2, A and X2 Y in FP64 on the FP64 matrix cores,
//       its inverse started on the split products as above and finished by
//       one FP64 Newton-Schulz step (two for BF16 pairs),
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
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

namespace {

constexpr int kTile = 64;       // output tile edge per workgroup
constexpr int kK = 64;          // k-step per LDS stage (two MFMA k-steps of 32)
constexpr int kLdsRow = kK + 8; // padded LDS row (halves): 144 B, conflict-free MFMA operand reads
constexpr int kGemmThreads = 256;
constexpr int kXcds = 8;        // workgroup b is dispatched to XCD b mod 8
constexpr float kLoScale = 2048.0f;            // 2^11
constexpr float kLoInv = 1.0f / 2048.0f;

// A matrix as FP32 (f, nullable) and/or as a split pair of 16-bit halves:
// FP16 x = hi + 2^-11 lo, or (bf = 1) BF16 x = hi + 2^-8 lo, each half the
// nearest value of its format to what is left of x.
struct SplitMat {
    float* f;
    _Float16* hi;       // 16-bit halves (BF16 bit patterns when bf = 1)
    _Float16* lo;
    int bf;
};

// State of the chemical-potential search, in device memory (doubles): the
// spectral bounds, the current mu and its doubling count n_d and scale
// b = beta / 2^n_d, the start polynomial, the bracket, the traces N and M of
// the last pass and the mu they were taken at, the result, and counters.
enum {
    kStLo = 0, kStHi, kStMu, kStB, kStNd, kStStart, kStBlo, kStBhi, kStN, kStM, kStMuPass, kStMuOut, kStNOut,
    kStPasses, kStDone, kStCount = 16
};
// Predicate flags (int, 1 = skip) of the launches of a search whose launch
// count is fixed in advance: pass p, doubling j of pass p, extra inverse-
// overlap iteration r.
constexpr int kMaxPasses = 16;
constexpr int kMaxNd = 40;
constexpr int kMaxNsExtra = 32;
constexpr int kFlPass = 0;
constexpr int kFlDbl = kFlPass + kMaxPasses;
constexpr int kFlNs = kFlDbl + kMaxPasses * kMaxNd;
constexpr int kFlCount = kFlNs + kMaxNsExtra + 1;

// Start of the expansion: 0 linear, 1 cubic, 2 degree 7.
enum { kStartLinear = 0, kStartCubic = 1, kStartSeptic = 2 };

// Doubling count and start polynomial for chemical potential mu and spectral
// bounds [lo, hi]: each doubling maps f(u) to f(2u), so n_d doublings from
// X0 = f_b(K), K = b (h - mu), b = beta / 2^n_d, give f_beta; the start must
// keep X0 in [0, 1] over the half-width R = max(|lo - mu|, |hi - mu|): the
// linear start for b R <= 2, the cubic for b R <= 4, the degree-7 polynomial
// for b R <= 8 (and at least 5 doublings after it).  A recorded pass (charge
// response) uses the linear start; `septic_only` (device-side search) always
// uses the degree-7 start with n_d >= 5.
__host__ __device__ inline int mixed_doublings(double beta, double lo, double hi, double mu, int rec, int septic_only,
                                               int* start) {
    const double R = fmax(fabs(lo - mu), fabs(hi - mu));
    const int nd7 = (int)ceil(log2(0.125 * beta * R));
    int nd;
    if (septic_only) {
        *start = kStartSeptic;
        nd = nd7 > 5 ? nd7 : 5;
    } else if (rec) {
        *start = kStartLinear;
        nd = (int)ceil(log2(0.5 * beta * R));
    } else if (nd7 >= 5) {
        *start = kStartSeptic;
        nd = nd7;
    } else {
        *start = kStartCubic;
        nd = (int)ceil(log2(0.25 * beta * R));
    }
    return nd < 1 ? 1 : (nd > kMaxNd ? kMaxNd : nd);
}

// One step of the search after a pass at mu gave the count N and its
// derivative beta M: safeguarded Newton inside the bracket [blo, bhi]
// (bisection when the Newton point leaves it or does not halve it).  The
// search is done when the count matches within tol, when the Newton step is
// below 1e-2 kT (the first-order term of the density then finishes it), or
// on the last pass; *dmu is then the first-order correction, applied when it
// lies within kT and the count is not yet matched.
__host__ __device__ inline void mixed_mu_step(double mu, double N, double M, double n_e, double beta, double kT,
                                              double tol, int last, double* blo, double* bhi, double* next,
                                              int* done, double* dmu) {
    const double dN = n_e - N, slope = beta * M;
    const double newton = slope > 0.0 ? dN / slope : INFINITY;
    *dmu = 0.0;
    *next = mu;
    *done = fabs(dN) <= tol || fabs(newton) <= 1e-2 * kT || last;
    if (*done) {
        if (fabs(dN) > tol && slope > 0.0 && fabs(newton) <= kT) *dmu = newton;
        return;
    }
    if (dN > 0.0) *blo = mu; else *bhi = mu;
    double x = slope > 0.0 ? mu + newton : 0.5 * (*blo + *bhi);
    if (!(x > *blo && x < *bhi) || fabs(x - mu) > 0.5 * (*bhi - *blo)) x = 0.5 * (*blo + *bhi);
    *next = x;
}

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
    const int* skip;     // nullable: the launch does nothing when *skip != 0 (device-side
                         // predication of launches whose count is fixed at capture time)
};

constexpr float kLoScaleBf = 256.0f;            // 2^8
constexpr float kLoInvBf = 1.0f / 256.0f;

// FP32 -> BF16 (round to nearest even) and back, as bit patterns
__device__ __forceinline__ _Float16 bf16_of(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
}
__device__ __forceinline__ float f32_of_bf16(_Float16 b) {
    return __builtin_bit_cast(float, (uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

__device__ __forceinline__ void split_one(float v, int bf, _Float16& h, _Float16& l) {
    if (bf) {
        h = bf16_of(v);
        l = bf16_of((v - f32_of_bf16(h)) * kLoScaleBf);
    } else {
        h = (_Float16)v;
        l = (_Float16)((v - (float)h) * kLoScale);
    }
}

__device__ __forceinline__ float join_one(_Float16 h, _Float16 l, int bf) {
    return bf ? f32_of_bf16(h) + kLoInvBf * f32_of_bf16(l) : (float)h + kLoInv * (float)l;
}

__device__ __forceinline__ void store_split(SplitMat m, int64_t idx, float v) {
    if (m.f) m.f[idx] = v;
    if (m.hi) {
        _Float16 h, l;
        split_one(v, m.bf, h, l);
        m.hi[idx] = h;
        m.lo[idx] = l;
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
            _Float16 hh, ll;
            split_one(x[q], m.bf, hh, ll);
            h[q] = hh;
            l[q] = ll;
        }
        *(half4*)(m.hi + idx) = h;
        *(half4*)(m.lo + idx) = l;
    }
}

// x = hi + 2^-11 lo (BF16: hi + 2^-8 lo) for four consecutive elements
__device__ __forceinline__ float4 load4(SplitMat m, int64_t idx) {
    if (m.f) return *(const float4*)(m.f + idx);
    const half4 h = *(const half4*)(m.hi + idx);
    const half4 l = *(const half4*)(m.lo + idx);
    return make_float4(join_one(h[0], l[0], m.bf), join_one(h[1], l[1], m.bf), join_one(h[2], l[2], m.bf),
                       join_one(h[3], l[3], m.bf));
}

// Four waves per SIMD (four workgroups per CU, as the LDS allows): the
// register budget is held to 128 per lane (no spills).
template <bool BF>
__global__ void __launch_bounds__(kGemmThreads) __attribute__((amdgpu_waves_per_eu(4))) k_gemm_split(const SubDesc* __restrict__ desc,
                                                            const int4* __restrict__ tiles, GemmArgs g) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[kGemmLds];
    _Float16* sAh = (_Float16*)lds;
    _Float16* sAl = sAh + kTile * kLdsRow;
    _Float16* sBh = sAl + kTile * kLdsRow;
    _Float16* sBl = sBh + kTile * kLdsRow;
    float* sC = (float*)lds;                    // reused after the k loop: [64][kOutRow]
    if (g.skip && *g.skip) return;
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
                    if constexpr (BF) {
                        const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah[i]), Al = __builtin_bit_cast(bf16x8, al[i]);
                        const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh[j]), Bl = __builtin_bit_cast(bf16x8, bl[j]);
                        acc_hh[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh, acc_hh[i][j], 0, 0, 0);
                        acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl, acc_x[i][j], 0, 0, 0);
                        acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, acc_x[i][j], 0, 0, 0);
                    } else {
                        acc_hh[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc_hh[i][j], 0, 0, 0);
                        acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc_x[i][j], 0, 0, 0);
                        acc_x[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc_x[i][j], 0, 0, 0);
                    }
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
                sC[ml * kOutRow + nl] = acc_hh[i][j][r] + (BF ? kLoInvBf : kLoInv) * acc_x[i][j][r];
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
            for (int r = 0; r < 4; ++r) x[r] = acc_hh[i][j][r] + (BF ? kLoInvBf : kLoInv) * acc_x[i][j][r];
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
// registers while the current one is multiplied, written to LDS with 16-byte
// stores.  LDS rows are padded to 34 (A) and 80 (B) doubles: with 64 banks
// of 4 bytes, the 32 lanes of a half-wave reading rows fr, k fk of A (2 fr +
// fk distinct mod 32) or k fk, columns fr of B (16 fk + fr distinct mod 32)
// touch every bank once.  The tile is staged
// in LDS (row stride 65) and written as coalesced rows; SYM (products of
// commuting symmetric matrices, upper tiles only) also writes the mirror
// tile from the transposed LDS read, and on a diagonal tile takes both
// halves from the upper triangle, so C is exactly symmetric.
constexpr int kK64 = 32;
constexpr int kA64Row = kK64 + 2;        // doubles per LDS row of the A slab
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

// Optional parts of an FP64 product: B + badd_scale * badd as the B operand
// (an FP32 correction added as the operand is staged), and the result also
// (or only, C = nullptr) written as split operands of cs_scale * C.
struct G64Extra {
    const float* badd;
    double badd_scale;
    SplitMat cs;
    double cs_scale;
    double a_shift;      // A - a_shift I as the A operand (subtracted on the diagonal as it is staged)
};

__device__ __forceinline__ void add8(const float* p, double s, double* v) {
    const float4 x = *(const float4*)p, y = *(const float4*)(p + 4);
    v[0] += s * x.x; v[1] += s * x.y; v[2] += s * x.z; v[3] += s * x.w;
    v[4] += s * y.x; v[5] += s * y.y; v[6] += s * y.z; v[7] += s * y.w;
}

template <typename TA, typename TB, bool SYM, bool SHIFT = false>
__global__ void __launch_bounds__(256) k_gemm64(const SubDesc* __restrict__ desc, const int4* __restrict__ tiles,
                                               const TA* __restrict__ A, const TB* __restrict__ B,
                                               const double* __restrict__ Cin, double* __restrict__ C,
                                               double alpha, double beta, double gamma,
                                               const int* __restrict__ skip, G64Extra x64) {
    __shared__ __align__(16) double lds[kG64Lds];
    if (skip && *skip) return;
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
    const float* pba = x64.badd ? x64.badd + base + (int64_t)rb * P + n0 + cb : nullptr;
    double va[8], vb[8];
    // SHIFT: the A slab's element (m0 + ra, k + ca + u) is on the diagonal for
    // u = m0 + ra - k - ca
    load8(pa, va);
    if constexpr (SHIFT) {
        const int q = m0 + ra - ca;
#pragma unroll
        for (int u = 0; u < 8; ++u) va[u] -= u == q ? x64.a_shift : 0.0;
    }
    load8(pb, vb);
    if (pba) add8(pba, x64.badd_scale, vb);
    double4v acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = double4v{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < P; k0 += kK64) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
            *(double2*)(sA + ra * kA64Row + ca + q) = make_double2(va[q], va[q + 1]);
            *(double2*)(sB + rb * kB64Row + cb + q) = make_double2(vb[q], vb[q + 1]);
        }
        __syncthreads();
        if (k0 + kK64 < P) {
            load8(pa + k0 + kK64, va);
            if constexpr (SHIFT) {
                const int q = m0 + ra - (k0 + kK64) - ca;
#pragma unroll
                for (int u = 0; u < 8; ++u) va[u] -= u == q ? x64.a_shift : 0.0;
            }
            load8(pb + (int64_t)(k0 + kK64) * P, vb);
            if (pba) add8(pba + (int64_t)(k0 + kK64) * P, x64.badd_scale, vb);
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
        if (C) C[idx] = v;
        if (x64.cs.hi) store_split(x64.cs, idx, (float)(x64.cs_scale * v));
    }
    if (SYM && !diag)
        for (int e = t; e < 64 * 64; e += 256) {
            const int nn = e >> 6, mm = e & 63;      // mirror tile row n0 + nn, column m0 + mm
            const int64_t idx = base + (int64_t)(n0 + nn) * P + m0 + mm;
            double v = alpha * sC[mm * kC64Row + nn];
            if (Cin) v += beta * Cin[idx];
            if (C) C[idx] = v;
            if (x64.cs.hi) store_split(x64.cs, idx, (float)(x64.cs_scale * v));
        }
}

// Z (FP16 hi/lo split) <- Z64, flat over every packed tile (padding included)
__global__ void __launch_bounds__(256) k_z64_to_split(int64_t n4, const double* __restrict__ Z64, SplitMat Z,
                                                     const int* __restrict__ skip) {
    if (skip && *skip) return;
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
                                                  double* __restrict__ part, const int* __restrict__ skip) {
    __shared__ double red[4];
    if (skip && *skip) return;
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, P = d.ld, nc = d.nc;
    double an = 0.0, am = 0.0;
    // four consecutive columns per thread (32-byte loads; the padded row
    // length P is a multiple of 64, columns from n on are skipped)
    const int q4 = P >> 2;
    for (int e = threadIdx.x; e < nc * q4; e += 256) {
        const int a = e / q4, c0 = (e - a * q4) * 4;
        if (c0 >= n) continue;
        const int64_t idx = d.off2 + (int64_t)a * P + c0;
        const double4 g = *(const double4*)(G + idx), g2 = *(const double4*)(G2 + idx),
                      v = *(const double4*)(V + idx);
        const double gv[4] = {g.x, g.y, g.z, g.w}, g2v[4] = {g2.x, g2.y, g2.z, g2.w}, vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (c0 + q < n) {
                an += gv[q] * vv[q];
                am += (gv[q] - g2v[q]) * vv[q];
            }
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
                                                double* Gk, double kappa, const double* __restrict__ mu_dev,
                                                const double* __restrict__ st, double beta) {
    // with mu_dev: kappa = (mu - mu of the expansion pass) beta, both read on the device
    if (mu_dev) kappa = (mu_dev[0] - st[kStMuPass]) * beta;
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
constexpr double kZResidMax = 1e-3;   // largest |Z s Z - I| entry accepted before refinement
constexpr double kRefineSig = 65536.0;  // scale of E and T as split operands in the refinement
constexpr double kLastSig = 16384.0;    // scale of the last doubling's residual I - A Y as split operands

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

// Z64 <- (Z + Z^T) / (2 sqrt(c)) in FP64 on the n x n block (padding copied:
// it stays the identity through the iteration), on the upper-tile list: a
// workgroup averages tile (I, J) with the transpose of tile (J, I) through
// LDS and writes both.  The split products leave Z symmetric only to the last
// bit of their epilogue rounding; the refinement needs it exactly symmetric.
__global__ void __launch_bounds__(256) k_scale_sym_to_f64(const SubDesc* __restrict__ desc,
                                                         const int4* __restrict__ tiles, const float* __restrict__ Zf,
                                                         const double* __restrict__ scale, int orthogonal,
                                                         double* __restrict__ Z64, const int* __restrict__ skip) {
    __shared__ float a[64][65], bt[64][65];
    if (skip && *skip) return;
    const int4 tl = tiles[blockIdx.x];
    if (tl.x < 0) return;
    const SubDesc d = desc[tl.x];
    const int P = d.ld, n = d.n;
    const int I0 = tl.y * 64, J0 = tl.z * 64;
    const double f = orthogonal ? 1.0 : 1.0 / sqrt(scale[tl.x]);
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        a[r][c] = Zf[d.off2 + (int64_t)(I0 + r) * P + J0 + c];
        bt[r][c] = Zf[d.off2 + (int64_t)(J0 + r) * P + I0 + c];
    }
    __syncthreads();
    // both tiles written row by row (coalesced): element (I0 + r, J0 + c) from
    // a[r][c] and its mirror partner, element (J0 + r, I0 + c) from bt[r][c] and
    // its partner a[c][r]; the average is the same expression for both
    // members of a pair, so a diagonal tile gets one value per element
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        const bool in1 = I0 + r < n && J0 + c < n, in2 = J0 + r < n && I0 + c < n;
        const double v1 = 0.5 * ((double)a[r][c] + (double)bt[c][r]);
        const double v2 = 0.5 * ((double)a[c][r] + (double)bt[r][c]);
        Z64[d.off2 + (int64_t)(I0 + r) * P + J0 + c] = in1 ? v1 * f : (double)a[r][c];
        Z64[d.off2 + (int64_t)(J0 + r) * P + I0 + c] = in2 ? v2 * f : (double)bt[r][c];
    }
}

// dst <- src^T over every subgraph's P x P tile, on the upper-tile list (both
// tiles of a pair through LDS); FP64 (dst64) and, when dsplit.hi is set, the
// split halves and FP32 copy of the transpose; copy (nullable) <- src
// With add: src + add * scale_s^-1/2 * inv_sig in place of src (copy may
// then be src itself: each element is read and written by one thread only).
__global__ void __launch_bounds__(256) k_transpose64(const SubDesc* __restrict__ desc, const int4* __restrict__ tiles,
                                                    const double* src, double* copy, const float* __restrict__ add,
                                                    const double* __restrict__ scale, double inv_sig,
                                                    double* __restrict__ dst64, SplitMat dsplit,
                                                    const int* __restrict__ skip) {
    // one 64 x 64 LDS tile, used twice: first the tile at (J0, I0), whose
    // transpose is the output at (I0, J0), then the tile at (I0, J0) for the
    // output at (J0, I0) (a diagonal tile is done after the first)
    __shared__ double t[64][65];
    if (skip && *skip) return;
    const int4 tl = tiles[blockIdx.x];
    if (tl.x < 0) return;
    const SubDesc d = desc[tl.x];
    const int P = d.ld;
    const int I0 = tl.y * 64, J0 = tl.z * 64;
    const double f = add ? inv_sig / sqrt(scale[tl.x]) : 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        const int R0 = pass == 0 ? J0 : I0, C0 = pass == 0 ? I0 : J0;     // tile read: rows R0.., cols C0..
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            const int64_t j = d.off2 + (int64_t)(R0 + r) * P + C0 + c;
            const double v = add ? src[j] + f * (double)add[j] : src[j];
            t[r][c] = v;
            if (copy) copy[j] = v;          // src as it is (with the addend), in place allowed
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            const int64_t i = d.off2 + (int64_t)(C0 + r) * P + R0 + c;     // dst[C0+r][R0+c] = src[R0+c][C0+r]
            const double v = t[c][r];
            if (dst64) dst64[i] = v;
            if (dsplit.hi) store_split(dsplit, i, (float)v);
        }
        if (I0 == J0) return;
        __syncthreads();
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
                                           SplitMat X, double mu, double q, double c0, const double* __restrict__ st,
                                           const int* __restrict__ skip) {
    if (skip && *skip) return;
    if (st) {                   // K = b (H - mu I) with mu and b of the device-side search
        mu = st[kStMu];
        q = -st[kStB];
        c0 = 0.0;
    }
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

__global__ void k_sum_parts(int n_sub, const double* __restrict__ part, double* __restrict__ out,
                            const int* __restrict__ skip) {
    __shared__ double red[kEw / 64];
    if (skip && *skip) return;
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
// max |E_ij| over the subgraph's n x n block (atomic, as the bit pattern of a
// non-negative double); with Es.hi, sig E is also written as split operands
// over the whole padded strip (for the refinement's split products)
__global__ void __launch_bounds__(kEw) k_resid_max(const SubDesc* __restrict__ desc, const double* __restrict__ E,
                                                  unsigned long long* __restrict__ out, SplitMat Es, double sig,
                                                  const int* __restrict__ skip) {
    if (skip && *skip) return;
    const SubDesc d = desc[blockIdx.x];
    const int P = d.ld, n = d.n, r0 = blockIdx.y * 64;
    if (r0 >= n) return;
    double m = 0.0;
    const int q4 = P >> 2;
    for (int e = threadIdx.x; e < 64 * q4; e += kEw) {
        const int i = r0 + e / q4, j0 = (e % q4) * 4;
        const int64_t idx = d.off2 + (int64_t)i * P + j0;
        const double4 x = *(const double4*)(E + idx);
        const double xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (i < n && j0 + q < n) {
                const double v = fabs(xv[q]);
                m = v == v ? fmax(m, v) : INFINITY;
            }
        if (Es.hi)
            store4(Es, idx, make_float4((float)(sig * x.x), (float)(sig * x.y), (float)(sig * x.z),
                                        (float)(sig * x.w)));
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

// X64 <- X (FP32 copy when present, else hi + 2^-11 lo), flat over every
// packed tile (X in whole storage)
__global__ void __launch_bounds__(256) k_split_to_f64(int64_t n4, SplitMat X, double* __restrict__ X64,
                                                     const int* __restrict__ skip) {
    if (skip && *skip) return;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n4; e += (int64_t)gridDim.x * 256) {
        const float4 v = load4(X, 4 * e);
        *(double4*)(X64 + 4 * e) = make_double4(v.x, v.y, v.z, v.w);
    }
}

// ------------------------------------------------- chemical-potential search
// Parameters of the search, fixed per gdm_find_mu call.
struct MuCfg {
    double n_e, beta, kT, tol, tol_final, guess;
    int rec;          // the passes are recorded for the charge response (linear start)
    int dev;          // device-side search: fixed launch counts, predicated
    int nd_launch;    // doublings launched per pass in the device-side search
    int max_passes;
};

// Plan the pass about to run at st[kStMu]: n_d, b and the start, and (device
// search) the doubling predicates of pass p: doubling j of the nd_launch
// launched runs iff j >= nd_launch - n_d.
__device__ void mu_plan_pass(const MuCfg& c, double* st, int* fl, int p, int* status) {
    int start = 0;
    int nd = mixed_doublings(c.beta, st[kStLo], st[kStHi], st[kStMu], c.rec, c.dev, &start);
    if (c.dev && nd > c.nd_launch) {
        gdm_raise(status, GDM_STATUS_CAPACITY);      // more doublings than were launched
        nd = c.nd_launch;
    }
    st[kStNd] = nd;
    st[kStStart] = start;
    st[kStB] = c.beta / ldexp(1.0, nd);
    if (c.dev && p < kMaxPasses) {
        fl[kFlPass + p] = 0;
        for (int j = 0; j < c.nd_launch; ++j) fl[kFlDbl + p * kMaxNd + j] = j < c.nd_launch - nd ? 1 : 0;
    }
}

// Global spectral bounds from the per-strip Gershgorin bounds, the bracket,
// the first mu (the device guess when given and inside the bounds, else the
// host guess, else the middle) and the plan of pass 0; later passes are
// marked skipped until a step asks for them.
__global__ void __launch_bounds__(kEw) k_mu_init(const double* __restrict__ bounds, int nb, const double* guess_dev,
                                                MuCfg c, double* __restrict__ st, int* __restrict__ fl,
                                                int* __restrict__ status) {
    __shared__ double red[kEw / 64];
    double lo = INFINITY, hi = -INFINITY;
    for (int k = threadIdx.x; k < nb; k += kEw) {
        lo = fmin(lo, bounds[2 * k]);
        hi = fmax(hi, bounds[2 * k + 1]);
    }
    lo = block_reduce_min(lo, red);
    hi = block_reduce_max(hi, red);
    if (threadIdx.x != 0) return;
    for (int k = 0; k < kStCount; ++k) st[k] = 0.0;
    if (!isfinite(lo) || !isfinite(hi)) {
        gdm_raise(status, GDM_STATUS_NAN);
        lo = -1.0;
        hi = 1.0;
    }
    st[kStLo] = lo;
    st[kStHi] = hi;
    st[kStBlo] = lo;
    st[kStBhi] = hi;
    double mu = 0.5 * (lo + hi);
    const double g = guess_dev ? guess_dev[0] : NAN;
    if (isfinite(g) && g > lo && g < hi) mu = g;
    else if (isfinite(c.guess) && c.guess > lo && c.guess < hi) mu = c.guess;
    st[kStMu] = mu;
    st[kStMuOut] = NAN;
    st[kStNOut] = NAN;
    if (c.dev)
        for (int p = 0; p < kMaxPasses; ++p) {
            fl[kFlPass + p] = 1;
            for (int j = 0; j < kMaxNd; ++j) fl[kFlDbl + p * kMaxNd + j] = 1;
        }
    mu_plan_pass(c, st, fl, 0, status);
}

// After pass p (skipped passes change nothing): record its traces, take the
// step, and plan pass p + 1, or finish with the result in kStMuOut/kStNOut.
__global__ void k_mu_update(int p, MuCfg c, const double* __restrict__ tr, double* __restrict__ st,
                            int* __restrict__ fl, int* __restrict__ status) {
    if (threadIdx.x != 0) return;
    if (c.dev && fl[kFlPass + p]) return;
    const double mu = st[kStMu], N = tr[0], M = tr[1];
    st[kStN] = N;
    st[kStM] = M;
    st[kStMuPass] = mu;
    st[kStPasses] = p + 1;
    if (!isfinite(N) || !isfinite(M)) gdm_raise(status, GDM_STATUS_NAN);
    double blo = st[kStBlo], bhi = st[kStBhi], next = mu, dmu = 0.0;
    int done = 0;
    mixed_mu_step(mu, N, M, c.n_e, c.beta, c.kT, c.tol, p + 1 >= c.max_passes, &blo, &bhi, &next, &done, &dmu);
    st[kStBlo] = blo;
    st[kStBhi] = bhi;
    st[kStDone] = done;
    if (done) {
        st[kStMuOut] = mu + dmu;
        st[kStNOut] = N + c.beta * M * dmu;
        return;
    }
    st[kStMu] = next;
    mu_plan_pass(c, st, fl, p + 1, status);
}

// Device-side search: copy the result to the caller's device scalars and
// raise the status word when the count misses n_e by more than tol_final.
__global__ void k_mu_final(MuCfg c, const double* __restrict__ st, double* __restrict__ mu_out,
                           double* __restrict__ n_out, int* __restrict__ status) {
    if (threadIdx.x != 0) return;
    const double mu = st[kStMuOut], n = st[kStNOut];
    mu_out[0] = mu;
    n_out[0] = n;
    if (!isfinite(mu) || !isfinite(n)) gdm_raise(status, GDM_STATUS_NAN);
    else if (fabs(n - c.n_e) > c.tol_final) gdm_raise(status, GDM_STATUS_NO_BRACKET);
}

// Inverse-overlap residual guard of the device-side search: round r > 0 is
// skipped once an earlier round met the residual bound; a round that runs
// and still misses it asks for round r + 1; after the last round a miss is
// a non-converged iteration.
__global__ void k_resid_flag(const double* __restrict__ emax, double bound, int r, int last, int* __restrict__ fl,
                             int* __restrict__ status) {
    if (threadIdx.x != 0) return;
    const int skipped = r > 0 && fl[kFlNs + r];
    const int ok = skipped || emax[0] <= bound;       // NaN counts as a miss
    fl[kFlNs + r + 1] = ok ? 1 : 0;
    if (last && !ok) gdm_raise(status, GDM_STATUS_NOT_CONVERGED);
}

// dst <- src over every packed tile (split halves and the FP32 copy when both
// have one), predicated
__global__ void __launch_bounds__(256) k_copy_split(int64_t n4, SplitMat src, SplitMat dst, const int* skip) {
    if (skip && *skip) return;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n4; e += (int64_t)gridDim.x * 256) {
        if (src.f && dst.f) *(float4*)(dst.f + 4 * e) = *(const float4*)(src.f + 4 * e);
        *(half4*)(dst.hi + 4 * e) = *(const half4*)(src.hi + 4 * e);
        *(half4*)(dst.lo + 4 * e) = *(const half4*)(src.lo + 4 * e);
    }
}

__global__ void k_zero1(double* p, const int* skip) {
    if (threadIdx.x == 0 && !(skip && *skip)) p[0] = 0.0;
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
    return SplitMat{f, hi, lo, ctx->plan.precision == GDM_MIXED_BF16};
}

static SplitMat none() { return SplitMat{nullptr, nullptr, nullptr, 0}; }

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
    gdm_buf(ctx, BUF_L, sizeof(double) * P.tot2 * 9, &ok);     // F/V, E/G, Z64, G2, D, X, X2, A, Z64^T (FP64)
    gdm_buf(ctx, BUF_MSTATE, sizeof(double) * kStCount + sizeof(int) * kFlCount, &ok);   // mu search state
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
static SplitMat hl(SplitMat m) { return SplitMat{nullptr, m.hi, m.lo, m.bf}; }

static int gemm(gdm_ctx* ctx, SplitMat A, SplitMat B, SplitMat O1, SplitMat O2, SplitMat E, float alpha,
                float beta, float gamma, const char* tag, int sym = 1, int packed = 0, const int* skip = nullptr) {
    // packed: bit 0 operands in upper-tile storage, bit 1 outputs (and E) on
    // upper tiles only; symmetric products only.  skip: device predicate.
    if (!sym) packed = 0;
    GemmArgs g{A, B, O1, O2, E, alpha, beta, gamma, sym, packed, skip};
    const int4* tl = (const int4*)ctx->b[BUF_TILES].p + (sym ? ctx->mixed_tiles : 0);
    const int64_t nt = sym ? ctx->mixed_tiles_sym : ctx->mixed_tiles;
    GDM_TIMED(ctx, tag);
    if (ctx->plan.precision == GDM_MIXED_BF16)
        hipLaunchKernelGGL(k_gemm_split<true>, dim3((unsigned)nt), dim3(kGemmThreads), 0, ctx->stream,
                           (const SubDesc*)ctx->b[BUF_DESC].p, tl, g);
    else
        hipLaunchKernelGGL(k_gemm_split<false>, dim3((unsigned)nt), dim3(kGemmThreads), 0, ctx->stream,
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

// Minimax starts of the inverse of A = 2 X^2 - 2 X + I, whose eigenvalues lie
// in [1/2, 1].  For a start y(a) of degree d the residual 1 - a y(a) is a
// polynomial of degree d + 1 equal to 1 at a = 0; its smallest maximum on
// [1/2, 1] is 1 / |T_{d+1}(-3)| (T the Chebyshev polynomial of the first kind,
// 4a - 3 mapping [1/2, 1] onto [-1, 1]), reached by the scaled T_{d+1} itself:
// 1/99 for the quadratic, 1/3363 for the quartic
// y4(a) = (23780 - 66240 a + 90880 a^2 - 61440 a^3 + 16384 a^4) / 3363.
// The quartic takes two products: Q = c4 A^2 + c3 A + c2 I (with A^2 kept as
// the raw product), then Y0 = Q A^2 + c1 A + c0 I; one Newton-Schulz step then
// leaves 3363^-2 = 8.8e-8, the split products' own rounding level, in one
// product fewer than the quadratic start's two steps (99^-4 = 1.0e-8).
static constexpr float kInvStart4[5] = {23780.0f / 3363.0f, -66240.0f / 3363.0f, 90880.0f / 3363.0f,
                                        -61440.0f / 3363.0f, 16384.0f / 3363.0f};

static int inv_start(gdm_ctx* ctx, SplitMat A, SplitMat Y, SplitMat T1, SplitMat T2, int pk, const int* sk) {
    if (ctx->mixed_inv_deg == 4) {
        const float* c = kInvStart4;
        GDM_TRY(gemm(ctx, A, A, hl(T1), hl(T2), hl(A), c[4], c[3], c[2], "foe_gemm", 1, pk, sk));
        return gemm(ctx, T2, T1, none(), hl(Y), hl(A), 1.0f, c[1], c[0], "foe_gemm", 1, pk, sk);
    }
    return gemm(ctx, A, A, none(), hl(Y), hl(A), 256.0f / 99.0f, -576.0f / 99.0f, 420.0f / 99.0f, "foe_gemm", 1, pk,
                sk);
}

// Doubling history for the charge response: X_k (which = 0), the input of
// doubling k, and Y_k (which = 1), its inverse (2 X_k^2 - 2 X_k + I)^-1, as
// FP16 hi/lo pairs.
static SplitMat hist(gdm_ctx* ctx, int k, int which) {
    const int64_t off = (int64_t)(2 * k + which) * ctx->plan.tot2;
    return SplitMat{nullptr, (_Float16*)ctx->b[BUF_HIST_HI].p + off, (_Float16*)ctx->b[BUF_HIST_LO].p + off,
                    ctx->plan.precision == GDM_MIXED_BF16};
}

static int last_doubling_f64(gdm_ctx* ctx, SplitMat Xin, SplitMat Yrec, const int* skip);

// Device state of the search: kStCount doubles, then the kFlCount int flags.
static double* mu_state(gdm_ctx* ctx) { return (double*)ctx->b[BUF_MSTATE].p; }
static int* mu_flags(gdm_ctx* ctx) { return (int*)(mu_state(ctx) + kStCount); }

// One full recursive expansion; leaves X (with its FP32 copy) in SL_X.
// Host-driven search (st == nullptr): at chemical potential mu with nd
// doublings from the given start, b = beta / 2^nd.  With a history buffer
// large enough, every X_k and Y_k is kept there (the products write into the
// history in place of the working slots, so recording adds no traffic).
// Device-side search (st != nullptr): the degree-7 start with mu and b read
// from the state, nd = the launched doubling count, the start skipped with
// the pass (pass_skip) and doubling j skipped while j < nd - n_d (dbl_skip[j]);
// the skipped doublings come first, so X holds the start when the first one
// that runs reads it.
static int foe_pass(gdm_ctx* ctx, double mu, double b, int nd, int start, const double* st, const int* pass_skip,
                    const int* dbl_skip) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const bool dev = st != nullptr;
    const bool rec = !dev && ctx->mixed_rec_cap >= nd && start == kStartLinear && ctx->mixed_rec_cap > 0;
    ctx->mixed_rec_nd = -1;
    ctx->mixed_x0_slope = b / 4.0;
    SplitMat X = slot(ctx, SL_X), X2 = slot(ctx, SL_X2), A = slot(ctx, SL_A), Rm = slot(ctx, SL_R);
    const SplitMat Ya = slot(ctx, SL_Y), Yb = slot(ctx, SL_YI);
    // upper-tile storage of the pass's symmetric matrices (not when recording:
    // the response reads the recorded X_k, Y_k whole)
    const int pk = (!rec && ctx->mixed_packed) ? 3 : 0;
    if (start != kStartLinear) {
        const SplitMat K = slot(ctx, SL_T);
        {
            GDM_TIMED(ctx, "mixed_misc");
            hipLaunchKernelGGL(k_x0, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, slot(ctx, SL_HP).f, hl(K), mu, -b,
                               0.0, st, pass_skip);
        }
        GDM_LAUNCH_CHECK(ctx);
        if (start == kStartSeptic) {
            // X0 = I/2 - K/4 + K (K^2 (K^2 (a7 K^2 + a5 I) + a3 I)), four products
            GDM_TRY(gemm(ctx, K, K, hl(Rm), hl(A), none(), kStart7[2], 0.0f, kStart7[1], "foe_gemm", 1, pk, pass_skip));
            GDM_TRY(gemm(ctx, Rm, A, none(), hl(Ya), none(), 1.0f, 0.0f, kStart7[0], "foe_gemm", 1, pk, pass_skip));
            GDM_TRY(gemm(ctx, Rm, Ya, hl(Yb), none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, pk, pass_skip));
            GDM_TRY(gemm(ctx, K, Yb, none(), hl(X), hl(K), 1.0f, -0.25f, 0.5f, "foe_gemm", 1, nd == 1 ? (pk & 1) : pk,
                         pass_skip));
        } else {
            GDM_TRY(gemm(ctx, K, K, hl(Rm), none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, pk));
            GDM_TRY(gemm(ctx, K, Rm, none(), hl(X), hl(K), 1.0f / 108.0f, -0.25f, 0.5f, "foe_gemm", 1,
                         nd == 1 ? (pk & 1) : pk));
        }
    } else {
        GDM_TIMED(ctx, "mixed_misc");
        hipLaunchKernelGGL(k_x0, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, slot(ctx, SL_HP).f,
                           rec ? hist(ctx, 0, 0) : X, mu, b / 4.0, 0.5, (const double*)nullptr, (const int*)nullptr);
    }
    GDM_LAUNCH_CHECK(ctx);
    const int ns = ctx->mixed_ns_inv;
    // the first nd - 1 doublings on the split products, the last in FP64
    for (int it = 0; it + 1 < nd; ++it) {
        const int* sk = dev ? dbl_skip + it : nullptr;
        const SplitMat Xk = rec ? hist(ctx, it, 0) : X;
        // X2 = X X ; A = 2 X2 - 2 X + I
        GDM_TRY(gemm(ctx, Xk, Xk, hl(X2), hl(A), hl(Xk), 2.0f, -2.0f, 1.0f, "foe_gemm", 1, pk, sk));
        // Newton-Schulz inverse of A (eigenvalues in [1/2, 1]) from the minimax
        // start (Rm and Yb hold the quartic start's A^2 and Q); each iteration
        // R = 2I - A Y, Y <- Y R squares the error
        SplitMat Y = (rec && ns == 0) ? hist(ctx, it, 1) : Ya;
        GDM_TRY(inv_start(ctx, A, Y, Rm, Yb, pk, sk));
        for (int k = 0; k < ns; ++k) {
            GDM_TRY(gemm(ctx, A, Y, none(), hl(Rm), none(), -1.0f, 0.0f, 2.0f, "foe_gemm", 1, pk, sk));
            const SplitMat Yn = (rec && k == ns - 1) ? hist(ctx, it, 1) : (Y.hi == Ya.hi ? Yb : Ya);
            GDM_TRY(gemm(ctx, Y, Rm, hl(Yn), none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, pk, sk));
            Y = Yn;
        }
        // X <- X2 Y
        const SplitMat Xn = rec ? hist(ctx, it + 1, 0) : hl(X);
        // the input of the FP64 doubling is written whole
        GDM_TRY(gemm(ctx, X2, Y, Xn, none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, it + 2 == nd ? (pk & 1) : pk,
                     sk));
    }
    // (the split halves: the FP32 copy of SL_X is written only by the FP64 doubling)
    GDM_TRY(last_doubling_f64(ctx, rec ? hist(ctx, nd - 1, 0) : hl(X), rec ? hist(ctx, nd - 1, 1) : none(),
                              pass_skip));
    if (rec) ctx->mixed_rec_nd = nd;
    return GDM_OK;
}

static double* z64(gdm_ctx* ctx) { return (double*)ctx->b[BUF_L].p + 2 * ctx->plan.tot2; }
// the transpose of the refined factor (FP64 region 8)
static double* z64t(gdm_ctx* ctx) { return (double*)ctx->b[BUF_L].p + 8 * ctx->plan.tot2; }

// FP64 products on all tiles (sym = 0) or on the upper tiles with mirrored
// output (sym = 1, symmetric products only)
template <typename TB>
static int gemm64_dd(gdm_ctx* ctx, const double* A, const TB* B, const double* Cin, double* C, double alpha,
                     double beta, double gamma, int sym, const int* skip = nullptr, const char* tag = "refine64",
                     G64Extra x64 = G64Extra{nullptr, 0.0, SplitMat{nullptr, nullptr, nullptr, 0}, 0.0, 0.0}) {
    GDM_TIMED(ctx, tag);
    const int4* tl = (const int4*)ctx->b[BUF_TILES].p + (sym ? ctx->mixed_tiles : 0);
    const unsigned nt = (unsigned)(sym ? ctx->mixed_tiles_sym : ctx->mixed_tiles);
    if (sym && x64.a_shift != 0.0)
        hipLaunchKernelGGL((k_gemm64<double, TB, true, true>), dim3(nt), dim3(256), 0, ctx->stream,
                           (const SubDesc*)ctx->b[BUF_DESC].p, tl, A, B, Cin, C, alpha, beta, gamma, skip, x64);
    else if (sym)
        hipLaunchKernelGGL((k_gemm64<double, TB, true>), dim3(nt), dim3(256), 0, ctx->stream,
                           (const SubDesc*)ctx->b[BUF_DESC].p, tl, A, B, Cin, C, alpha, beta, gamma, skip, x64);
    else
        hipLaunchKernelGGL((k_gemm64<double, TB, false>), dim3(nt), dim3(256), 0, ctx->stream,
                           (const SubDesc*)ctx->b[BUF_DESC].p, tl, A, B, Cin, C, alpha, beta, gamma, skip, x64);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

template <typename TB>
static int gemm64_core(gdm_ctx* ctx, const double* A, const TB* B, double* C, const char* tag,
                       const int* skip = nullptr) {
    GDM_TIMED(ctx, tag);
    const int4* tl = (const int4*)ctx->b[BUF_TILES].p + ctx->mixed_tiles + ctx->mixed_tiles_sym;
    hipLaunchKernelGGL((k_gemm64<double, TB, false>), dim3((unsigned)ctx->mixed_tiles_core), dim3(256), 0, ctx->stream,
                       (const SubDesc*)ctx->b[BUF_DESC].p, tl, A, B, (const double*)nullptr, C, 1.0, 0.0, 0.0, skip,
                       G64Extra{nullptr, 0.0, SplitMat{nullptr, nullptr, nullptr, 0}, 0.0, 0.0});
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

static double* fp64_region(gdm_ctx* ctx, int k) { return (double*)ctx->b[BUF_L].p + (int64_t)k * ctx->plan.tot2; }

// The last doubling of a pass in FP64 on the matrix cores (the final
// refinement step of the expansion): A = 2 X^2 - 2 X + I in FP64 (one
// product, which also writes A as split operands), Y = A^-1, and
// X <- X^2 Y = I/2 + (X - I/2) Y.  The inverse starts on the split products: A as split
// operands, the minimax start of the other doublings (the quartic of
// kInvStart4 with one split Newton-Schulz step by default, or the quadratic
// (420 I - 576 A + 256 A^2)/99 with two) leave I - A Y at the split
// products' rounding level
// (~1e-7 for FP16 pairs, ~1e-5 for BF16 pairs).  Then FP64 steps
// R = 2I - A Y, Y <- Y R: each maps I - A Y to (I - A Y)^2 exactly, for any
// Y, so one step (FP16 pairs) or two (BF16 pairs) leave ~1e-14 / ~1e-20,
// below the 3.6e-12 that three FP64 steps from Y0 = 4I - 5A + 2A^2 reached
// (a residual left after an exact step is a square, never negative, so it
// lowers every partly occupied state: ~1.9e-6 would bias the count by ~1e-3
// e at 80,000 electrons).  The doubling map is superattracting at 0 and 1,
// so the FP32-level errors of the split-product doublings in those states
// are squared away here instead of summing into a systematic bias of the
// electron count (~2e-8 per orbital), which would move mu inside a gap by
// that bias over N'(mu).  The result goes to SL_X (FP32 copy and split,
// whole) and, for the traces and the density, stays in FP64 region 5; a
// recorded pass also keeps the split Y for the response.  All matrices
// commute (polynomials in h_perp) up to the residual, so every product
// computes upper tiles and mirrors them (the asymmetry a mirrored Y R drops
// is of the order of the residual times the split error).
static int last_doubling_f64(gdm_ctx* ctx, SplitMat Xin, SplitMat Yrec, const int* skip) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    double* X = fp64_region(ctx, 5);        // the result
    double* Xi = fp64_region(ctx, 6);       // the input
    double* A = fp64_region(ctx, 7);
    double* Ya = fp64_region(ctx, 4);
    double* Yb = fp64_region(ctx, 3);
    double* R = fp64_region(ctx, 1);
    const int64_t n4 = P.tot2 / 4;
    {
        GDM_TIMED(ctx, "last64");
        hipLaunchKernelGGL(k_split_to_f64, dim3(4096), dim3(256), 0, ctx->stream, n4, Xin, Xi, skip);
    }
    GDM_LAUNCH_CHECK(ctx);
    // A = 2 X^2 - 2 X + I by one product, in FP64 and as split operands
    GDM_TRY(gemm64_dd(ctx, Xi, (const double*)Xi, Xi, A, 2.0, -2.0, 1.0, 1, skip, "last64",
                      G64Extra{nullptr, 0.0, slot(ctx, SL_A), 1.0, 0.0}));
    // split start and Newton-Schulz steps (whole storage: A comes whole)
    const SplitMat As = slot(ctx, SL_A), Rs = slot(ctx, SL_R), Ysa = slot(ctx, SL_Y), Ysb = slot(ctx, SL_YI);
    SplitMat Ys = Ysa;
    GDM_TRY(inv_start(ctx, As, Ys, Rs, Ysb, 0, skip));
    // FP16 pairs: the last split step also keeps its FP32 result Yf (in the FP32
    // copy of SL_X, free until this doubling's output), and Yf is the Y of the
    // FP64 steps below, read as FP32 operands (no FP64 copy of Y)
    const bool yf = P.precision != GDM_MIXED_BF16 && ctx->mixed_ns_inv > 0;
    float* Yf = slot(ctx, SL_X).f;
    for (int k = 0; k < ctx->mixed_ns_inv; ++k) {
        GDM_TRY(gemm(ctx, As, Ys, none(), hl(Rs), none(), -1.0f, 0.0f, 2.0f, "foe_gemm", 1, 0, skip));
        const SplitMat Yn = Ys.hi == Ysa.hi ? Ysb : Ysa;
        const SplitMat Yo = (yf && k + 1 == ctx->mixed_ns_inv) ? SplitMat{Yf, Yn.hi, Yn.lo, Yn.bf} : hl(Yn);
        GDM_TRY(gemm(ctx, Ys, Rs, Yo, none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, 0, skip));
        Ys = Yn;
    }
    if (!yf) {
        GDM_TIMED(ctx, "last64");
        hipLaunchKernelGGL(k_split_to_f64, dim3(4096), dim3(256), 0, ctx->stream, n4, hl(Ys), Ya, skip);
        GDM_LAUNCH_CHECK(ctx);
    }
    double* Y = Ya;
    const int final_ns = P.precision == GDM_MIXED_BF16 ? 2 : 1;
    for (int k = 0; k + 1 < final_ns; ++k) {
        GDM_TRY(gemm64_dd(ctx, A, Y, nullptr, R, -1.0, 0.0, 2.0, 1, skip, "last64"));   // R = 2I - A Y
        double* Yn = Y == Ya ? Yb : Ya;
        GDM_TRY(gemm64_dd(ctx, Y, R, nullptr, Yn, 1.0, 0.0, 0.0, 1, skip, "last64"));   // Y <- Y R
        Y = Yn;
    }
    // The last step as a correction, Y R = Y + Y rho with rho = I - A Y: only rho
    // needs FP64 (a residual of ~1e-7, ~1e-10 after an FP64 step for BF16 pairs);
    // Y rho needs ~1e-7 relative accuracy for an error of ~1e-14, which the split
    // products give.  rho leaves its FP64 product as split operands of
    // kLastSig rho (no FP64 copy), W = Y (kLastSig rho) on the split products
    // (with the split Y: it differs from the FP64 Y by ~1e-7 relative, which
    // changes Y rho by ~1e-14), and X2 (Y + W / kLastSig) is one FP64 product
    // whose B operand adds the correction as it is staged.
    const SplitMat W{slot(ctx, SL_Z2).f, nullptr, nullptr, 0};
    // X2 A^-1 = I/2 + (X - I/2) A^-1 (2 X^2 = A + 2 X - I): the product takes X
    // with I/2 subtracted on its diagonal as it is staged and adds I/2, so
    // neither X^2 nor X - I/2 is stored
    const G64Extra to_rho{nullptr, 0.0, hl(Rs), kLastSig, 0.0}, add_w{W.f, 1.0 / kLastSig, none(), 0.0, 0.5};
    if (yf)
        GDM_TRY(gemm64_dd(ctx, A, (const float*)Yf, nullptr, nullptr, -1.0, 0.0, 1.0, 1, skip, "last64", to_rho));
    else
        GDM_TRY(gemm64_dd(ctx, A, (const double*)Y, nullptr, nullptr, -1.0, 0.0, 1.0, 1, skip, "last64", to_rho));
    GDM_TRY(gemm(ctx, Ys, hl(Rs), W, none(), none(), 1.0f, 0.0f, 0.0f, "foe_gemm", 1, 0, skip));
    if (yf)       // X <- I/2 + (X - I/2)(Y + Y rho)
        GDM_TRY(gemm64_dd(ctx, Xi, (const float*)Yf, nullptr, X, 1.0, 0.0, 0.5, 1, skip, "last64", add_w));
    else
        GDM_TRY(gemm64_dd(ctx, Xi, (const double*)Y, nullptr, X, 1.0, 0.0, 0.5, 1, skip, "last64", add_w));
    GDM_TIMED(ctx, "last64");
    if (Yrec.hi) {
        if (yf)
            hipLaunchKernelGGL(k_copy_split, dim3(2048), dim3(256), 0, ctx->stream, n4, hl(Ys), Yrec, skip);
        else
            hipLaunchKernelGGL(k_z64_to_split, dim3(4096), dim3(256), 0, ctx->stream, n4, Y, Yrec, skip);
        GDM_LAUNCH_CHECK(ctx);
    }
    hipLaunchKernelGGL(k_z64_to_split, dim3(4096), dim3(256), 0, ctx->stream, n4, X, slot(ctx, SL_X), skip);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

// FP64 core traces of the last pass: N = 2 sum_core (Z X Z s)_aa and
// M = 2 sum_core (Z (X - X^2) Z s)_aa (the count's derivative is beta M),
// into the trace buffer's two scalars at 2 n_sub (enqueued only).
static int traces(gdm_ctx* ctx, const int* skip) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    double* part = (double*)ctx->b[BUF_TR].p;
    double* G = fp64_region(ctx, 1);
    double* G2 = fp64_region(ctx, 3);
    double* V = fp64_region(ctx, 0);
    const double* X = fp64_region(ctx, 5);       // X of the pass in FP64 (last_doubling_f64)
    GDM_TRY(gemm64_core<double>(ctx, z64(ctx), X, G, "traces", skip));
    GDM_TRY(gemm64_core<double>(ctx, G, X, G2, "traces", skip));     // Z[core,:] X^2 = G X
    GDM_TIMED(ctx, "traces");
    hipLaunchKernelGGL(k_trace_dot, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, G, G2, V, part, skip);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kEw), 0, ctx->stream, P.n_sub, part, part + 2 * (size_t)P.n_sub,
                       skip);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

static int read_state(gdm_ctx* ctx, double* h) {
    GDM_HIP(ctx, hipMemcpyAsync(h, mu_state(ctx), sizeof(double) * kStCount, hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GDM_OK;
}

int gdm_mixed_find_mu(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg, const int32_t* row_ptr,
                      const int32_t* col, int64_t nnz, const double* H, const double* S, double n_e, double kT,
                      double mu_guess, double tol_N, double* mu_out, double* n_out) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const bool dev = ctx->mu_out_device != 0;
    if (dev && ctx->mixed_rec_cap > 0)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_find_mu: the device-side mixed search does not record the expansion "
                                        "for the charge response (gdm_set_response(ctx, 0) first)");
    const double beta = 1.0 / kT;
    const int orth = S == nullptr;
    double* h64 = (double*)ctx->b[BUF_A].p;
    double* s64 = (double*)ctx->b[BUF_S].p;
    double* scale = (double*)ctx->b[BUF_NDBL].p;
    double* bounds = (double*)ctx->b[BUF_GERSH].p;
    double* st = mu_state(ctx);
    int* fl = mu_flags(ctx);
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
    auto ns_step = [&](bool full_z, const int* sk) -> int {
        GDM_TRY(gemm(ctx, Z, Y, none(), hl(T), none(), -0.5f, 0.0f, 1.5f, "ns_gemm", 1, pkz, sk));
        GDM_TRY(gemm(ctx, Y, T, hl(Y2), none(), none(), 1.0f, 0.0f, 0.0f, "ns_gemm", 1, pkz, sk));
        GDM_TRY(gemm(ctx, T, Z, full_z ? Z2 : hl(Z2), none(), none(), 1.0f, 0.0f, 0.0f, "ns_gemm", 1,
                     full_z ? (pkz & 1) : pkz, sk));
        return GDM_OK;
    };
    if (!orth) {
        // Y0 = (s/c) Z0 = a (s/c) + b (s/c)^2 (Z0 from k_prep)
        GDM_TRY(gemm(ctx, Y, Y, none(), hl(Y2), hl(Y), kZ0b, kZ0a, 0.0f, "ns_gemm", 1, pkz));
        std::swap(Y, Y2);
        for (int it = 0; it < ctx->mixed_ns_z; ++it) {
            GDM_TRY(ns_step(it + 1 == ctx->mixed_ns_z, nullptr));
            std::swap(Y, Y2);
            std::swap(Z, Z2);
        }
    }
    ctx->mixed_ns_z_used = orth ? 0 : ctx->mixed_ns_z;
    // FP64 residual refinement of Z (Z s Z = I): Z64 = Z / sqrt(c) in FP64,
    // F = s Z64, E = Z64 F - I, Z64 <- Z64 (I - E/2 + 3/8 E^2) (residual
    // O(E^3)); E and the update are symmetric products (upper tiles,
    // mirrored).  The refinement also removes any systematic bias of the split
    // products from Z64, which the electron count (and so mu) depends on.
    // While max |E_ij| is too large for one step, the coupled iteration
    // continues first: on
    // the host, or on the device through predicated extra rounds (each with
    // its iteration written back into the working slots).
    {
        double* F = fp64_region(ctx, 0);
        double* E = fp64_region(ctx, 1);
        double* Z64 = z64(ctx);
        double* emax_d = (double*)ctx->b[BUF_TR].p + 2 * (size_t)P.n_sub + 4;
        const int extras = std::min(ctx->mixed_ns_z_extra, kMaxNsExtra - 1);
        for (int extra = 0;; ++extra) {
            const int* sk = (dev && extra > 0) ? fl + kFlNs + extra : nullptr;
            if (dev && extra > 0 && !orth) {
                // one more coupled iteration, run only while the last round missed
                GDM_TRY(ns_step(true, sk));
                const int64_t n4 = P.tot2 / 4;
                hipLaunchKernelGGL(k_copy_split, dim3(2048), dim3(256), 0, ctx->stream, n4, hl(Y2), hl(Y), sk);
                GDM_LAUNCH_CHECK(ctx);
                hipLaunchKernelGGL(k_copy_split, dim3(2048), dim3(256), 0, ctx->stream, n4, Z2, Z, sk);
                GDM_LAUNCH_CHECK(ctx);
            }
            {
                GDM_TIMED(ctx, "refine64");
                hipLaunchKernelGGL(k_scale_sym_to_f64, dim3((unsigned)ctx->mixed_tiles_sym), dim3(256), 0, ctx->stream,
                                   desc, (const int4*)ctx->b[BUF_TILES].p + ctx->mixed_tiles, Z.f, scale, orth, Z64,
                                   sk);
            }
            GDM_LAUNCH_CHECK(ctx);
            if (orth) break;                                                  // Z = I exactly
            GDM_TRY(gemm64_dd(ctx, s64, Z64, nullptr, F, 1.0, 0.0, 0.0, 0, sk));     // F = s Z
            GDM_TRY(gemm64_dd(ctx, Z64, F, nullptr, E, 1.0, 0.0, -1.0, 1, sk));     // E = Z (s Z) - I
            {
                GDM_TIMED(ctx, "refine64");
                hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, ctx->stream, emax_d, sk);
                GDM_LAUNCH_CHECK(ctx);
                hipLaunchKernelGGL(k_resid_max, strip_grid(P), dim3(kEw), 0, ctx->stream, desc, E,
                                   (unsigned long long*)emax_d, hl(slot(ctx, SL_A)), kRefineSig, sk);
            }
            GDM_LAUNCH_CHECK(ctx);
            if (dev) {
                hipLaunchKernelGGL(k_resid_flag, dim3(1), dim3(64), 0, ctx->stream, emax_d, kZResidMax, extra,
                                   extra == extras ? 1 : 0, fl, ctx->d_status);
                GDM_LAUNCH_CHECK(ctx);
                if (extra == extras) break;
                ++ctx->mixed_ns_z_used;       // launched (the stats report those that ran)
                continue;
            }
            double emax = 0.0;
            GDM_HIP(ctx, hipMemcpyAsync(&emax, emax_d, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (emax <= kZResidMax) break;
            if (extra >= ctx->mixed_ns_z_extra || !std::isfinite(emax))
                return gdm_fail(ctx, GDM_E_NOT_CONVERGED,
                                "mixed: inverse-overlap factor residual %.3g after %d Newton-Schulz iterations "
                                "(overlap too ill-conditioned)", emax, ctx->mixed_ns_z_used);
            GDM_TRY(ns_step(true, nullptr));
            std::swap(Y, Y2);
            std::swap(Z, Z2);
            ++ctx->mixed_ns_z_used;
        }
        const SplitMat W{slot(ctx, SL_X).f, nullptr, nullptr, 0};
        if (!orth) {
            // third-order refinement Z1 = Z (I + E)^-1/2 = Z (I - E/2 + 3/8 E^2 + O(E^3)) with
            // E = Z s Z - I for the symmetric Z: T = 3/8 E^2 - E/2 is a polynomial in E, so
            // Z1^T s Z1 = (I + T)(I + E)(I + T) = I + O(E^3) holds exactly in algebra, whatever
            // the rounding errors of Z (which do not commute with s) are; Z1 itself is not
            // symmetric, so its product is formed on all tiles and the later steps use
            // Z1^T h Z1 and Z1 X Z1^T (D does not depend on which factor of s^-1 is used).
            // A symmetric step would leave those errors in place: Z s Z - I stays at the
            // FP32 level (1e-7) with a negative trace, a bias of the electron count.
            // Only E needs FP64 (a difference from I); the correction Z T is below
            // |E| <= 1e-3 (the guard) and needs ~1e-9 relative accuracy, which the split
            // products give: with sig E as split operands (written by k_resid_max, sig =
            // 2^16 keeping |E| down to 1e-9 in normal FP16), sig T = 3/(8 sig) (sig E)^2 -
            // (sig E)/2 and W = Z (sig T) on the split products, and
            // Z1 = Z64 + W / (sig sqrt(c)) in FP64 by the transpose pass below.  A rounding
            // error of T or W perturbs Z1^T s Z1 by its own size (~1e-13), not by |E|^2.
            const SplitMat Es = hl(slot(ctx, SL_A)), Ts = hl(slot(ctx, SL_R));
            GDM_TRY(gemm(ctx, Es, Es, none(), Ts, Es, (float)(0.375 / kRefineSig), -0.5f, 0.0f, "ns_gemm", 1, 0));
            GDM_TRY(gemm(ctx, Z, Ts, W, none(), none(), 1.0f, 0.0f, 0.0f, "ns_gemm", 0));
        }
        // Z1 into Z64 (in place), Z1^T in FP64 (the density's right factor) and as
        // split operands with an FP32 copy (the split products of h_perp and of the
        // response), in one pass
        Z = slot(ctx, SL_Z);
        {
            GDM_TIMED(ctx, "refine64");
            hipLaunchKernelGGL(k_transpose64, dim3((unsigned)ctx->mixed_tiles_sym), dim3(256), 0, ctx->stream, desc,
                               (const int4*)ctx->b[BUF_TILES].p + ctx->mixed_tiles, (const double*)Z64,
                               orth ? (double*)nullptr : Z64, orth ? (const float*)nullptr : (const float*)W.f, scale,
                               1.0 / kRefineSig, z64t(ctx), Z, (const int*)nullptr);
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
    // mu: safeguarded Newton steps on the FP64 traces (k_mu_update, the same
    // arithmetic whether the host or the device drives the passes)
    MuCfg cfg;
    cfg.n_e = n_e;
    cfg.beta = beta;
    cfg.kT = kT;
    cfg.tol = std::max(tol_N, 1e-10 * n_e);
    cfg.tol_final = std::max(tol_N, 1e-7 * n_e);
    cfg.guess = mu_guess;
    cfg.rec = ctx->mixed_rec_cap > 0;
    cfg.dev = dev;
    cfg.nd_launch = ctx->mixed_nd_launch;
    cfg.max_passes = dev ? ctx->mixed_dev_passes : std::min(ctx->mixed_max_passes, kMaxPasses);
    const double* part_nm = (const double*)ctx->b[BUF_TR].p + 2 * (size_t)P.n_sub;
    const int nb = (int)(P.n_sub * strip_grid(P).y);
    hipLaunchKernelGGL(k_mu_init, dim3(1), dim3(kEw), 0, ctx->stream, bounds, nb, dev ? mu_out : nullptr, cfg, st, fl,
                       ctx->d_status);
    GDM_LAUNCH_CHECK(ctx);
    double hs[kStCount];
    if (dev) {
        for (int p = 0; p < cfg.max_passes; ++p) {
            GDM_TRY(foe_pass(ctx, 0.0, 0.0, cfg.nd_launch, kStartSeptic, st, fl + kFlPass + p,
                             fl + kFlDbl + p * kMaxNd));
            GDM_TRY(traces(ctx, fl + kFlPass + p));
            hipLaunchKernelGGL(k_mu_update, dim3(1), dim3(64), 0, ctx->stream, p, cfg, part_nm, st, fl, ctx->d_status);
            GDM_LAUNCH_CHECK(ctx);
        }
        hipLaunchKernelGGL(k_mu_final, dim3(1), dim3(64), 0, ctx->stream, cfg, st, mu_out, n_out, ctx->d_status);
        GDM_LAUNCH_CHECK(ctx);
        ctx->mixed_passes = -1;             // on the device; gdm_mixed_stats reads them
        ctx->mixed_nd = -1;
        ctx->mixed_beta = beta;
        ctx->mixed_dev_state = true;
        return GDM_OK;
    }
    GDM_TRY(read_state(ctx, hs));
    for (int p = 0; p < cfg.max_passes; ++p) {
        GDM_TRY(foe_pass(ctx, hs[kStMu], hs[kStB], (int)hs[kStNd], (int)hs[kStStart], nullptr, nullptr, nullptr));
        GDM_TRY(traces(ctx, nullptr));
        hipLaunchKernelGGL(k_mu_update, dim3(1), dim3(64), 0, ctx->stream, p, cfg, part_nm, st, fl, ctx->d_status);
        GDM_LAUNCH_CHECK(ctx);
        const int nd_pass = (int)hs[kStNd];
        GDM_TRY(read_state(ctx, hs));
        ctx->mixed_nd = nd_pass;
        if (hs[kStDone] != 0.0) break;
    }
    ctx->mixed_dev_state = false;
    ctx->mixed_passes = (int)hs[kStPasses];
    ctx->mixed_mu_pass = hs[kStMuPass];
    ctx->mixed_slope = beta * hs[kStM];
    ctx->mixed_beta = beta;
    *mu_out = hs[kStMuOut];
    *n_out = hs[kStNOut];
    return GDM_OK;
}

// mu_dev: when non-null, mu is read on the device (a device-side search's
// result) and the first-order term uses the device state's pass mu
int gdm_mixed_density(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, const double* mu_dev, double kT,
                      double* D_core) {
    const Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const double beta = 1.0 / kT;
    const double kappa = mu_dev ? 0.0 : (mu - ctx->mixed_mu_pass) * beta;
    double* G = fp64_region(ctx, 1);
    double* G2 = fp64_region(ctx, 3);
    double* Gk = fp64_region(ctx, 0);
    double* Dp = fp64_region(ctx, 4);
    // D[core,:] = (G + kappa (G - G2)) Z,  G = Z[core,:] X, G2 = Z[core,:] X^2 of the last pass
    {
        GDM_TIMED(ctx, "dcore");
        hipLaunchKernelGGL(k_combine, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, G, G, G2, Gk, kappa, mu_dev,
                           (const double*)mu_state(ctx), beta);
    }
    GDM_LAUNCH_CHECK(ctx);
    GDM_TRY(gemm64_core<double>(ctx, Gk, z64t(ctx), Dp, "dcore"));      // D[core,:] = G Z1^T
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
    if (ctx->mixed_rec_cap <= 0 || !gdm_is_mixed(P.precision) || P.n_sub <= 0) {
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
        hipLaunchKernelGGL(k_trace_dot, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, Gd, Gd, R0, part,
                           (const int*)nullptr);
        GDM_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kEw), 0, ctx->stream, P.n_sub, part,
                           part + 2 * (size_t)P.n_sub, (const int*)nullptr);
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
        hipLaunchKernelGGL(k_combine, dim3(P.n_sub), dim3(256), 0, ctx->stream, desc, Gd, G, G2, Gd, kappa,
                           (const double*)nullptr, (const double*)nullptr, 0.0);
    }
    GDM_LAUNCH_CHECK(ctx);
    GDM_TRY(gemm64_core<double>(ctx, Gd, z64t(ctx), R1, "response"));
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

extern "C" int gdm_set_mixed_inverse_start(gdm_ctx* ctx, int degree) {
    if (!ctx) return GDM_E_ARG;
    if (degree != 2 && degree != 4)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_set_mixed_inverse_start: degree must be 2 or 4");
    ctx->mixed_inv_deg = degree;
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

extern "C" int gdm_set_mixed_capture(gdm_ctx* ctx, int passes, int nd_launch) {
    if (!ctx) return GDM_E_ARG;
    if (passes < 1 || passes > kMaxPasses || nd_launch < 5 || nd_launch > kMaxNd)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_set_mixed_capture: passes 1..%d, nd_launch 5..%d", kMaxPasses, kMaxNd);
    ctx->mixed_dev_passes = passes;
    ctx->mixed_nd_launch = nd_launch;
    return GDM_OK;
}

extern "C" int gdm_mixed_mu_state(gdm_ctx* ctx, double* mu_pass, double* n_pass, double* slope) {
    if (!ctx) return GDM_E_ARG;
    if (!gdm_is_mixed(ctx->plan.precision) || !ctx->b[BUF_MSTATE].p)
        return gdm_fail(ctx, GDM_E_STATE, "gdm_mixed_mu_state: no mixed plan");
    double hs[kStCount];
    GDM_TRY(read_state(ctx, hs));
    if (mu_pass) *mu_pass = hs[kStMuPass];
    if (n_pass) *n_pass = hs[kStN];
    if (slope) *slope = ctx->mixed_beta * hs[kStM];
    return GDM_OK;
}

// pass mu of the last search (read from the device after a device-side one)
int gdm_mixed_pass_mu(gdm_ctx* ctx, double* mu_pass) {
    if (!ctx->mixed_dev_state) {
        *mu_pass = ctx->mixed_mu_pass;
        return GDM_OK;
    }
    double hs[kStCount];
    GDM_TRY(read_state(ctx, hs));
    *mu_pass = hs[kStMuPass];
    return GDM_OK;
}

extern "C" int gdm_mixed_stats(gdm_ctx* ctx, int* passes, int* n_doublings, int64_t* gemm_launches,
                               double* flops_per_launch, double* bytes_per_launch, int* ns_z_used) {
    if (!ctx) return GDM_E_ARG;
    if (ctx->mixed_dev_state && ctx->b[BUF_MSTATE].p) {
        double hs[kStCount];
        GDM_TRY(read_state(ctx, hs));
        ctx->mixed_passes = (int)hs[kStPasses];
        ctx->mixed_nd = (int)hs[kStNd];
    }
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
    if (!gdm_is_mixed(P.precision) || which < 0 || which >= 3 || sub < 0 || sub >= P.n_sub || !out)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_debug_slot: bad argument");
    const SubDesc& d = P.desc[sub];
    GDM_HIP(ctx, hipMemcpyAsync(out, slot(ctx, kDebugSlots[which]).f + d.off2, sizeof(float) * (size_t)d.ld * d.ld,
                                hipMemcpyDeviceToDevice, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GDM_OK;
}
