// Self-consistent-charge shell and the learned starting charges.
//
// SCC (SI section D; the scaled-delta kernel K = -c I of the Shadow MD
// section is the linear mixer): V_I = U_I q_I + k_e sum_J q_J psi(R_J - R_I)
// with the Ewald split psi = real-space erfc(eta r)/r over a cutoff CSR +
// reciprocal sum over k != 0 + self term -2 eta / sqrt(pi); mixing
// n <- n + c (q0[n] - n).
//
// Learned guess: per-atom radial descriptors (16 Gaussians x 2 neighbour
// species), one 32-64-64-1 SiLU network per central species, prediction
// shifted to zero net charge.  FP32 training kernels (forward, loss,
// backward with a deterministic block-partial reduction, Adam) and a BF16
// inference forward (BF16 weights, inputs and activations, FP32
// accumulation).
#include "gdm_internal.h"

#include <cmath>
#include <mutex>

namespace {

constexpr int kNR = 16;            // Gaussians per species
constexpr int kNF = 32;            // features
constexpr int kH = 64;             // hidden width
constexpr int kNP = kH * kNF + kH + kH * kH + kH + kH + 1;   // 6337 parameters per network
constexpr int kOffB1 = kH * kNF;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;

__device__ __forceinline__ void min_image(const double* pos, int i, int j, double3 L, double3 iL, double* dx,
                                          double* dy, double* dz) {
    double x = pos[3 * j] - pos[3 * i], y = pos[3 * j + 1] - pos[3 * i + 1], z = pos[3 * j + 2] - pos[3 * i + 2];
    x -= L.x * rint(x * iL.x);
    y -= L.y * rint(y * iL.y);
    z -= L.z * rint(z * iL.z);
    *dx = x;
    *dy = y;
    *dz = z;
}

// ---------------------------------------------------------------- descriptors
__global__ void k_descriptors(int n, const double* __restrict__ pos, const int32_t* __restrict__ species,
                              double3 L, double3 iL, const int32_t* __restrict__ rp, const int32_t* __restrict__ cl,
                              double rcut, double width, double c0, double dc, double* __restrict__ feats) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a0[kNR], a1[kNR];
#pragma unroll
    for (int q = 0; q < kNR; ++q) a0[q] = a1[q] = 0.0;
    const double inv2w2 = 1.0 / (2.0 * width * width);
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int j = cl[k];
        double dx, dy, dz;
        min_image(pos, i, j, L, iL, &dx, &dy, &dz);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (!(r < rcut)) continue;
        const double fc = 0.5 * (cos(M_PI * r / rcut) + 1.0);
        const double w0 = species[j] == 0 ? fc : 0.0, w1 = fc - w0;
#pragma unroll
        for (int q = 0; q < kNR; ++q) {
            const double t = r - (c0 + q * dc);
            const double g = exp(-t * t * inv2w2);
            a0[q] += g * w0;
            a1[q] += g * w1;
        }
    }
    double* out = feats + (int64_t)i * kNF;
#pragma unroll
    for (int q = 0; q < kNR; ++q) {
        out[q] = a0[q];
        out[kNR + q] = a1[q];
    }
}

// Per-species feature sums for standardisation, stats[(s*3 + m)*32 + f]:
// m = 0 count, 1 sum, 2 sum of squares.  Block = 32 threads (one feature
// each); blocks stride over atoms and add their partials atomically.
__global__ void k_feature_sums(int n, const double* __restrict__ feats, const int32_t* __restrict__ species,
                               double* __restrict__ stats) {
    const int f = threadIdx.x;
    if (f >= kNF) return;
    double c[2] = {0, 0}, s1[2] = {0, 0}, s2[2] = {0, 0};
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int sp = species[i] != 0;
        const double x = feats[(int64_t)i * kNF + f];
        c[sp] += 1.0;
        s1[sp] += x;
        s2[sp] += x * x;
    }
    for (int sp = 0; sp < 2; ++sp) {
        atomicAdd(&stats[(sp * 3 + 0) * kNF + f], c[sp]);
        atomicAdd(&stats[(sp * 3 + 1) * kNF + f], s1[sp]);
        atomicAdd(&stats[(sp * 3 + 2) * kNF + f], s2[sp]);
    }
}

// norm[s][0..31] = mean, norm[s][32..63] = max(std, 1e-6) (population std)
__global__ void k_feature_norm(const double* __restrict__ stats, float* __restrict__ norm) {
    const int t = threadIdx.x;
    if (t >= 2 * kNF) return;
    const int sp = t / kNF, f = t % kNF;
    const double c = stats[(sp * 3 + 0) * kNF + f];
    const double mean = c > 0 ? stats[(sp * 3 + 1) * kNF + f] / c : 0.0;
    const double var = c > 0 ? stats[(sp * 3 + 2) * kNF + f] / c - mean * mean : 0.0;
    norm[sp * 2 * kNF + f] = (float)mean;
    norm[sp * 2 * kNF + kNF + f] = (float)fmax(sqrt(fmax(var, 0.0)), 1e-6);
}

// ---------------------------------------------------------------------- MLP
__device__ __forceinline__ float silu(float x) { return x / (1.0f + expf(-x)); }
__device__ __forceinline__ float dsilu(float x) {
    const float s = 1.0f / (1.0f + expf(-x));
    return s * (1.0f + x * (1.0f - s));
}

template <bool BF16>
__device__ __forceinline__ float rnd(float x) {
    if (!BF16) return x;
    return (float)(__bf16)x;
}

// y_i = net_{species_i}(x_i) for every atom; both networks and both feature
// normalisations staged in LDS (weights read as wave-wide broadcasts).
template <bool BF16>
__global__ void __launch_bounds__(256) k_mlp_forward(int n, const int32_t* __restrict__ species,
                                                    const double* __restrict__ feats,
                                                    const float* __restrict__ params, const float* __restrict__ norm,
                                                    float* __restrict__ y) {
    __shared__ float w[2 * kNP];
    __shared__ float nm[4 * kNF];
    for (int k = threadIdx.x; k < 2 * kNP; k += 256) w[k] = rnd<BF16>(params[k]);
    for (int k = threadIdx.x; k < 4 * kNF; k += 256) nm[k] = norm[k];
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int sp = species[i] != 0;
    const float* W = w + sp * kNP;
    const float* N = nm + sp * 2 * kNF;
    float x[kNF];
    for (int f = 0; f < kNF; ++f) x[f] = rnd<BF16>(((float)feats[(int64_t)i * kNF + f] - N[f]) / N[kNF + f]);
    float h1[kH];
    for (int j = 0; j < kH; ++j) {
        float acc = W[kOffB1 + j];
        for (int f = 0; f < kNF; ++f) acc = fmaf(W[j * kNF + f], x[f], acc);
        h1[j] = rnd<BF16>(silu(acc));
    }
    float out = W[kOffB3];
    for (int j = 0; j < kH; ++j) {
        float acc = W[kOffB2 + j];
        for (int k = 0; k < kH; ++k) acc = fmaf(W[kOffW2 + j * kH + k], h1[k], acc);
        out = fmaf(W[kOffW3 + j], rnd<BF16>(silu(acc)), out);
    }
    y[i] = out;
}

__device__ double block_sum_1024(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// residual statistics over all n atoms (one block of 1024):
// out[0] = mean(y), out[1] = mean(r), out[2] = mean(r^2), r = y - mean(y) - q_ref
__global__ void __launch_bounds__(1024) k_loss(int n, const float* __restrict__ y, const double* __restrict__ qref,
                                              double* __restrict__ out) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += (double)y[i];
    const double ybar = block_sum_1024(s, red) / n;
    double sr = 0.0, sr2 = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double r = (double)y[i] - ybar - qref[i];
        sr += r;
        sr2 += r * r;
    }
    const double rbar = block_sum_1024(sr, red) / n;
    const double l = block_sum_1024(sr2, red) / n;
    if (threadIdx.x == 0) {
        out[0] = ybar;
        out[1] = rbar;
        out[2] = l;
    }
}

// neutral charges q = y - mean(y) in FP64 (one block of 1024)
__global__ void __launch_bounds__(1024) k_center(int n, const float* __restrict__ y, double* __restrict__ q) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += (double)y[i];
    const double ybar = block_sum_1024(s, red) / n;
    for (int i = threadIdx.x; i < n; i += 1024) q[i] = (double)y[i] - ybar;
}

// Backward over a block of 64 consecutive atoms: activations of each atom
// with its own species' network in LDS, then each thread accumulates its
// share of both networks' parameter gradients over the block (atoms of the
// other species contribute nothing) into partial[block][2][kNP]; the blocks
// are summed in a fixed order by k_reduce_partials.
constexpr int kBA = 64;

__global__ void __launch_bounds__(256) k_mlp_backward(int n, const int32_t* __restrict__ species,
                                                     const double* __restrict__ feats,
                                                     const float* __restrict__ params,
                                                     const float* __restrict__ norm, const float* __restrict__ y,
                                                     const double* __restrict__ qref, const double* __restrict__ st,
                                                     double scale, float* __restrict__ partial) {
    __shared__ float sx[kBA][kNF + 1];
    __shared__ float sa1[kBA][kH + 1];    // silu(z1)
    __shared__ float sz1[kBA][kH + 1];
    __shared__ float sa2[kBA][kH + 1];    // silu(z2)
    __shared__ float sd2[kBA][kH + 1];
    __shared__ float sd1[kBA][kH + 1];
    __shared__ float sg[kBA];
    __shared__ int ssp[kBA];
    const int t = threadIdx.x;
    const int a0 = blockIdx.x * kBA;
    const int na = min(kBA, n - a0);
    for (int a = t; a < kBA; a += 256) {
        float g = 0.f;
        int sp = 0;
        if (a < na) {
            const int i = a0 + a;
            sp = species[i] != 0;
            const double r = (double)y[i] - st[0] - qref[i];
            g = (float)(scale * (r - st[1]));
        }
        sg[a] = g;
        ssp[a] = sp;
    }
    __syncthreads();
    for (int e = t; e < kBA * kNF; e += 256) {
        const int a = e / kNF, f = e % kNF;
        const float* N = norm + ssp[a] * 2 * kNF;
        sx[a][f] = a < na ? ((float)feats[(int64_t)(a0 + a) * kNF + f] - N[f]) / N[kNF + f] : 0.f;
    }
    __syncthreads();
    for (int e = t; e < kBA * kH; e += 256) {           // z1 = W1 x + b1
        const int a = e / kH, j = e % kH;
        const float* W = params + ssp[a] * kNP;
        float acc = W[kOffB1 + j];
        for (int f = 0; f < kNF; ++f) acc = fmaf(W[j * kNF + f], sx[a][f], acc);
        sz1[a][j] = acc;
        sa1[a][j] = silu(acc);
    }
    __syncthreads();
    for (int e = t; e < kBA * kH; e += 256) {           // z2, d2 = g W3 silu'(z2)
        const int a = e / kH, j = e % kH;
        const float* W = params + ssp[a] * kNP;
        float acc = W[kOffB2 + j];
        for (int k = 0; k < kH; ++k) acc = fmaf(W[kOffW2 + j * kH + k], sa1[a][k], acc);
        sa2[a][j] = silu(acc);
        sd2[a][j] = sg[a] * W[kOffW3 + j] * dsilu(acc);
    }
    __syncthreads();
    for (int e = t; e < kBA * kH; e += 256) {           // d1 = (W2^T d2) silu'(z1)
        const int a = e / kH, k = e % kH;
        const float* W = params + ssp[a] * kNP;
        float acc = 0.f;
        for (int j = 0; j < kH; ++j) acc = fmaf(W[kOffW2 + j * kH + k], sd2[a][j], acc);
        sd1[a][k] = acc * dsilu(sz1[a][k]);
    }
    __syncthreads();
    float* gp = partial + (int64_t)blockIdx.x * 2 * kNP;
    for (int pp = t; pp < 2 * kNP; pp += 256) {
        const int sp = pp / kNP, p = pp % kNP;
        float acc = 0.f;
        if (p < kOffB1) {                       // W1[j][f]
            const int j = p / kNF, f = p % kNF;
            for (int a = 0; a < kBA; ++a)
                if (ssp[a] == sp) acc = fmaf(sd1[a][j], sx[a][f], acc);
        } else if (p < kOffW2) {                // b1
            const int j = p - kOffB1;
            for (int a = 0; a < kBA; ++a)
                if (ssp[a] == sp) acc += sd1[a][j];
        } else if (p < kOffB2) {                // W2[j][k]
            const int q = p - kOffW2, j = q / kH, k = q % kH;
            for (int a = 0; a < kBA; ++a)
                if (ssp[a] == sp) acc = fmaf(sd2[a][j], sa1[a][k], acc);
        } else if (p < kOffW3) {                // b2
            const int j = p - kOffB2;
            for (int a = 0; a < kBA; ++a)
                if (ssp[a] == sp) acc += sd2[a][j];
        } else if (p < kOffB3) {                // W3[j]
            const int j = p - kOffW3;
            for (int a = 0; a < kBA; ++a)
                if (ssp[a] == sp) acc = fmaf(sg[a], sa2[a][j], acc);
        } else {                                // b3
            for (int a = 0; a < kBA; ++a)
                if (ssp[a] == sp) acc += sg[a];
        }
        gp[pp] = acc;
    }
}

__global__ void k_reduce_partials(int nblocks, const float* __restrict__ partial, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= 2 * kNP) return;
    float acc = 0.f;
    for (int b = 0; b < nblocks; ++b) acc += partial[(int64_t)b * 2 * kNP + p];
    grad[p] = acc;
}

__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ Ewald
// S(R) of the screened interaction gamma = 1/R - S: Coulomb energy of two
// unit exponential densities tau^3/(8 pi) exp(-tau r) (Slater 1s), closed
// form in any length unit (tau in 1/length, S in 1/length).
__device__ double slater_short(double ta, double tb, double R) {
    if (fabs(ta - tb) < 1e-6 * (ta + tb)) {
        const double t = 0.5 * (ta + tb);
        return exp(-t * R) * (1.0 / R + 11.0 * t / 16.0 + 3.0 * t * t * R / 16.0 + t * t * t * R * R / 48.0);
    }
    const double a2 = ta * ta, b2 = tb * tb;
    const double dab = a2 - b2, dba = -dab;
    const double pa = exp(-ta * R) * (b2 * b2 * ta / (2.0 * dab * dab) - (b2 * b2 * b2 - 3.0 * b2 * b2 * a2) / (dab * dab * dab * R));
    const double pb = exp(-tb * R) * (a2 * a2 * tb / (2.0 * dba * dba) - (a2 * a2 * a2 - 3.0 * a2 * a2 * b2) / (dba * dba * dba * R));
    return pa + pb;
}

// real space over the cutoff CSR (r < rc): sum_J q_J (erfc(eta r)/r - S(tau_I, tau_J, r)),
// the screening term only when screened != 0.  One wave per atom: the lanes
// take every 64th pair of its row (rows hold hundreds of pairs at 12 A), then
// a wave sum, so a launch has as many waves as atoms.
constexpr int kRealAtoms = 4;      // atoms (waves) per workgroup
__global__ void __launch_bounds__(64 * kRealAtoms) k_ewald_real(int n, const double* __restrict__ pos,
                                                                const int32_t* __restrict__ species, double3 L,
                                                                double3 iL, const int32_t* __restrict__ rp,
                                                                const int32_t* __restrict__ cl, double rc, double eta,
                                                                int screened, double tau0, double tau1,
                                                                const double* __restrict__ q, double* __restrict__ V) {
    const int i = blockIdx.x * kRealAtoms + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= n) return;                 // uniform over the wave
    const double ti = species[i] == 0 ? tau0 : tau1;
    double acc = 0.0;
    for (int k = rp[i] + lane; k < rp[i + 1]; k += 64) {
        const int j = cl[k];
        double dx, dy, dz;
        min_image(pos, i, j, L, iL, &dx, &dy, &dz);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (!(r < rc)) continue;
        double g = erfc(eta * r) / r;
        if (screened) g -= slater_short(ti, species[j] == 0 ? tau0 : tau1, r);
        acc += q[j] * g;
    }
    acc = gdm_wave_sum(acc);
    if (lane == 0) V[i] = acc;
}

// structure factors over the half space of k-vectors: C(k) = sum q cos(k.R), S(k) = sum q sin(k.R)
__global__ void __launch_bounds__(256) k_ewald_sk(int n, const double* __restrict__ pos,
                                                 const double* __restrict__ q, const double4* __restrict__ kv,
                                                 double* __restrict__ CS) {
    __shared__ double rc_[256], rs_[256];
    const double4 k = kv[blockIdx.x];
    if (k.w == 0.0) {          // outside the k sphere (full-grid table): no contribution
        if (threadIdx.x == 0) {
            CS[2 * blockIdx.x] = 0.0;
            CS[2 * blockIdx.x + 1] = 0.0;
        }
        return;
    }
    double c = 0.0, s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        const double ph = k.x * pos[3 * j] + k.y * pos[3 * j + 1] + k.z * pos[3 * j + 2];
        double sn, cs;
        sincos(ph, &sn, &cs);
        c += q[j] * cs;
        s += q[j] * sn;
    }
    rc_[threadIdx.x] = c;
    rs_[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            rc_[threadIdx.x] += rc_[threadIdx.x + o];
            rs_[threadIdx.x] += rs_[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        CS[2 * blockIdx.x] = rc_[0];
        CS[2 * blockIdx.x + 1] = rs_[0];
    }
}

// V_I = U_I q_I + ke [ real_I + 2 sum_{k in half space} w(k) (cos(k.R_I) C + sin(k.R_I) S) - 2 eta/sqrt(pi) q_I ]
// with w(k) = (4 pi / V) exp(-k^2 / 4 eta^2) / k^2 stored in kv[].w
__global__ void k_ewald_recip(int n, int nk, const double* __restrict__ pos, const int32_t* __restrict__ species,
                              const double* __restrict__ q, const double4* __restrict__ kv,
                              const double* __restrict__ CS, double eta, double ke, double U0, double U1,
                              double* __restrict__ V) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < nk; ++k) {
        const double4 kk = kv[k];
        if (kk.w == 0.0) continue;          // uniform over the wave
        const double ph = kk.x * pos[3 * i] + kk.y * pos[3 * i + 1] + kk.z * pos[3 * i + 2];
        double sn, cs;
        sincos(ph, &sn, &cs);
        acc += kk.w * (cs * CS[2 * k] + sn * CS[2 * k + 1]);
    }
    const double self = -2.0 * eta / sqrt(M_PI) * q[i];
    V[i] = (species[i] == 0 ? U0 : U1) * q[i] + ke * (V[i] + 2.0 * acc + self);
}

// V_I from the real-space part already in V and the chunks of the
// reciprocal sum (k_ewald_recip_lines), added in chunk order
__global__ void k_ewald_finish(int n, int nchunk, const double* __restrict__ part,
                               const int32_t* __restrict__ species, const double* __restrict__ q, double eta,
                               double ke, double U0, double U1, double* __restrict__ V) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int y = 0; y < nchunk; ++y) acc += part[(int64_t)y * n + i];
    const double self = -2.0 * eta / sqrt(M_PI) * q[i];
    V[i] = (species[i] == 0 ? U0 : U1) * q[i] + ke * (V[i] + 2.0 * acc + self);
}

// Structure factors and reciprocal sums over lines of the full k grid
// (k_ewald_ktable order: line (a, b) holds c = -K..K, consecutive kz apart by
// dkz = 2 pi / Lz).  Along a line the phase advances by the same factor
// e^{i dkz z}, so e^{i k.R} of the next point is one complex product away:
// one sincos per atom for a line's (or block's) first point and one for the
// step, instead of one per point.  Points of weight 0 (outside the sphere or
// the half space) contribute nothing.

// a line is non-empty iff its c = 0 point is inside (that point has the
// smallest |k| of the line), or it is the line a = b = 0 (c > 0 only)
__device__ __forceinline__ bool line_live(const double4* __restrict__ kv, int line, int K) {
    const int w = 2 * K + 1;
    return kv[line * w + K].w != 0.0 || line == K;
}

// C(k), S(k) of NQ charge vectors for C consecutive points of one line per
// workgroup (the phases are shared by the vectors)
template <int NQ, int C>
__global__ void __launch_bounds__(256) k_ewald_sk_lines(int n, int K, const double* __restrict__ pos,
                                                       const double* __restrict__ q0, const double* __restrict__ q1,
                                                       const double4* __restrict__ kv, double dkz,
                                                       double* __restrict__ CS0, double* __restrict__ CS1) {
    __shared__ double red[4][2 * C * NQ];
    const int w = 2 * K + 1, nb = (w + C - 1) / C;
    const int line = blockIdx.x / nb, g0 = line * w + (blockIdx.x % nb) * C;
    const int cnt = min(C, line * w + w - g0);
    bool any = false;
    for (int t = 0; t < cnt; ++t) any = any || kv[g0 + t].w != 0.0;
    if (!any) {
        if (threadIdx.x < 2 * cnt) {
            CS0[2 * (int64_t)g0 + threadIdx.x] = 0.0;
            if (NQ == 2) CS1[2 * (int64_t)g0 + threadIdx.x] = 0.0;
        }
        return;
    }
    const double4 k0 = kv[g0];
    double ac[NQ][C], as[NQ][C];
#pragma unroll
    for (int v = 0; v < NQ; ++v)
#pragma unroll
        for (int t = 0; t < C; ++t) ac[v][t] = as[v][t] = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        const double x = pos[3 * j], y = pos[3 * j + 1], z = pos[3 * j + 2];
        double qj[NQ];
        qj[0] = q0[j];
        if (NQ == 2) qj[NQ - 1] = q1[j];
        double sn, cs, sd, cd;
        sincos(k0.x * x + k0.y * y + k0.z * z, &sn, &cs);
        sincos(dkz * z, &sd, &cd);
#pragma unroll
        for (int t = 0; t < C; ++t) {
#pragma unroll
            for (int v = 0; v < NQ; ++v) {
                ac[v][t] += qj[v] * cs;
                as[v][t] += qj[v] * sn;
            }
            const double c2 = cs * cd - sn * sd;
            sn = sn * cd + cs * sd;
            cs = c2;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NQ; ++v)
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const double c = gdm_wave_sum(ac[v][t]), sv = gdm_wave_sum(as[v][t]);
            if (lane == 0) {
                red[wave][2 * (v * C + t)] = c;
                red[wave][2 * (v * C + t) + 1] = sv;
            }
        }
    __syncthreads();
    if (threadIdx.x < 2 * cnt * NQ) {
        const int v = threadIdx.x / (2 * cnt), e = threadIdx.x - v * 2 * cnt, t = e >> 1;
        const int slot = 2 * (v * C + t) + (e & 1);
        const double val = red[0][slot] + red[1][slot] + red[2][slot] + red[3][slot];
        (v == 0 ? CS0 : CS1)[2 * (int64_t)g0 + e] = kv[g0 + t].w != 0.0 ? val : 0.0;
    }
}
constexpr int kSkC = 16;       // points per workgroup, one charge vector
constexpr int kSkC2 = 8;       // points per workgroup, two charge vectors

// part[y * n + i] = sum over the lines of chunk y of w(k) (cos(k.R_i) C + sin(k.R_i) S)
__global__ void __launch_bounds__(128) k_ewald_recip_lines(int n, int K, int lines_per_chunk,
                                                          const double* __restrict__ pos,
                                                          const double4* __restrict__ kv,
                                                          const double* __restrict__ CS, double dkz,
                                                          double* __restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int w = 2 * K + 1, nlines = (K + 1) * w;
    const int l0 = blockIdx.y * lines_per_chunk, l1 = min(nlines, l0 + lines_per_chunk);
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    double sd, cd;
    sincos(dkz * z, &sd, &cd);
    double acc = 0.0;
    for (int line = l0; line < l1; ++line) {
        if (!line_live(kv, line, K)) continue;          // uniform over the wave
        const int g0 = line * w;
        const double4 k0 = kv[g0];
        double sn, cs;
        sincos(k0.x * x + k0.y * y + k0.z * z, &sn, &cs);
        for (int c = 0; c < w; ++c) {
            const double wk = kv[g0 + c].w;
            acc += wk * (cs * CS[2 * (int64_t)(g0 + c)] + sn * CS[2 * (int64_t)(g0 + c) + 1]);
            const double c2 = cs * cd - sn * sd;
            sn = sn * cd + cs * sd;
            cs = c2;
        }
    }
    part[(int64_t)blockIdx.y * n + i] = acc;
}

// the force's reciprocal part over the lines of chunk blockIdx.y:
// part[(y * n + i) * 3 + x] = sum_k w_k k_x [a_i (S_b cos - C_b sin) + b_i (S_a cos - C_a sin)]
__global__ void __launch_bounds__(128) k_ewald_force_recip_lines(int n, int K, int lines_per_chunk,
                                                                const double* __restrict__ pos,
                                                                const double* __restrict__ qa,
                                                                const double* __restrict__ qb,
                                                                const double4* __restrict__ kv,
                                                                const double* __restrict__ CSa,
                                                                const double* __restrict__ CSb, double dkz,
                                                                double* __restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int w = 2 * K + 1, nlines = (K + 1) * w;
    const int l0 = blockIdx.y * lines_per_chunk, l1 = min(nlines, l0 + lines_per_chunk);
    const double ai = qa[i], bi = qb[i];
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    double sd, cd;
    sincos(dkz * z, &sd, &cd);
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int line = l0; line < l1; ++line) {
        if (!line_live(kv, line, K)) continue;
        const int g0 = line * w;
        const double4 k0 = kv[g0];
        double sn, cs;
        sincos(k0.x * x + k0.y * y + k0.z * z, &sn, &cs);
        double tx = 0.0, tz = 0.0;       // sum of t and of t kz over the line
        for (int c = 0; c < w; ++c) {
            const double4 kk = kv[g0 + c];
            const int64_t e = 2 * (int64_t)(g0 + c);
            const double t = kk.w * (ai * (CSb[e + 1] * cs - CSb[e] * sn) + bi * (CSa[e + 1] * cs - CSa[e] * sn));
            tx += t;
            tz += t * kk.z;
            const double c2 = cs * cd - sn * sd;
            sn = sn * cd + cs * sd;
            cs = c2;
        }
        gx += tx * k0.x;
        gy += tx * k0.y;
        gz += tz;
    }
    double* o = part + ((int64_t)blockIdx.y * n + i) * 3;
    o[0] = gx;
    o[1] = gy;
    o[2] = gz;
}

// k-vector table over the full grid a = 0..K, b, c = -K..K (index
// (a (2K+1) + b + K) (2K+1) + c + K): weight w(k) inside the half space
// (a > 0) or (a = 0, b > 0) or (a = b = 0, c > 0) and the sphere k^2 <= kc2,
// 0 outside (those points contribute nothing to the structure factors and
// reciprocal sums that read the table).
__global__ void k_ewald_ktable(int K, double Lx, double Ly, double Lz, double eta, double kc2, double V3,
                               double4* __restrict__ kv) {
    const int w = 2 * K + 1;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (K + 1) * w * w) return;
    const int a = g / (w * w), b = (g / w) % w - K, c = g % w - K;
    const double kx = 2 * M_PI * a / Lx, ky = 2 * M_PI * b / Ly, kz = 2 * M_PI * c / Lz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    double wt = 0.0;
    if (!(a == 0 && (b < 0 || (b == 0 && c <= 0))) && !(k2 > kc2))
        wt = 4.0 * M_PI / V3 * exp(-k2 / (4.0 * eta * eta)) / k2;
    kv[g] = make_double4(kx, ky, kz, wt);
}

// n <- n + c (q0 - n); partial sums of (q0 - n)^2 per block
__global__ void k_mix(int n, double* __restrict__ nv, const double* __restrict__ q0, double c,
                      double* __restrict__ part) {
    __shared__ double red[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double r2 = 0.0;
    if (i < n) {
        const double r = q0[i] - nv[i];
        r2 = r * r;
        nv[i] += c * r;
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Anderson acceleration of the SCC fixed-point map (type II, memory m,
// mixing c), one block of 1024 threads over all n entries:
//   F = q0 - n; ring slot k % (depth+1) <- (n, F);
//   dF_j, dn_j: differences of consecutive stored iterates (j < m = min(depth, k));
//   gamma = argmin || F - dF gamma || by modified Gram-Schmidt QR of dF;
//   n <- n + c F - sum_j gamma_j (dn_j + c dF_j).
// work: [depth+1][n] iterates, [depth+1][n] residuals, [depth][n] Q columns.
constexpr int kAT = 1024;
constexpr int kMaxDepth = 8;

__device__ double block_sum_kat(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < kAT / 64; ++w) r += red[w];
    return r;
}

__global__ void __launch_bounds__(kAT) k_anderson(int n, double* __restrict__ nv, const double* __restrict__ q0,
                                                 double c, int depth, int k, double* __restrict__ work,
                                                 double* __restrict__ out) {
    __shared__ double red[kAT / 64];
    __shared__ double R[kMaxDepth][kMaxDepth];
    __shared__ double gam[kMaxDepth];
    __shared__ int keep[kMaxDepth];
    const int slots = depth + 1;
    double* Nh = work;
    double* Fh = work + (int64_t)slots * n;
    double* Qc = work + (int64_t)2 * slots * n;
    const int cur = k % slots;
    double s2 = 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) {
        const double f = q0[i] - nv[i];
        Nh[(int64_t)cur * n + i] = nv[i];
        Fh[(int64_t)cur * n + i] = f;
        s2 += f * f;
    }
    const double fnorm2 = block_sum_kat(s2, red);
    if (threadIdx.x == 0) out[0] = sqrt(fnorm2 / n);
    const int m = min(depth, k);
    // QR of the residual differences, column by column
    for (int j = 0; j < m; ++j) {
        const int a = (k - m + j) % slots, b = (k - m + j + 1) % slots;
        double* qj = Qc + (int64_t)j * n;
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += kAT) {
            const double v = Fh[(int64_t)b * n + i] - Fh[(int64_t)a * n + i];
            qj[i] = v;
            s += v * v;
        }
        const double orig = sqrt(block_sum_kat(s, red));
        for (int l = 0; l < j; ++l) {
            const double* ql = Qc + (int64_t)l * n;
            double d = 0.0;
            for (int i = threadIdx.x; i < n; i += kAT) d += ql[i] * qj[i];
            const double rl = keep[l] ? block_sum_kat(d, red) : 0.0;
            if (threadIdx.x == 0) R[l][j] = rl;
            for (int i = threadIdx.x; i < n; i += kAT) qj[i] -= rl * ql[i];
        }
        double t = 0.0;
        for (int i = threadIdx.x; i < n; i += kAT) t += qj[i] * qj[i];
        const double rjj = sqrt(block_sum_kat(t, red));
        const bool ok = rjj > 1e-12 * orig && rjj > 0.0;
        if (threadIdx.x == 0) {
            R[j][j] = rjj;
            keep[j] = ok;
        }
        const double inv = ok ? 1.0 / rjj : 0.0;
        for (int i = threadIdx.x; i < n; i += kAT) qj[i] *= inv;
        __syncthreads();
    }
    // rhs Q^T F_k, then back substitution R gamma = rhs over the kept columns
    for (int j = 0; j < m; ++j) {
        const double* qj = Qc + (int64_t)j * n;
        double d = 0.0;
        for (int i = threadIdx.x; i < n; i += kAT) d += qj[i] * Fh[(int64_t)cur * n + i];
        const double rhs = block_sum_kat(d, red);
        if (threadIdx.x == 0) gam[j] = rhs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = m - 1; j >= 0; --j) {
            if (!keep[j]) {
                gam[j] = 0.0;
                continue;
            }
            double v = gam[j];
            for (int l = j + 1; l < m; ++l) v -= R[j][l] * gam[l];
            gam[j] = v / R[j][j];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kAT) {
        const double f = Fh[(int64_t)cur * n + i];
        double x = nv[i] + c * f;
        for (int j = 0; j < m; ++j) {
            const int a = (k - m + j) % slots, b = (k - m + j + 1) % slots;
            const double dn = Nh[(int64_t)b * n + i] - Nh[(int64_t)a * n + i];
            const double df = Fh[(int64_t)b * n + i] - Fh[(int64_t)a * n + i];
            x -= gam[j] * (dn + c * df);
        }
        nv[i] = x;
    }
}

// Low-rank preconditioned Krylov kernel of the quasi-Newton SCF step with
// K0 = -k0 I (one block of 1024 threads over all n entries; the directional
// derivatives come from the charge response, one call per rank):
//   begin: r = K0 f = k0 (n - q0) (f = q0 - n), v_0 = r / |r|;
//   add j: f_vj = K0 J v_j = k0 (v_j - dq_j) (J v_j = dq_j - v_j); QR of
//          [f_v0 .. f_vj] by modified Gram-Schmidt, one column per call
//          (two passes; a numerically dependent column is dropped);
//          g = Q^T r, c = R^-1 g = argmin || F_v c - r ||, its relative
//          residual; next direction v_{j+1} = f_vj orthogonalised against
//          v_0 .. v_j (two passes);
//   apply: n <- n - alpha (V c + complete (r - Q g)).
// work (caller-owned, kept over the calls of one step): r [n], V [cap][n],
// Q [cap][n], R [cap][cap], c [cap], g [cap], |r|, k0.
constexpr int kMaxRank = 16;

struct KrylovWork {
    double *r, *V, *Q, *R, *c, *g, *sc;
};

__device__ __forceinline__ KrylovWork krylov_work(double* w, int n, int cap) {
    KrylovWork k;
    k.r = w;
    k.V = w + n;
    k.Q = k.V + (int64_t)cap * n;
    k.R = k.Q + (int64_t)cap * n;
    k.c = k.R + cap * cap;
    k.g = k.c + cap;
    k.sc = k.g + cap;
    return k;
}

__global__ void __launch_bounds__(kAT) k_krylov_begin(int n, const double* __restrict__ nv,
                                                     const double* __restrict__ q0, double k0, int cap,
                                                     double* work, double* __restrict__ out) {
    __shared__ double red[kAT / 64];
    const KrylovWork w = krylov_work(work, n, cap);
    double s2 = 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) {
        const double f = q0[i] - nv[i];
        w.r[i] = -k0 * f;
        s2 += f * f;
    }
    const double fn = sqrt(block_sum_kat(s2, red));
    const double rn = k0 * fn;
    const double inv = rn > 0.0 ? 1.0 / rn : 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) w.V[i] = w.r[i] * inv;
    if (threadIdx.x == 0) {
        w.sc[0] = rn;
        w.sc[1] = k0;
        out[0] = fn / sqrt((double)n);
    }
}

__global__ void __launch_bounds__(kAT) k_krylov_add(int n, int j, const double* __restrict__ dq, int cap,
                                                   double* work, double* __restrict__ out) {
    __shared__ double red[kAT / 64];
    __shared__ double g[kMaxRank];
    const KrylovWork w = krylov_work(work, n, cap);
    const double* vj = w.V + (int64_t)j * n;
    double* qj = w.Q + (int64_t)j * n;
    const double k0 = w.sc[1];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) {
        const double f = k0 * (vj[i] - dq[i]);
        qj[i] = f;
        s += f * f;
    }
    const double orig = sqrt(block_sum_kat(s, red));
    // column j of R: projections on the earlier Q columns, twice
    for (int l = 0; l < j; ++l)
        if (threadIdx.x == 0) w.R[l * cap + j] = 0.0;
    for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l < j; ++l) {
            const double* ql = w.Q + (int64_t)l * n;
            double d = 0.0;
            for (int i = threadIdx.x; i < n; i += kAT) d += ql[i] * qj[i];
            const double rl = block_sum_kat(d, red);
            for (int i = threadIdx.x; i < n; i += kAT) qj[i] -= rl * ql[i];
            if (threadIdx.x == 0) w.R[l * cap + j] += rl;
        }
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) t += qj[i] * qj[i];
    const double rjj = sqrt(block_sum_kat(t, red));
    const bool keep = rjj > 1e-12 * orig && rjj > 0.0;
    const double inv = keep ? 1.0 / rjj : 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) qj[i] *= inv;
    if (threadIdx.x == 0) w.R[j * cap + j] = keep ? rjj : 0.0;
    // g = Q^T r, c = R^-1 g over the kept columns
    for (int l = 0; l <= j; ++l) {
        const double* ql = w.Q + (int64_t)l * n;
        double d = 0.0;
        for (int i = threadIdx.x; i < n; i += kAT) d += ql[i] * w.r[i];
        const double gl = block_sum_kat(d, red);
        if (threadIdx.x == 0) {
            g[l] = gl;
            w.g[l] = gl;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int l = j; l >= 0; --l) {
            const double rll = w.R[l * cap + l];
            if (rll == 0.0) {
                w.c[l] = 0.0;
                continue;
            }
            double v = g[l];
            for (int m = l + 1; m <= j; ++m) v -= w.R[l * cap + m] * w.c[m];
            w.c[l] = v / rll;
        }
    }
    __syncthreads();
    // relative residual || r - Q g || / || r ||
    double e2 = 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) {
        double e = w.r[i];
        for (int l = 0; l <= j; ++l) e -= g[l] * w.Q[(int64_t)l * n + i];
        e2 += e * e;
    }
    const double res = sqrt(block_sum_kat(e2, red));
    const double rn = w.sc[0];
    if (threadIdx.x == 0) out[0] = rn > 0.0 ? res / rn : 0.0;
    if (j + 1 >= cap) return;
    // next Krylov direction
    double* vn = w.V + (int64_t)(j + 1) * n;
    for (int i = threadIdx.x; i < n; i += kAT) vn[i] = k0 * (vj[i] - dq[i]);
    for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l <= j; ++l) {
            const double* vl = w.V + (int64_t)l * n;
            double d = 0.0;
            for (int i = threadIdx.x; i < n; i += kAT) d += vl[i] * vn[i];
            const double p = block_sum_kat(d, red);
            for (int i = threadIdx.x; i < n; i += kAT) vn[i] -= p * vl[i];
        }
    double u = 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) u += vn[i] * vn[i];
    const double un = sqrt(block_sum_kat(u, red));
    const double ui = un > 1e-14 * orig && un > 0.0 ? 1.0 / un : 0.0;
    for (int i = threadIdx.x; i < n; i += kAT) vn[i] *= ui;
    if (threadIdx.x == 0) out[1] = ui > 0.0 ? 0.0 : 1.0;     // 1: the Krylov space is exhausted
}

__global__ void k_krylov_apply(int n, int rank, int cap, double alpha, int complete, double* work,
                               double* __restrict__ nv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const KrylovWork w = krylov_work(work, n, cap);
    double d = 0.0;
    for (int l = 0; l < rank; ++l) d += w.c[l] * w.V[(int64_t)l * n + i];
    if (complete) {
        double e = w.r[i];
        for (int l = 0; l < rank; ++l) e -= w.g[l] * w.Q[(int64_t)l * n + i];
        d += e;
    }
    nv[i] -= alpha * d;
}

// a = 2 q - n
__global__ void k_two_q_minus_n(int n, const double* __restrict__ q, const double* __restrict__ nv,
                                double* __restrict__ a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 2.0 * q[i] - nv[i];
}

// dS/dR of slater_short, term by term from its closed form
__device__ double slater_short_deriv(double ta, double tb, double R) {
    if (fabs(ta - tb) < 1e-6 * (ta + tb)) {
        const double t = 0.5 * (ta + tb);
        const double p = 1.0 / R + 11.0 * t / 16.0 + 3.0 * t * t * R / 16.0 + t * t * t * R * R / 48.0;
        const double dp = -1.0 / (R * R) + 3.0 * t * t / 16.0 + t * t * t * R / 24.0;
        return exp(-t * R) * (dp - t * p);
    }
    double out = 0.0;
    for (int side = 0; side < 2; ++side) {
        const double a = side ? tb : ta, b = side ? ta : tb;
        const double a2 = a * a, b2 = b * b, d = a2 - b2;
        const double A = b2 * b2 * a / (2.0 * d * d);
        const double Bc = (b2 * b2 * b2 - 3.0 * b2 * b2 * a2) / (d * d * d);
        out += exp(-a * R) * (-a * (A - Bc / R) + Bc / (R * R));
    }
    return out;
}

// F_K += -d/dR_K (1/2 a^T gamma b) with gamma_KJ = k_e [psi(R_J - R_K) - S]:
//   real space over the cutoff CSR (r < rc): 1/2 k_e sum_J (a_K b_J + a_J b_K) g'(r) u,
//     g(r) = erfc(eta r)/r (- S(tau_K, tau_J, r) when screened), u = (R_J - R_K)/r;
//   reciprocal space over the half space of k (weights w_k = 4 pi/V exp(-k^2/4eta^2)/k^2):
//     -k_e sum_k w_k k [a_K (S_b cos - C_b sin) + b_K (S_a cos - C_a sin)](k . R_K)
//   with (C_x, S_x)(k) = sum_J x_J (cos, sin)(k . R_J) (the k and -k terms are equal).
__global__ void __launch_bounds__(64 * kRealAtoms) k_ewald_force_real(
    int n, const double* __restrict__ pos, const int32_t* __restrict__ species, double3 L, double3 iL,
    const int32_t* __restrict__ rp, const int32_t* __restrict__ cl, double rc, double eta, int screened, double tau0,
    double tau1, const double* __restrict__ qa, const double* __restrict__ qb, double ke, double* __restrict__ F) {
    const int i = blockIdx.x * kRealAtoms + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= n) return;                 // uniform over the wave
    const double ti = species[i] == 0 ? tau0 : tau1;
    const double ai = qa[i], bi = qb[i];
    const double c2 = 2.0 / sqrt(M_PI);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int k = rp[i] + lane; k < rp[i + 1]; k += 64) {
        const int j = cl[k];
        double dx, dy, dz;
        min_image(pos, i, j, L, iL, &dx, &dy, &dz);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (!(r < rc)) continue;
        double gp = -erfc(eta * r) / (r * r) - c2 * eta * exp(-eta * eta * r * r) / r;
        if (screened) gp -= slater_short_deriv(ti, species[j] == 0 ? tau0 : tau1, r);
        const double w = 0.5 * (ai * qb[j] + qa[j] * bi) * gp / r;
        fx += w * dx;
        fy += w * dy;
        fz += w * dz;
    }
    fx = gdm_wave_sum(fx);
    fy = gdm_wave_sum(fy);
    fz = gdm_wave_sum(fz);
    if (lane == 0) {
        F[3 * i] += ke * fx;
        F[3 * i + 1] += ke * fy;
        F[3 * i + 2] += ke * fz;
    }
}

__global__ void k_ewald_force_finish(int n, int nchunk, const double* __restrict__ part, double ke,
                                     double* __restrict__ F) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int y = 0; y < nchunk; ++y) {
        const double* o = part + ((int64_t)y * n + i) * 3;
        gx += o[0];
        gy += o[1];
        gz += o[2];
    }
    F[3 * i] -= ke * gx;
    F[3 * i + 1] -= ke * gy;
    F[3 * i + 2] -= ke * gz;
}

}  // namespace

// ---------------------------------------------------------------------- host

static int check_ctx_sys(gdm_ctx* ctx, const gdm_system* sys) {
    if (!sys || !sys->pos || !sys->species || sys->n_atoms <= 0)
        return gdm_fail(ctx, GDM_E_ARG, "null system or no atoms");
    return GDM_OK;
}

extern "C" int gdm_descriptors(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr, const int32_t* col,
                               double* feats) {
    if (!ctx) return GDM_E_ARG;
    int rc = check_ctx_sys(ctx, sys);
    if (rc) return rc;
    if (!row_ptr || !col || !feats) return gdm_fail(ctx, GDM_E_ARG, "gdm_descriptors: null argument");
    const int n = sys->n_atoms;
    GDM_TIMED(ctx, "descriptors");
    hipLaunchKernelGGL(k_descriptors, dim3((n + 127) / 128), dim3(128), 0, ctx->stream, n, sys->pos, sys->species,
                       make_double3(sys->box[0], sys->box[1], sys->box[2]),
                       make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]), row_ptr, col, 5.0, 0.3, 0.8,
                       3.2 / 15.0, feats);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_feature_sums(gdm_ctx* ctx, int32_t n, const double* feats, const int32_t* species,
                                double* stats) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !feats || !species || !stats) return gdm_fail(ctx, GDM_E_ARG, "gdm_feature_sums: bad argument");
    hipLaunchKernelGGL(k_feature_sums, dim3(256), dim3(kNF), 0, ctx->stream, n, feats, species, stats);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_feature_norm(gdm_ctx* ctx, const double* stats, float* norm) {
    if (!ctx) return GDM_E_ARG;
    if (!stats || !norm) return gdm_fail(ctx, GDM_E_ARG, "gdm_feature_norm: null argument");
    hipLaunchKernelGGL(k_feature_norm, dim3(1), dim3(2 * kNF), 0, ctx->stream, stats, norm);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_mlp_forward(gdm_ctx* ctx, int32_t n, const int32_t* species, const double* feats,
                               const float* params, const float* norm, int bf16, float* y) {
    if (!ctx) return GDM_E_ARG;
    if (n < 0 || (n > 0 && (!species || !feats || !params || !norm || !y)))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_mlp_forward: bad argument");
    if (n == 0) return GDM_OK;
    GDM_TIMED(ctx, "mlp_forward");
    if (bf16)
        hipLaunchKernelGGL(k_mlp_forward<true>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, species, feats,
                           params, norm, y);
    else
        hipLaunchKernelGGL(k_mlp_forward<false>, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, species, feats,
                           params, norm, y);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_mlp_loss(gdm_ctx* ctx, int32_t n, const float* y, const double* q_ref, double* stats3) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !y || !q_ref || !stats3) return gdm_fail(ctx, GDM_E_ARG, "gdm_mlp_loss: bad argument");
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, ctx->stream, n, y, q_ref, stats3);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_mlp_charges(gdm_ctx* ctx, int32_t n, const float* y, double* q) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !y || !q) return gdm_fail(ctx, GDM_E_ARG, "gdm_mlp_charges: bad argument");
    hipLaunchKernelGGL(k_center, dim3(1), dim3(1024), 0, ctx->stream, n, y, q);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_mlp_backward(gdm_ctx* ctx, int32_t n, const int32_t* species, const double* feats,
                                const float* params, const float* norm, const float* y, const double* q_ref,
                                const double* stats3, float* partial, float* grad) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !species || !feats || !params || !norm || !y || !q_ref || !stats3 || !partial || !grad)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_mlp_backward: bad argument");
    const int nb = (n + kBA - 1) / kBA;
    GDM_TIMED(ctx, "mlp_backward");
    hipLaunchKernelGGL(k_mlp_backward, dim3(nb), dim3(256), 0, ctx->stream, n, species, feats, params, norm, y, q_ref,
                       stats3, 2.0 / n, partial);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_reduce_partials, dim3((2 * kNP + 255) / 256), dim3(256), 0, ctx->stream, nb, partial, grad);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_adam_step(gdm_ctx* ctx, int32_t n, float* params, const float* grad, float* m, float* v,
                             int32_t t, float lr, float b1, float b2, float eps) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || t <= 0 || !params || !grad || !m || !v) return gdm_fail(ctx, GDM_E_ARG, "gdm_adam_step: bad argument");
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, params, grad, m, v, lr, b1, b2,
                       eps, c1, c2);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

// chunks of whole k-grid lines for the (atom blocks) x (chunks) launches:
// enough workgroups to fill the device, at least 2 lines per chunk
static void ewald_line_chunks(int n, int nlines, int* nchunk, int* lines_per_chunk) {
    const int ablocks = (n + 127) / 128;
    int c = std::max(1, 4096 / ablocks);
    c = std::min(c, std::max(1, nlines / 2));
    *lines_per_chunk = (nlines + c - 1) / c;
    *nchunk = (nlines + *lines_per_chunk - 1) / *lines_per_chunk;
}

static int check_ewald(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr, const int32_t* col, double rcut,
                       double eta, int32_t k_max, int32_t k_max_limit, const double hubbard_U[2], const double* tau,
                       const double* q, double* V, const char* who) {
    int rc = check_ctx_sys(ctx, sys);
    if (rc) return rc;
    if (!row_ptr || !col || !q || !V || !hubbard_U || !(rcut > 0) || !(eta > 0) || k_max < 1 || k_max > k_max_limit)
        return gdm_fail(ctx, GDM_E_ARG, "%s: bad argument (k_max %d, at most %d)", who, k_max, k_max_limit);
    if (tau && !(tau[0] > 0 && tau[1] > 0)) return gdm_fail(ctx, GDM_E_ARG, "%s: tau must be positive", who);
    for (int a = 0; a < 3; ++a)
        if (sys->box[a] <= 2.0 * rcut) return gdm_fail(ctx, GDM_E_ARG, "%s: box must exceed 2 rcut", who);
    return GDM_OK;
}

extern "C" int gdm_ewald_potential(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr, const int32_t* col,
                                   double rcut, double eta, int32_t k_max, const double hubbard_U[2],
                                   const double* tau, const double* q, double* V) {
    if (!ctx) return GDM_E_ARG;
    int rc = check_ewald(ctx, sys, row_ptr, col, rcut, eta, k_max, 64, hubbard_U, tau, q, V, "gdm_ewald_potential");
    if (rc) return rc;
    // the full k grid a = 0..K, b, c = -K..K on the device (weight 0 outside
    // the half space (a > 0) or (a = 0, b > 0) or (a = b = 0, c > 0) and the
    // sphere |k| <= 2 pi K / max L), summed line by line
    const double V3 = sys->box[0] * sys->box[1] * sys->box[2];
    const double kc2 = std::pow(2.0 * M_PI * k_max / std::max(sys->box[0], std::max(sys->box[1], sys->box[2])), 2);
    const int w = 2 * k_max + 1, nk = (k_max + 1) * w * w, nlines = (k_max + 1) * w;
    const int n = sys->n_atoms;
    int nchunk = 1, lpc = 1;
    ewald_line_chunks(n, nlines, &nchunk, &lpc);
    bool ok = true;
    double4* dkv = (double4*)gdm_buf(
        ctx, BUF_EWALD, sizeof(double4) * nk + sizeof(double) * (2 * (size_t)nk + (size_t)nchunk * n), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_ewald_potential: workspace allocation failed");
    double* CS = (double*)(dkv + nk);
    double* part = CS + 2 * (int64_t)nk;
    const double3 L = make_double3(sys->box[0], sys->box[1], sys->box[2]);
    const double3 iL = make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]);
    const double dkz = 2.0 * M_PI / sys->box[2];
    GDM_TIMED(ctx, "ewald");
    hipLaunchKernelGGL(k_ewald_ktable, dim3((nk + 255) / 256), dim3(256), 0, ctx->stream, k_max, sys->box[0],
                       sys->box[1], sys->box[2], eta, kc2, V3, dkv);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_real, dim3((n + kRealAtoms - 1) / kRealAtoms), dim3(64 * kRealAtoms), 0, ctx->stream,
                       n, sys->pos, sys->species, L, iL, row_ptr, col, rcut, eta, tau ? 1 : 0, tau ? tau[0] : 0.0,
                       tau ? tau[1] : 0.0, q, V);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL((k_ewald_sk_lines<1, kSkC>), dim3(nlines * ((w + kSkC - 1) / kSkC)), dim3(256), 0, ctx->stream,
                       n, k_max, sys->pos, q, q, dkv, dkz, CS, CS);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_recip_lines, dim3((n + 127) / 128, nchunk), dim3(128), 0, ctx->stream, n, k_max, lpc,
                       sys->pos, dkv, CS, dkz, part);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_finish, dim3((n + 127) / 128), dim3(128), 0, ctx->stream, n, nchunk, part, sys->species,
                       q, eta, 14.399645, hubbard_U[0], hubbard_U[1], V);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

// ------------------------------------------------ Ewald without allocation
// Scratch of gdm_ewald_potential_noalloc: the k-vector table (one double4 per
// point of the full (K+1)(2K+1)^2 grid) followed by the structure factors (two
// doubles per point), for K <= kNoAllocKMax: 48 B per point, 6.7 MB at K = 32.
// Every point is rewritten by each call, so nothing needs clearing.  One copy
// per GPU, held until the process ends, shared by every call on that GPU.
constexpr int kNoAllocKMax = 32;
constexpr int64_t kNoAllocGrid = (int64_t)(kNoAllocKMax + 1) * (2 * kNoAllocKMax + 1) * (2 * kNoAllocKMax + 1);
static __device__ __align__(256) double scratch[kNoAllocGrid * 6];

// Device address of `scratch` on the context's device, looked up once per
// device (the host-side name of the array is not a device address).
static int scratch_ptr(gdm_ctx* ctx, double** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return gdm_fail(ctx, GDM_E_ARG, "scratch: device %d out of range", ctx->device);
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[ctx->device]) {
        int cur = 0;
        GDM_HIP(ctx, hipGetDevice(&cur));
        if (cur != ctx->device) GDM_HIP(ctx, hipSetDevice(ctx->device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != ctx->device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return gdm_hip(ctx, e, "hipGetSymbolAddress(scratch)");
        ptr[ctx->device] = p;
    }
    *out = (double*)ptr[ctx->device];
    return GDM_OK;
}

extern "C" int gdm_ewald_potential_noalloc(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr,
                                           const int32_t* col, double rcut, double eta, int32_t k_max,
                                           const double hubbard_U[2], const double* tau, const double* q, double* V) {
    if (!ctx) return GDM_E_ARG;
    int rc = check_ewald(ctx, sys, row_ptr, col, rcut, eta, k_max, kNoAllocKMax, hubbard_U, tau, q, V,
                         "gdm_ewald_potential_noalloc");
    if (rc) return rc;
    double* sp = nullptr;
    if ((rc = scratch_ptr(ctx, &sp))) return rc;
    const int w = 2 * k_max + 1;
    const int nk = (k_max + 1) * w * w;
    double4* dkv = (double4*)sp;
    double* CS = sp + 4 * (int64_t)nk;
    const double V3 = sys->box[0] * sys->box[1] * sys->box[2];
    const double kc2 = std::pow(2.0 * M_PI * k_max / std::max(sys->box[0], std::max(sys->box[1], sys->box[2])), 2);
    const int n = sys->n_atoms;
    const double3 L = make_double3(sys->box[0], sys->box[1], sys->box[2]);
    const double3 iL = make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]);
    GDM_TIMED(ctx, "ewald");
    hipLaunchKernelGGL(k_ewald_ktable, dim3((nk + 255) / 256), dim3(256), 0, ctx->stream, k_max, sys->box[0],
                       sys->box[1], sys->box[2], eta, kc2, V3, dkv);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_real, dim3((n + kRealAtoms - 1) / kRealAtoms), dim3(64 * kRealAtoms), 0, ctx->stream,
                       n, sys->pos, sys->species, L, iL, row_ptr, col, rcut, eta, tau ? 1 : 0, tau ? tau[0] : 0.0,
                       tau ? tau[1] : 0.0, q, V);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_sk, dim3(nk), dim3(256), 0, ctx->stream, n, sys->pos, q, dkv, CS);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_recip, dim3((n + 127) / 128), dim3(128), 0, ctx->stream, n, nk, sys->pos,
                       sys->species, q, dkv, CS, eta, 14.399645, hubbard_U[0], hubbard_U[1], V);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_ewald_forces(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr, const int32_t* col,
                                double rcut, double eta, int32_t k_max, const double* tau, const double* q,
                                const double* n_vec, double* F) {
    if (!ctx) return GDM_E_ARG;
    const double U_unused[2] = {0.0, 0.0};
    int rc = check_ewald(ctx, sys, row_ptr, col, rcut, eta, k_max, 64, U_unused, tau, q, F, "gdm_ewald_forces");
    if (rc) return rc;
    if (!n_vec) return gdm_fail(ctx, GDM_E_ARG, "gdm_ewald_forces: null charge vector n_vec");
    const int w = 2 * k_max + 1;
    const int nk = (k_max + 1) * w * w, nlines = (k_max + 1) * w;
    int nchunk = 1, lpc = 1;
    ewald_line_chunks(sys->n_atoms, nlines, &nchunk, &lpc);
    bool ok = true;
    double* ws = (double*)gdm_buf(
        ctx, BUF_EWALD, sizeof(double) * (8 * (size_t)nk + sys->n_atoms + 3 * (size_t)nchunk * sys->n_atoms), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_ewald_forces: workspace allocation failed");
    const double dkz = 2.0 * M_PI / sys->box[2];
    const int skb = nlines * ((w + kSkC2 - 1) / kSkC2);
    double4* dkv = (double4*)ws;
    double* CSa = ws + 4 * (int64_t)nk;
    double* CSb = CSa + 2 * (int64_t)nk;
    double* a = CSb + 2 * (int64_t)nk;     // a = 2 q - n
    double* part = a + sys->n_atoms;
    const double* b = n_vec;
    const double V3 = sys->box[0] * sys->box[1] * sys->box[2];
    const double kc2 = std::pow(2.0 * M_PI * k_max / std::max(sys->box[0], std::max(sys->box[1], sys->box[2])), 2);
    const int n = sys->n_atoms;
    const double3 L = make_double3(sys->box[0], sys->box[1], sys->box[2]);
    const double3 iL = make_double3(sys->inv_box[0], sys->inv_box[1], sys->inv_box[2]);
    GDM_TIMED(ctx, "ewald_forces");
    hipLaunchKernelGGL(k_two_q_minus_n, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, q, n_vec, a);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_ktable, dim3((nk + 255) / 256), dim3(256), 0, ctx->stream, k_max, sys->box[0],
                       sys->box[1], sys->box[2], eta, kc2, V3, dkv);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL((k_ewald_sk_lines<2, kSkC2>), dim3(skb), dim3(256), 0, ctx->stream, n, k_max, sys->pos, a, b,
                       dkv, dkz, CSa, CSb);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_force_real, dim3((n + kRealAtoms - 1) / kRealAtoms), dim3(64 * kRealAtoms), 0,
                       ctx->stream, n, sys->pos, sys->species, L, iL, row_ptr, col, rcut, eta, tau ? 1 : 0,
                       tau ? tau[0] : 0.0, tau ? tau[1] : 0.0, a, b, 14.399645, F);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_force_recip_lines, dim3((n + 127) / 128, nchunk), dim3(128), 0, ctx->stream, n, k_max,
                       lpc, sys->pos, a, b, dkv, CSa, CSb, dkz, part);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_ewald_force_finish, dim3((n + 127) / 128), dim3(128), 0, ctx->stream, n, nchunk, part,
                       14.399645, F);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_scc_mix(gdm_ctx* ctx, int32_t n, double* n_vec, const double* q0, double mix, double* rms_out) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !n_vec || !q0 || !rms_out) return gdm_fail(ctx, GDM_E_ARG, "gdm_scc_mix: bad argument");
    const int nb = (n + 255) / 256;
    bool ok = true;
    double* part = (double*)gdm_buf(ctx, BUF_MIXPART, sizeof(double) * nb, &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_scc_mix: workspace allocation failed");
    hipLaunchKernelGGL(k_mix, dim3(nb), dim3(256), 0, ctx->stream, n, n_vec, q0, mix, part);
    GDM_LAUNCH_CHECK(ctx);
    std::vector<double> h(nb);
    GDM_HIP(ctx, hipMemcpyAsync(h.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (double v : h) s += v;
    *rms_out = std::sqrt(s / n);
    return GDM_OK;
}

extern "C" int gdm_scc_anderson(gdm_ctx* ctx, int32_t n, double* n_vec, const double* q0, double mix, int32_t depth,
                                int32_t k, double* work, double* rms_out) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !n_vec || !q0 || !work || !rms_out || depth < 0 || depth > kMaxDepth || k < 0)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_scc_anderson: bad argument");
    bool ok = true;
    double* out = (double*)gdm_buf(ctx, BUF_MIXPART, sizeof(double), &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_scc_anderson: workspace allocation failed");
    hipLaunchKernelGGL(k_anderson, dim3(1), dim3(kAT), 0, ctx->stream, n, n_vec, q0, mix, depth, k, work, out);
    GDM_LAUNCH_CHECK(ctx);
    GDM_HIP(ctx, hipMemcpyAsync(rms_out, out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GDM_OK;
}

extern "C" int gdm_krylov_begin(gdm_ctx* ctx, int32_t n, const double* n_vec, const double* q0, double k0,
                                int32_t max_rank, double* work, double* rms_out) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !n_vec || !q0 || !work || !rms_out || max_rank < 1 || max_rank > kMaxRank || !(k0 > 0.0))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_krylov_begin: bad argument");
    bool ok = true;
    double* out = (double*)gdm_buf(ctx, BUF_KRYLOV, sizeof(double) * 2, &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_krylov_begin: workspace allocation failed");
    hipLaunchKernelGGL(k_krylov_begin, dim3(1), dim3(kAT), 0, ctx->stream, n, n_vec, q0, k0, max_rank, work, out);
    GDM_LAUNCH_CHECK(ctx);
    GDM_HIP(ctx, hipMemcpyAsync(rms_out, out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GDM_OK;
}

extern "C" int gdm_krylov_add(gdm_ctx* ctx, int32_t n, int32_t j, const double* dq, int32_t max_rank, double* work,
                              double* rel_out, int32_t* exhausted_out) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !dq || !work || !rel_out || max_rank < 1 || max_rank > kMaxRank || j < 0 || j >= max_rank)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_krylov_add: bad argument");
    bool ok = true;
    double* out = (double*)gdm_buf(ctx, BUF_KRYLOV, sizeof(double) * 2, &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_krylov_add: workspace allocation failed");
    {
        const int rc = gdm_fill_f64(ctx, out, 2, 0.0);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_krylov_add, dim3(1), dim3(kAT), 0, ctx->stream, n, j, dq, max_rank, work, out);
    GDM_LAUNCH_CHECK(ctx);
    double h[2];
    GDM_HIP(ctx, hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *rel_out = h[0];
    if (exhausted_out) *exhausted_out = h[1] != 0.0;
    return GDM_OK;
}

extern "C" int gdm_krylov_apply(gdm_ctx* ctx, int32_t n, int32_t rank, int32_t max_rank, double alpha,
                                int32_t complete, double* n_vec, double* work) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !n_vec || !work || max_rank < 1 || max_rank > kMaxRank || rank < 1 || rank > max_rank ||
        !std::isfinite(alpha))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_krylov_apply: bad argument");
    hipLaunchKernelGGL(k_krylov_apply, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, rank, max_rank, alpha,
                       complete, work, n_vec);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}
