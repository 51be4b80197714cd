// FP64 subgraph solver ("direct diagonalization" option of the paper's
// subgraph step): per subgraph
//   s = L L^T (Cholesky),  h_perp = L^-1 h L^-T,  h_perp = Hh T Hh^T
//   (Householder), T = R diag(lam) R^T (implicit QL, rotations recorded),
// and only the 2*nc core rows are pushed through the reflectors and the
// rotations:  C[core,:] = (L^-T)[core,:] Hh R,  Q[core,:] = I[core,:] Hh R,
//   w_k = sum_{a in core} C_ak (L Q)_ak            (core electron weights)
//   D[core,:] = (C[core,:] diag(f) R^T Hh^T) L^-1  (collected core rows, Eq. 3)
// so after the O(n^3) reductions everything is O(nc n^2).
// The basis Z = L^-T gives the same D as Z = s^-1/2 (any Z with Z Z^T = s^-1).
#include "gdm_internal.h"

#include <map>
#include <mutex>

#include <algorithm>
#include <cmath>

namespace {

constexpr int kThreads = 256;   // threads per workgroup for the per-subgraph kernels

// ------------------------------------------------------------- Cholesky
// Left-looking, column by column: row j of L staged in LDS; each wave forms
// the dot products of the rows below with it (lanes over the inner index).
__global__ void __launch_bounds__(kThreads) k_potrf(const SubDesc* __restrict__ desc, double* __restrict__ Sd,
                                             int* __restrict__ status) {
    extern __shared__ double rowj[];
    __shared__ double s_diag;
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, ld = d.ld;
    double* a = Sd + d.off2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < n; ++j) {
        // diagonal
        if (wave == 0) {
            double acc = 0.0;
            for (int k = lane; k < j; k += 64) {
                double v = a[(int64_t)j * ld + k];
                acc += v * v;
            }
            acc = gdm_wave_sum(acc);
            if (lane == 0) {
                double v = a[(int64_t)j * ld + j] - acc;
                if (!(v > 0.0)) {
                    gdm_raise(status, GDM_STATUS_NOT_PD);
                    v = 1.0;
                }
                v = sqrt(v);
                a[(int64_t)j * ld + j] = v;
                s_diag = v;
            }
        }
        for (int k = threadIdx.x; k < j; k += kThreads) rowj[k] = a[(int64_t)j * ld + k];
        __syncthreads();
        const double inv = 1.0 / s_diag;
        for (int i = j + 1 + wave; i < n; i += kThreads / 64) {
            const double* ri = a + (int64_t)i * ld;
            double acc = 0.0;
            for (int k = lane; k < j; k += 64) acc += ri[k] * rowj[k];
            acc = gdm_wave_sum(acc);
            if (lane == 0) a[(int64_t)i * ld + j] = (ri[j] - acc) * inv;
        }
        __syncthreads();
    }
}

// ------------------------------------------- triangular solves, h_perp
// X = L^-1 B (forward substitution), one thread per right-hand side column.
// MODE 0: B = A (h), result into T.   MODE 1: B = T^T, result into A.
template <int MODE>
__global__ void __launch_bounds__(kThreads) k_trsm(const SubDesc* __restrict__ desc, const double* __restrict__ Lm,
                                            double* __restrict__ A, double* __restrict__ T) {
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, ld = d.ld;
    const double* l = Lm + d.off2;
    double* a = A + d.off2;
    double* t = T + d.off2;
    double* X = MODE == 0 ? t : a;
    for (int c = threadIdx.x; c < n; c += kThreads) {
        for (int i = 0; i < n; ++i) {
            double b = MODE == 0 ? a[(int64_t)i * ld + c] : t[(int64_t)c * ld + i];
            const double* li = l + (int64_t)i * ld;
            double acc = 0.0;
            for (int k = 0; k < i; ++k) acc += li[k] * X[(int64_t)k * ld + c];
            X[(int64_t)i * ld + c] = (b - acc) / li[i];
        }
    }
}

// A <- (A + A^T)/2 (exact symmetry for the reduction)
__global__ void __launch_bounds__(kThreads) k_symmetrize(const SubDesc* __restrict__ desc, double* __restrict__ A) {
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, ld = d.ld;
    double* a = A + d.off2;
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += kThreads) {
        int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        if (j <= i) continue;
        double v = 0.5 * (a[(int64_t)i * ld + j] + a[(int64_t)j * ld + i]);
        a[(int64_t)i * ld + j] = v;
        a[(int64_t)j * ld + i] = v;
    }
}

// ------------------------------------------------ Householder tridiagonal
// Unblocked reduction on full symmetric storage.  Step k reflects x =
// A[k+1:, k] onto beta e_1 with H = I - tau v v^T, v_0 = 1; v (without the
// unit) is stored in row k of A from column k+2 on; d, e, tau per subgraph.
__device__ __forceinline__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = gdm_wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    return s;
}

__global__ void __launch_bounds__(kThreads) k_sytrd(const SubDesc* __restrict__ desc, double* __restrict__ A,
                                             double* __restrict__ Dg, double* __restrict__ Eg,
                                             double* __restrict__ Tau) {
    extern __shared__ double sm[];
    __shared__ double red[kThreads / 64];
    const SubDesc dsc = desc[blockIdx.x];
    const int n = dsc.n, ld = dsc.ld;
    double* a = A + dsc.off2;
    double* dd = Dg + dsc.offv;
    double* ee = Eg + dsc.offv;
    double* tau = Tau + dsc.offv;
    double* v = sm;          // [n]
    double* w = sm + n;      // [n]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < n - 2; ++k) {
        const int m = n - k - 1;             // length of x
        const double* rowk = a + (int64_t)k * ld + (k + 1);   // x (row k == column k)
        double part = 0.0;
        for (int i = 1 + threadIdx.x; i < m; i += kThreads) {
            double x = rowk[i];
            part += x * x;
        }
        const double xn2 = block_sum(part, red);
        const double alpha = rowk[0];
        double beta, t, scale;
        if (xn2 == 0.0) {
            beta = alpha;
            t = 0.0;
            scale = 0.0;
        } else {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            t = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        for (int i = threadIdx.x; i < m; i += kThreads) v[i] = i == 0 ? 1.0 : rowk[i] * scale;
        __syncthreads();
        if (threadIdx.x == 0) {
            dd[k] = a[(int64_t)k * ld + k];
            ee[k] = beta;
            tau[k] = t;
        }
        // p = t * A22 v  (A22 = A[k+1:, k+1:]); one wave per row
        for (int i = wave; i < m; i += kThreads / 64) {
            const double* ri = a + (int64_t)(k + 1 + i) * ld + (k + 1);
            double acc = 0.0;
            for (int j = lane; j < m; j += 64) acc += ri[j] * v[j];
            acc = gdm_wave_sum(acc);
            if (lane == 0) w[i] = t * acc;
        }
        __syncthreads();
        part = 0.0;
        for (int i = threadIdx.x; i < m; i += kThreads) part += w[i] * v[i];
        const double pv = block_sum(part, red);
        const double half = 0.5 * t * pv;
        for (int i = threadIdx.x; i < m; i += kThreads) w[i] = w[i] - half * v[i];
        __syncthreads();
        // A22 -= v w^T + w v^T
        for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += kThreads) {
            int i = (int)(e / m), j = (int)(e - (int64_t)i * m);
            double* p = a + (int64_t)(k + 1 + i) * ld + (k + 1 + j);
            *p = *p - v[i] * w[j] - w[i] * v[j];
        }
        __syncthreads();
        // store v (tail) in row k beyond the sub-diagonal
        for (int i = 1 + threadIdx.x; i < m; i += kThreads) a[(int64_t)k * ld + (k + 1 + i)] = v[i];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (n >= 2) {
            dd[n - 2] = a[(int64_t)(n - 2) * ld + (n - 2)];
            ee[n - 2] = a[(int64_t)(n - 1) * ld + (n - 2)];
        }
        dd[n - 1] = a[(int64_t)(n - 1) * ld + (n - 1)];
        ee[n - 1] = 0.0;
        if (n >= 2) tau[n - 2] = 0.0;
        tau[n - 1] = 0.0;
    }
}

// ---------------------------------------------------- implicit QL (steqr)
// One wave per subgraph; lane 0 iterates on d, e held in LDS.  Every plane
// rotation (i, c, s) acting on columns (i, i+1) as
//   z_i' = c z_i - s z_{i+1},  z_{i+1}' = s z_i + c z_{i+1}
// is appended to the subgraph's record, in application order.
__global__ void __launch_bounds__(64) k_steqr(const SubDesc* __restrict__ desc, const double* __restrict__ Dg,
                                             const double* __restrict__ Eg, double* __restrict__ Lam,
                                             double* __restrict__ RotC, double* __restrict__ RotS,
                                             int32_t* __restrict__ RotI, int64_t* __restrict__ RotN,
                                             int* __restrict__ status) {
    extern __shared__ double sm[];
    const SubDesc dsc = desc[blockIdx.x];
    const int n = dsc.n;
    double* d = sm;
    double* e = sm + n;
    for (int i = threadIdx.x; i < n; i += 64) {
        d[i] = Dg[dsc.offv + i];
        e[i] = Eg[dsc.offv + i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* rc = RotC + dsc.offr;
        double* rs = RotS + dsc.offr;
        int32_t* ri = RotI + dsc.offr;
        const int64_t cap = dsc.rot_cap;
        int64_t nrot = 0;
        bool bad = false;
        e[n - 1] = 0.0;
        const double eps = 1.1102230246251565e-16;
        for (int l = 0; l < n && !bad; ++l) {
            int iter = 0;
            for (;;) {
                int m = l;
                for (; m < n - 1; ++m) {
                    double dd = fabs(d[m]) + fabs(d[m + 1]);
                    if (fabs(e[m]) <= eps * dd) break;
                }
                if (m == l) break;
                if (++iter > 60) {
                    bad = true;
                    gdm_raise(status, GDM_STATUS_NOT_CONVERGED);
                    break;
                }
                // Wilkinson-type shift from the leading 2x2 block
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = hypot(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + copysign(r, g));
                double s = 1.0, c = 1.0, p = 0.0;
                bool underflow = false;
                for (int i = m - 1; i >= l; --i) {
                    double f = s * e[i];
                    double b = c * e[i];
                    r = hypot(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= p;
                        e[m] = 0.0;
                        underflow = true;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    if (nrot < cap) {
                        rc[nrot] = c;
                        rs[nrot] = s;
                        ri[nrot] = i;
                    }
                    ++nrot;
                }
                if (underflow) continue;
                d[l] -= p;
                e[l] = g;
                e[m] = 0.0;
            }
        }
        if (nrot > cap) gdm_raise(status, GDM_STATUS_CAPACITY);
        RotN[blockIdx.x] = nrot < cap ? nrot : cap;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 64) Lam[dsc.offv + i] = d[i];
}

// --------------------------------------- core rows through Hh and R
// The 2*nc rows to be transformed (rows 0..nc-1 start as I[core,:], rows
// nc..2nc-1 as (L^-T)[core,:]) are independent, so they are processed in
// chunks held in LDS: block (s, c) takes rows c*RC .. of subgraph s, one lane
// per row, row stride n + 1 doubles.  Each row is initialised (unit row, or
// forward substitution L y = e_c), multiplied by the reflectors H_0 ...
// H_{n-3} and the recorded QL rotations in order, and written to G in the
// column-interleaved layout G[i*R + r] (R = 2*nc).
constexpr int kRowLds = 144 * 1024;     // LDS bytes for one chunk of rows
constexpr int kRowThreads = 64;

__host__ __device__ inline int chunk_rows(int n) {
    const int r = kRowLds / (8 * (n + 1));
    return r > kRowThreads ? kRowThreads : (r < 1 ? 1 : r);
}

// row <- row - t (row . v) v on row[off .. off+m), v = (1, vk[1..m-1]); one
// lane per row (act); the reflector entries are uniform loads
__device__ __forceinline__ void reflect_row(double* row, bool act, int off, int m, const double* vk, double t) {
    if (!act) return;
    double* x = row + off;
    double dot = x[0];
    for (int i = 1; i < m; ++i) dot += x[i] * vk[i];
    dot *= t;
    x[0] -= dot;
    for (int i = 1; i < m; ++i) x[i] -= dot * vk[i];
}

__global__ void __launch_bounds__(kRowThreads) k_core_rows(const SubDesc* __restrict__ desc,
                                                      const double* __restrict__ Lm, const double* __restrict__ A,
                                                      const double* __restrict__ Tau,
                                                      const double* __restrict__ RotC,
                                                      const double* __restrict__ RotS,
                                                      const int32_t* __restrict__ RotI,
                                                      const int64_t* __restrict__ RotN, double* __restrict__ G) {
    extern __shared__ double rows[];
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, nc = d.nc, ld = d.ld, R = 2 * nc;
    const int RC = chunk_rows(n), S = n + 1;
    const int r0 = blockIdx.y * RC;
    if (r0 >= R) return;
    const int nr = min(RC, R - r0);
    const int lane = threadIdx.x;
    const bool act = lane < nr;
    const int r = r0 + lane;
    double* row = rows + (int64_t)(act ? lane : 0) * S;
    const double* l = Lm + d.off2;
    // initial rows: unit rows, or columns of L^-1 by forward substitution
    // (y_k = 0 for k < c)
    if (act)
        for (int i = 0; i < n; ++i) row[i] = (r < nc && i == r) ? 1.0 : 0.0;
    if (act && r >= nc) {
        const int c = r - nc;
        for (int i = c; i < n; ++i) {
            const double* li = l + (int64_t)i * ld;
            double acc = i == c ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) acc -= li[k] * row[k];
            row[i] = acc / li[i];
        }
    }
    const double* a = A + d.off2;
    const double* tau = Tau + d.offv;
    for (int k = 0; k < n - 2; ++k) {
        const double t = tau[k];
        if (t == 0.0) continue;
        reflect_row(row, act, k + 1, n - k - 1, a + (int64_t)k * ld + k + 1, t);
    }
    // rotations in order
    if (act) {
        const int64_t nrot = RotN[blockIdx.x];
        const double* rc = RotC + d.offr;
        const double* rs = RotS + d.offr;
        const int32_t* ri = RotI + d.offr;
        for (int64_t q = 0; q < nrot; ++q) {
            const int i = ri[q];
            const double c = rc[q], sn = rs[q];
            const double gi = row[i], gj = row[i + 1];
            row[i] = c * gi - sn * gj;
            row[i + 1] = sn * gi + c * gj;
        }
    }
    double* g = G + 2 * d.offc;
    for (int i = 0; i < n; ++i)
        if (act) g[(int64_t)i * R + r] = row[i];
}

// w_k = sum_{a<nc} C[a][k] * (L_cc Q_core)[a][k]: the core weight of
// eigenvector k, (C^T s C)_core diagonal contribution, with s C = L Q
__global__ void __launch_bounds__(kThreads) k_core_weights(const SubDesc* __restrict__ desc,
                                                          const double* __restrict__ Lm,
                                                          const double* __restrict__ G, double* __restrict__ W) {
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, nc = d.nc, ld = d.ld, R = 2 * nc;
    const double* l = Lm + d.off2;
    const double* g = G + 2 * d.offc;
    for (int k = threadIdx.x; k < n; k += kThreads) {
        double acc = 0.0;
        for (int aa = 0; aa < nc; ++aa) {
            const double* la = l + (int64_t)aa * ld;
            double lq = 0.0;
            for (int b = 0; b <= aa; ++b) lq += la[b] * g[(int64_t)k * R + b];
            acc += g[(int64_t)k * R + nc + aa] * lq;
        }
        W[d.offv + k] = acc;
    }
}

// ------------------------------------------------------- D core rows
// U = C_core diag(f);  M = U R^T Hh^T;  D_core = M L^-1 (solve D L = M).
__device__ __forceinline__ double fermi_fp64(double x, double beta) {
    if (x > 0.0) {
        double e = exp(-beta * x);
        return e / (1.0 + e);
    }
    double e = exp(beta * x);
    return 1.0 / (1.0 + e);
}

// Core rows r < nc in LDS chunks as above: u = C[r,:] diag(f), then
// u <- u R^T (rotations in reverse order, transposed), u <- u H_{n-3} ... H_0,
// and D[r,:] from D L = u (columns from the right), written row-wise.
__global__ void __launch_bounds__(kRowThreads) k_dcore(const SubDesc* __restrict__ desc,
                                                  const double* __restrict__ Lm, const double* __restrict__ A,
                                                  const double* __restrict__ Tau, const double* __restrict__ RotC,
                                                  const double* __restrict__ RotS, const int32_t* __restrict__ RotI,
                                                  const int64_t* __restrict__ RotN, const double* __restrict__ G,
                                                  const double* __restrict__ Lam, double mu_host,
                                                  const double* __restrict__ mu_dev, double beta,
                                                  double* __restrict__ Dout, double* __restrict__ EigOut) {
    extern __shared__ double rows[];
    const double mu = mu_dev ? *mu_dev : mu_host;      // mu from device memory when given
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n, nc = d.nc, ld = d.ld, R2 = 2 * nc;
    const int RC = chunk_rows(n), S = n + 1;
    const int r0 = blockIdx.y * RC;
    if (r0 >= nc) return;
    const int nr = min(RC, nc - r0);
    const int lane = threadIdx.x;
    const bool act = lane < nr;
    const int r = r0 + lane;
    double* row = rows + (int64_t)(act ? lane : 0) * S;
    const double* l = Lm + d.off2;
    const double* g = G + 2 * d.offc;
    if (EigOut && blockIdx.y == 0)
        for (int k = lane; k < n; k += kRowThreads) EigOut[d.offe + k] = Lam[d.offv + k];
    for (int k = 0; k < n; ++k)
        if (act) row[k] = g[(int64_t)k * R2 + nc + r] * fermi_fp64(Lam[d.offv + k] - mu, beta);
    // rotations in reverse order, transposed
    if (act) {
        const int64_t nrot = RotN[blockIdx.x];
        const double* rc = RotC + d.offr;
        const double* rs = RotS + d.offr;
        const int32_t* ri = RotI + d.offr;
        for (int64_t q = nrot - 1; q >= 0; --q) {
            const int i = ri[q];
            const double c = rc[q], sn = rs[q];
            const double ui = row[i], uj = row[i + 1];
            row[i] = c * ui + sn * uj;
            row[i + 1] = -sn * ui + c * uj;
        }
    }
    const double* a = A + d.off2;
    const double* tau = Tau + d.offv;
    for (int k = n - 3; k >= 0; --k) {
        const double t = tau[k];
        if (t == 0.0) continue;
        reflect_row(row, act, k + 1, n - k - 1, a + (int64_t)k * ld + k + 1, t);
    }
    // D L = u: D_j = (u_j - sum_{i>j} D_i L_ij) / L_jj, from the last column
    if (act)
        for (int j = n - 1; j >= 0; --j) {
            double acc = row[j];
            for (int i = j + 1; i < n; ++i) acc -= row[i] * l[(int64_t)i * ld + j];
            row[j] = acc / l[(int64_t)j * ld + j];
        }
    __syncthreads();
    double* out = Dout + d.offd;
    for (int rr = 0; rr < nr; ++rr)
        for (int jj = lane; jj < n; jj += kRowThreads) out[(int64_t)(r0 + rr) * n + jj] = rows[(int64_t)rr * S + jj];
}

// ------------------------------------------------ chemical potential
// Multisection on N(mu) = 2 sum w f(lam - mu): each round evaluates K
// candidates mu_j = lo + (hi - lo) j/(K+1); the new interval is the one where
// N crosses n_e (same rule as bisection: N(mid) < n_e -> lo = mid).
constexpr int kMuK = 256;

__global__ void __launch_bounds__(kMuK) k_mu_bounds(const SubDesc* __restrict__ desc, int n_sub,
                                                   const double* __restrict__ Lam, double* __restrict__ state) {
    __shared__ double smin[kMuK], smax[kMuK];
    double lo = INFINITY, hi = -INFINITY;
    for (int s = 0; s < n_sub; ++s) {
        const SubDesc d = desc[s];
        for (int k = threadIdx.x; k < d.n; k += kMuK) {
            double v = Lam[d.offv + k];
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int o = kMuK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        state[0] = smin[0] - 1.0;   // lo
        state[1] = smax[0] + 1.0;   // hi
        state[2] = 0.0;             // mu
        state[3] = 0.0;             // N(mu)
    }
}

// partial[s * K + j] = 2 sum_k w_k f(lam_k - mu_j) over subgraph s
__global__ void __launch_bounds__(kMuK) k_mu_partial(const SubDesc* __restrict__ desc,
                                                    const double* __restrict__ Lam, const double* __restrict__ Wt,
                                                    const double* __restrict__ state, double beta, int final_pass,
                                                    double* __restrict__ partial) {
    extern __shared__ double lw[];    // lam [n], w [n]
    const SubDesc d = desc[blockIdx.x];
    const int n = d.n;
    for (int k = threadIdx.x; k < n; k += kMuK) {
        lw[k] = Lam[d.offv + k];
        lw[n + k] = Wt[d.offv + k];
    }
    __syncthreads();
    const double lo = state[0], hi = state[1];
    const int j = threadIdx.x;
    const double mu = final_pass ? state[2] : lo + (hi - lo) * ((double)(j + 1) / (double)(kMuK + 1));
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += lw[n + k] * fermi_fp64(lw[k] - mu, beta);
    partial[(int64_t)blockIdx.x * kMuK + j] = 2.0 * acc;
}

__global__ void __launch_bounds__(kMuK) k_mu_pick(int n_sub, const double* __restrict__ partial, double n_e,
                                                 int final_pass, double tol, double* __restrict__ state,
                                                 int* __restrict__ status) {
    __shared__ double Nj[kMuK];
    const int j = threadIdx.x;
    double acc = 0.0;
    for (int s = 0; s < n_sub; ++s) acc += partial[(int64_t)s * kMuK + j];
    Nj[j] = acc;
    __syncthreads();
    if (j == 0) {
        if (final_pass) {
            state[3] = Nj[0];
            return;
        }
        double lo = state[0], hi = state[1];
        if (hi - lo > tol) {
            int first = kMuK;   // first candidate with N >= n_e
            for (int q = 0; q < kMuK; ++q)
                if (!(Nj[q] < n_e)) {
                    first = q;
                    break;
                }
            double nlo = first == 0 ? lo : lo + (hi - lo) * ((double)first / (double)(kMuK + 1));
            double nhi = first == kMuK ? hi : lo + (hi - lo) * ((double)(first + 1) / (double)(kMuK + 1));
            state[0] = nlo;
            state[1] = nhi;
        }
        state[2] = 0.5 * (state[0] + state[1]);
    }
}

// Final step of the device-output mode of the search: copy mu and N(mu) to
// the caller's device scalars and raise the status word when the count
// misses n_e by more than tol (or is not finite).
__global__ void k_mu_out(const double* __restrict__ state, double n_e, double tol, double* __restrict__ mu_out,
                         double* __restrict__ n_out, int* __restrict__ status) {
    if (threadIdx.x != 0) return;
    const double mu = state[2], n = state[3];
    mu_out[0] = mu;
    n_out[0] = n;
    if (!isfinite(mu) || !isfinite(n)) gdm_raise(status, GDM_STATUS_NAN);
    else if (fabs(n - n_e) > tol) gdm_raise(status, GDM_STATUS_NO_BRACKET);
}

}  // namespace

// ----------------------------------------------------------------- host

// Dynamic LDS above 64 KiB needs the kernel attribute raised first.  The
// largest value set so far is remembered per device and kernel, so the
// attribute call happens at plan time and never inside a solve call (which
// may be under stream capture).
static int set_lds(gdm_ctx* ctx, const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return GDM_OK;
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> raised;
    std::lock_guard<std::mutex> lock(mu);
    size_t& have = raised[{ctx->device, fn}];
    if (bytes <= have) return GDM_OK;
    GDM_HIP(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    have = bytes;
    return GDM_OK;
}

// LDS bytes of the FP64 kernels for a plan: one matrix row or column
// (lds_n), the core-row kernel's row chunks and the density kernel's.
struct Fp64Lds {
    size_t n = 0, core_rows = 0, dcore = 0;
    int core_chunks = 1, dcore_chunks = 1;
};

static Fp64Lds fp64_lds(const Plan& P) {
    Fp64Lds L;
    L.n = sizeof(double) * (size_t)P.max_n;
    for (int s = 0; s < P.n_sub; ++s) {
        const SubDesc& dd = P.desc[s];
        const int rcn = chunk_rows(dd.n);
        const size_t rows = sizeof(double) * (size_t)rcn * (dd.n + 1);
        L.core_rows = std::max(L.core_rows, rows);
        L.dcore = std::max(L.dcore, rows);
        L.core_chunks = std::max(L.core_chunks, (2 * dd.nc + rcn - 1) / rcn);
        L.dcore_chunks = std::max(L.dcore_chunks, (dd.nc + rcn - 1) / rcn);
    }
    return L;
}

int gdm_fp64_plan_lds(gdm_ctx* ctx) {
    const Fp64Lds L = fp64_lds(ctx->plan);
    int rc;
    if ((rc = set_lds(ctx, (const void*)k_potrf, L.n))) return rc;
    if ((rc = set_lds(ctx, (const void*)k_sytrd, 2 * L.n))) return rc;
    if ((rc = set_lds(ctx, (const void*)k_steqr, 2 * L.n))) return rc;
    if ((rc = set_lds(ctx, (const void*)k_core_rows, L.core_rows))) return rc;
    if ((rc = set_lds(ctx, (const void*)k_mu_partial, 2 * L.n))) return rc;
    return set_lds(ctx, (const void*)k_dcore, L.dcore);
}

int gdm_fp64_find_mu(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg, const int32_t* row_ptr,
                     const int32_t* col, int64_t nnz, const double* H, const double* S, double n_e, double kT,
                     double* mu_out, double* n_out) {
    Plan& P = ctx->plan;
    const int ns = P.n_sub;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    double* A = (double*)ctx->b[BUF_A].p;
    double* Sd = (double*)ctx->b[BUF_S].p;
    double* T = (double*)ctx->b[BUF_L].p;
    double* Dg = (double*)ctx->b[BUF_D].p;
    double* Eg = (double*)ctx->b[BUF_E].p;
    double* Tau = (double*)ctx->b[BUF_TAU].p;
    double* Lam = (double*)ctx->b[BUF_LAM].p;
    double* Wt = (double*)ctx->b[BUF_W].p;
    double* RotC = (double*)ctx->b[BUF_ROTC].p;
    double* RotS = (double*)ctx->b[BUF_ROTS].p;
    int32_t* RotI = (int32_t*)ctx->b[BUF_ROTI].p;
    int64_t* RotN = (int64_t*)ctx->b[BUF_ROTN].p;
    double* G = (double*)ctx->b[BUF_QC].p;
    double* state = (double*)ctx->b[BUF_MU].p;
    double* partial = (double*)ctx->b[BUF_MUPART].p;
    const int orth = S == nullptr;
    int rc;
    if ((rc = gdm_launch_gather(ctx, sys, sg, row_ptr, col, nnz, H, S, A, Sd, orth))) return rc;
    const Fp64Lds L = fp64_lds(P);
    const size_t lds_n = L.n;
    if ((rc = set_lds(ctx, (const void*)k_potrf, lds_n))) return rc;
    GDM_LAUNCH_CHECK(ctx);
    { GDM_TIMED(ctx, "potrf");
    hipLaunchKernelGGL(k_potrf, dim3(ns), dim3(kThreads), lds_n, ctx->stream, desc, Sd, ctx->d_status);
    }
    GDM_LAUNCH_CHECK(ctx);
    { GDM_TIMED(ctx, "trsm");
    hipLaunchKernelGGL(k_trsm<0>, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, Sd, A, T);
    }
    GDM_LAUNCH_CHECK(ctx);
    { GDM_TIMED(ctx, "trsm");
    hipLaunchKernelGGL(k_trsm<1>, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, Sd, A, T);
    }
    GDM_LAUNCH_CHECK(ctx);
    { GDM_TIMED(ctx, "symmetrize");
    hipLaunchKernelGGL(k_symmetrize, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, A);
    }
    GDM_LAUNCH_CHECK(ctx);
    if ((rc = set_lds(ctx, (const void*)k_sytrd, 2 * lds_n))) return rc;
    { GDM_TIMED(ctx, "sytrd");
    hipLaunchKernelGGL(k_sytrd, dim3(ns), dim3(kThreads), 2 * lds_n, ctx->stream, desc, A, Dg, Eg, Tau);
    }
    GDM_LAUNCH_CHECK(ctx);
    if ((rc = set_lds(ctx, (const void*)k_steqr, 2 * lds_n))) return rc;
    { GDM_TIMED(ctx, "steqr");
    hipLaunchKernelGGL(k_steqr, dim3(ns), dim3(64), 2 * lds_n, ctx->stream, desc, Dg, Eg, Lam, RotC, RotS, RotI,
                       RotN, ctx->d_status);
    }
    GDM_LAUNCH_CHECK(ctx);
    {
        const size_t lds_rows = L.core_rows;
        const int chunks = L.core_chunks;
        if ((rc = set_lds(ctx, (const void*)k_core_rows, lds_rows))) return rc;
        GDM_TIMED(ctx, "core_rows");
        hipLaunchKernelGGL(k_core_rows, dim3(ns, chunks), dim3(kRowThreads), lds_rows, ctx->stream, desc, Sd, A, Tau,
                           RotC, RotS, RotI, RotN, G);
        GDM_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_core_weights, dim3(ns), dim3(kThreads), 0, ctx->stream, desc, Sd, G, Wt);
    }
    GDM_LAUNCH_CHECK(ctx);
    // chemical potential: multisection rounds
    const double beta = 1.0 / kT;
    GDM_TIMED(ctx, "mu");
    hipLaunchKernelGGL(k_mu_bounds, dim3(1), dim3(kMuK), 0, ctx->stream, desc, ns, Lam, state);
    GDM_LAUNCH_CHECK(ctx);
    const size_t lds_lw = 2 * lds_n;
    if ((rc = set_lds(ctx, (const void*)k_mu_partial, lds_lw))) return rc;
    const int rounds = 7;   // 257^7 > 1e16: any bracket narrower than 1e4 eV reaches 1e-12 eV
    for (int it = 0; it < rounds; ++it) {
        hipLaunchKernelGGL(k_mu_partial, dim3(ns), dim3(kMuK), lds_lw, ctx->stream, desc, Lam, Wt, state, beta, 0,
                           partial);
        GDM_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_mu_pick, dim3(1), dim3(kMuK), 0, ctx->stream, ns, partial, n_e, 0, 1e-12, state,
                           ctx->d_status);
        GDM_LAUNCH_CHECK(ctx);
    }
    hipLaunchKernelGGL(k_mu_partial, dim3(ns), dim3(kMuK), lds_lw, ctx->stream, desc, Lam, Wt, state, beta, 1,
                       partial);
    GDM_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_mu_pick, dim3(1), dim3(kMuK), 0, ctx->stream, ns, partial, n_e, 1, 1e-12, state,
                       ctx->d_status);
    GDM_LAUNCH_CHECK(ctx);
    if (ctx->mu_out_device) {
        // device scalars, no host synchronisation: the count check raises the
        // status word, which gdm_check reports
        hipLaunchKernelGGL(k_mu_out, dim3(1), dim3(64), 0, ctx->stream, state, n_e, 1e-6 * std::max(1.0, n_e), mu_out,
                           n_out, ctx->d_status);
        GDM_LAUNCH_CHECK(ctx);
        return GDM_OK;
    }
    double hs[4];
    GDM_HIP(ctx, hipMemcpyAsync(hs, state, sizeof(hs), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *mu_out = hs[2];
    *n_out = hs[3];
    return GDM_OK;
}

int gdm_fp64_density(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, const double* mu_dev, double kT,
                     double* D_core, double* eig_out) {
    Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    int rc;
    const Fp64Lds L = fp64_lds(P);
    const size_t lds_rows = L.dcore;
    const int chunks = L.dcore_chunks;
    if ((rc = set_lds(ctx, (const void*)k_dcore, lds_rows))) return rc;
    { GDM_TIMED(ctx, "dcore");
    hipLaunchKernelGGL(k_dcore, dim3(P.n_sub, chunks), dim3(kRowThreads), lds_rows, ctx->stream, desc,
                       (const double*)ctx->b[BUF_S].p, (const double*)ctx->b[BUF_A].p, (const double*)ctx->b[BUF_TAU].p,
                       (const double*)ctx->b[BUF_ROTC].p, (const double*)ctx->b[BUF_ROTS].p,
                       (const int32_t*)ctx->b[BUF_ROTI].p, (const int64_t*)ctx->b[BUF_ROTN].p,
                       (const double*)ctx->b[BUF_QC].p, (const double*)ctx->b[BUF_LAM].p, mu, mu_dev, 1.0 / kT, D_core,
                       eig_out);
    }
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}
