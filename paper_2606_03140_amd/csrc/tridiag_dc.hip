// Divide and conquer for the symmetric tridiagonal eigenproblem of the FP64
// path (the tridiagonal T = Hh^T h_perp Hh left by the Householder reduction).
//
// T is cut recursively at balanced points into leaves of at most 64 rows.  A
// cut between rows m-1 and m writes T as diag(T1, T2) + rho v v^T with
// v = e_{m-1} + sign(e) e_m, rho = |e_{m-1}| (Cuppen's rank-one tearing; the
// two diagonal entries next to the cut lose rho).  Leaves are solved by the
// implicit QL iteration with the eigenvector matrix accumulated (one wave per
// leaf).  Each merge turns the eigenpairs of its two children into those of
// diag(D1, D2) + rho z z^T, z = (last row of Q1, sign(e) first row of Q2):
//   * sort the poles d, then deflate (published method: Dongarra & Sorensen,
//     SIAM J. Sci. Stat. Comput. 8 (1987)): a component with negligible
//     rho |z_i| keeps (d_i, e_i); two close poles are rotated so that one z
//     component vanishes, the rotated pair forming chains;
//   * the remaining roots of 1/rho + sum z_i^2 / (d_i - x) = 0, one per gap
//     between poles, are found relative to the nearer pole (x = d_o + tau)
//     by a two-pole rational model step (Bunch, Nielsen & Sorensen, Numer.
//     Math. 31 (1978)) safeguarded by bisection;
//   * z is recomputed from the roots (Gu & Eisenstat, SIAM J. Matrix Anal.
//     Appl. 16 (1995)) and the eigenvectors are u_j = zhat / (d - x_j),
//     normalised, so they are orthogonal to working precision.
// Every merge stores its k x k orthogonal factor U (rows: the children's
// eigenvector columns, columns: the merged eigenpairs, in no particular
// order), so V_T = B_leaf B_1 ... B_top with B_l block diagonal.  The
// eigenvectors themselves are never formed: the 2 nc core rows are multiplied
// by the factors level by level (k_dc_apply, leaves first) and the density's
// nc rows by their transposes (top first), as batched FP64 products.
#include "gdm_internal.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

namespace {

constexpr double kEps = 2.220446049250313e-16;   // 2^-52
constexpr int kLeafMax = 64;                     // leaf rows (one wave)
constexpr int kMergeThreads = 512;      // threads per merge workgroup
constexpr int kMergeThreadsFew = 1024;  // when a round has fewer merges than CUs
constexpr int kMergeBytesPerRow = 7 * 8 + 4 * 4; // LDS of the merge kernel per row of the block

__host__ __device__ inline int dc_bound(int n, int level, int i) {
    return (int)(((int64_t)i * n) >> level);
}

// ---------------------------------------------------------------- leaves
// One wave per leaf.  The QL iteration (uniform: every lane computes the same
// scalars from d, e in LDS) applies each plane rotation to the columns
// (i, i+1) of V, lane r updating row r.  Output: eigenvalues (unsorted), V
// row-major as the leaf's factor, and V's first and last rows.
__global__ void __launch_bounds__(kLeafMax) k_dc_leaf(const SubDesc* __restrict__ desc,
                                                      const DcNode* __restrict__ nodes,
                                                      const double* __restrict__ Dg, const double* __restrict__ Eg,
                                                      double* __restrict__ LamA, double* __restrict__ LamB,
                                                      double* __restrict__ FrA, double* __restrict__ FrB,
                                                      double* __restrict__ LrA, double* __restrict__ LrB,
                                                      double* __restrict__ U, int* __restrict__ status) {
    constexpr int S = kLeafMax + 1;
    __shared__ double d[kLeafMax], e[kLeafMax], V[kLeafMax * S];
    const DcNode nd = nodes[blockIdx.x];
    const SubDesc sd = desc[nd.sub];
    const int lo = nd.lo, b = nd.hi - nd.lo, n = sd.n;
    const int lane = threadIdx.x;
    const double* dg = Dg + sd.offv;
    const double* eg = Eg + sd.offv;
    if (lane < b) {
        d[lane] = dg[lo + lane];
        e[lane] = lane + 1 < b ? eg[lo + lane] : 0.0;
        for (int c = 0; c < b; ++c) V[lane * S + c] = lane == c ? 1.0 : 0.0;
    }
    __syncthreads();
    if (lane == 0) {
        // the tears at both ends of the leaf
        if (lo > 0) d[0] -= fabs(eg[lo - 1]);
        if (nd.hi < n) d[b - 1] -= fabs(eg[nd.hi - 1]);
    }
    __syncthreads();
    const double eps = 1.1102230246251565e-16;
    bool bad = false;
    for (int l = 0; l < b && !bad; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < b - 1; ++m) {
                const double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) {
                bad = true;
                if (lane == 0) gdm_raise(status, GDM_STATUS_NOT_CONVERGED);
                break;
            }
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool underflow = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i], bb = c * e[i];
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
                r = (d[i] - g) * s + 2.0 * c * bb;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - bb;
                if (lane < b) {
                    double* v = V + lane * S;
                    const double a0 = v[i], a1 = v[i + 1];
                    v[i] = c * a0 - s * a1;
                    v[i + 1] = s * a0 + c * a1;
                }
            }
            if (underflow) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    __syncthreads();
    const int pb = nd.level & 1;
    const int64_t o = sd.offv + lo;
    if (lane < b) {
        (pb ? LamB : LamA)[o + lane] = d[lane];
        (pb ? FrB : FrA)[o + lane] = V[lane];
        (pb ? LrB : LrA)[o + lane] = V[(b - 1) * S + lane];
    }
    double* u = U + nd.offu;
    for (int r = 0; r < b; ++r)
        if (lane < b) u[r * b + lane] = V[r * S + lane];
}

// --------------------------------------------------------------- secular
// Root j of 1/r2 + sum_i z_i^2 / (d_i - x) = 0 (d strictly increasing,
// r2 > 0) as x = d[o] + tau.  The root lies in (d_j, d_j+1) (j < K-1) or in
// (d_j, d_j + r2 |z|^2]; the sign of the secular function at the middle of
// the gap picks the nearer pole as origin.  Each step fits the poles left of
// and at d_j (psi) and right of it (phi) with one pole each, matching value
// and slope, and solves the resulting quadratic; a step that leaves the
// bracket is replaced by bisection.
__device__ double dc_root(const double* __restrict__ dn, const double* __restrict__ zn, int K, double r2, int j,
                          int* origin) {
    const double inv = 1.0 / r2;
    int o;
    double a, b;
    if (j < K - 1) {
        const double h = 0.5 * (dn[j + 1] - dn[j]);
        double f = inv;
        for (int i = 0; i < K; ++i) f += zn[i] * zn[i] / ((dn[i] - dn[j]) - h);
        if (f >= 0.0) {
            o = j;
            a = 0.0;
            b = h;
        } else {
            o = j + 1;
            a = -h;
            b = 0.0;
        }
    } else {
        double zz = 0.0;
        for (int i = 0; i < K; ++i) zz += zn[i] * zn[i];
        o = j;
        a = 0.0;
        b = r2 * zz;
    }
    *origin = o;
    const double dor = dn[o];
    double tau = 0.5 * (a + b);
    for (int it = 0; it < 96; ++it) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
        for (int i = 0; i < K; ++i) {
            const double q = zn[i] / ((dn[i] - dor) - tau);
            if (i <= j) {
                psi += zn[i] * q;
                dpsi += q * q;
            } else {
                phi += zn[i] * q;
                dphi += q * q;
            }
        }
        const double f = inv + psi + phi;
        if (f == 0.0) break;
        if (f > 0.0) b = tau;
        else a = tau;
        const double err = 8.0 * (inv + fabs(psi) + fabs(phi)) + fabs(tau) * (dpsi + dphi);
        if (fabs(f) <= kEps * err) break;
        if (b - a <= 2.0 * kEps * fmax(fabs(a), fabs(b))) break;
        double nt = NAN;
        const double DA = (dn[j] - dor) - tau;
        if (j < K - 1) {
            const double DB = (dn[j + 1] - dor) - tau;
            const double q1 = dpsi * DA * DA, q2 = dphi * DB * DB;
            const double c0 = inv + (psi - dpsi * DA) + (phi - dphi * DB);
            const double B1 = c0 * (DA + DB) + q1 + q2, C0 = DA * DB * f;
            const double disc = B1 * B1 - 4.0 * c0 * C0;
            if (disc >= 0.0) {
                const double sq = sqrt(disc);
                double e1, e2;
                if (B1 >= 0.0) {
                    e1 = (B1 + sq) / (2.0 * c0);
                    e2 = 2.0 * C0 / (B1 + sq);
                } else {
                    e1 = 2.0 * C0 / (B1 - sq);
                    e2 = (B1 - sq) / (2.0 * c0);
                }
                double eta = NAN;
                if (isfinite(e1) && e1 > DA && e1 < DB) eta = e1;
                if (isfinite(e2) && e2 > DA && e2 < DB && (isnan(eta) || fabs(e2) < fabs(eta))) eta = e2;
                nt = tau + eta;
            }
        } else {
            const double c0 = inv + (psi - dpsi * DA);
            if (c0 > 0.0) nt = tau + DA + dpsi * DA * DA / c0;
        }
        if (!(nt > a && nt < b)) nt = 0.5 * (a + b);
        tau = nt;
    }
    return tau;
}

// ----------------------------------------------------------------- merge
// One workgroup per merge.  Children (level + 1) hold their eigenvalues and
// first / last eigenvector rows at [lo, mid) and [mid, hi) of the buffers of
// parity (level + 1) & 1; the merge writes its own at parity level & 1 and
// its factor U (k x k, row-major) at offu.  Chain records (cosine, sine,
// next, previous) live in global scratch at [lo, hi).
template <int MT>
__global__ void __launch_bounds__(MT) k_dc_merge(
    const SubDesc* __restrict__ desc, const DcNode* __restrict__ nodes, const double* __restrict__ Eg,
    double* __restrict__ LamA, double* __restrict__ LamB, double* __restrict__ FrA, double* __restrict__ FrB,
    double* __restrict__ LrA, double* __restrict__ LrB, double* __restrict__ Cs, double* __restrict__ Sn,
    int32_t* __restrict__ Nx, int32_t* __restrict__ Pv, double* __restrict__ U) {
    extern __shared__ double sm[];
    __shared__ int sK;
    const DcNode nd = nodes[blockIdx.x];
    const SubDesc sd = desc[nd.sub];
    const int lo = nd.lo, k1 = nd.mid - nd.lo, k = nd.hi - nd.lo;
    double* ds = sm;          // sorted poles (deflated values in place)
    double* ws = ds + k;      // sorted z, then the weight of each position in its owner's vector
    double* dn = ws + k;      // undeflated poles (first: unsorted children eigenvalues)
    double* zh = dn + k;      // undeflated z, then zhat (first: unsorted z)
    double* tau = zh + k;     // roots relative to their origin
    double* f1x = tau + k;    // first row of child 1 (zero over child 2)
    double* l2x = f1x + k;    // last row of child 2 (zero over child 1)
    int32_t* src = (int32_t*)(l2x + k);   // sorted position -> children index
    int32_t* ndp = src + k;               // undeflated item -> sorted position
    int32_t* org = ndp + k;               // root -> origin item; [K, k): deflated positions
    int32_t* own = org + k;               // position -> owning undeflated item (-2: alone, -3: chained)
    const int tid = threadIdx.x;
    const int cb = (nd.level + 1) & 1, ob = nd.level & 1;
    const int64_t o = sd.offv + lo;
    const double* lamc = (cb ? LamB : LamA) + o;
    const double* fc = (cb ? FrB : FrA) + o;
    const double* lc = (cb ? LrB : LrA) + o;
    const double et = Eg[sd.offv + nd.mid - 1];
    const double r2 = 2.0 * fabs(et);
    const double sg = et < 0.0 ? -1.0 : 1.0;
    double* cs = Cs + o;
    double* sn = Sn + o;
    int32_t* nx = Nx + o;
    int32_t* pv = Pv + o;
    for (int t = tid; t < k; t += MT) {
        dn[t] = lamc[t];
        zh[t] = (t < k1 ? lc[t] : sg * fc[t]) * 0.70710678118654752440;
        f1x[t] = t < k1 ? fc[t] : 0.0;
        l2x[t] = t < k1 ? 0.0 : lc[t];
        nx[t] = -1;
        pv[t] = -1;
        src[t] = t;       // a valid index even if non-finite values leave a rank unfilled
    }
    __syncthreads();
    // stable rank sort of the poles
    for (int t = tid; t < k; t += MT) {
        const double v = dn[t];
        int r = 0;
        for (int u = 0; u < k; ++u) {
            const double w = dn[u];
            r += (w < v) || (w == v && u < t);
        }
        ds[r] = v;
        ws[r] = zh[t];
        src[r] = t;
    }
    __syncthreads();
    // deflation, in pole order (one lane)
    if (tid == 0) {
        double dmax = 0.0, zmax = 0.0;
        for (int p = 0; p < k; ++p) {
            dmax = fmax(dmax, fabs(ds[p]));
            zmax = fmax(zmax, fabs(ws[p]));
        }
        const double tol = 8.0 * kEps * fmax(dmax, zmax);
        int K = 0, Kd = 0, pj = -1;
        for (int j = 0; j < k; ++j) {
            if (r2 * fabs(ws[j]) <= tol) {
                own[j] = -2;
                org[k - 1 - Kd++] = j;
                continue;
            }
            if (pj < 0) {
                pj = j;
                continue;
            }
            // rotate (pj, j) so that z_pj vanishes; keep it if the neglected
            // coupling c s (d_j - d_pj) is below the tolerance
            const double r = hypot(ws[pj], ws[j]);
            const double c = ws[j] / r, s = ws[pj] / r;
            if (fabs((ds[j] - ds[pj]) * c * s) <= tol) {
                const double dp = c * c * ds[pj] + s * s * ds[j];
                const double dq = s * s * ds[pj] + c * c * ds[j];
                ds[pj] = dp;
                ds[j] = dq;
                ws[j] = r;
                ws[pj] = 0.0;
                own[pj] = -3;
                nx[pj] = j;
                pv[j] = pj;
                cs[pj] = c;
                sn[pj] = s;
                org[k - 1 - Kd++] = pj;
            } else {
                own[pj] = K;
                ndp[K++] = pj;
            }
            pj = j;
        }
        if (pj >= 0) {
            own[pj] = K;
            ndp[K++] = pj;
        }
        sK = K;
    }
    __syncthreads();
    const int K = sK;
    for (int i = tid; i < K; i += MT) {
        const int p = ndp[i];
        dn[i] = ds[p];
        zh[i] = ws[p];
    }
    __syncthreads();
    for (int j = tid; j < K; j += MT) {
        int og;
        tau[j] = dc_root(dn, zh, K, r2, j, &og);
        org[j] = og;
    }
    __syncthreads();
    // zhat_i^2 = prod_j (x_j - d_i) / (r2 prod_{j != i} (d_j - d_i)), each
    // root paired with an adjacent pole so every factor is a positive ratio
    for (int i = tid; i < K; i += MT) {
        const double di = dn[i];
        double v = ((dn[org[K - 1]] - di) + tau[K - 1]) / r2;
        for (int j = 0; j < K - 1; ++j) v *= ((dn[org[j]] - di) + tau[j]) / ((j < i ? dn[j] : dn[j + 1]) - di);
        zh[i] = copysign(sqrt(fmax(v, 0.0)), zh[i]);
    }
    __syncthreads();
    // weights: an undeflated position owns itself (weight 1); a chain
    // a_1 .. a_m (rotations (a_t, a_t+1)) is owned by its survivor a_m with
    // weight c_{i-1} prod_{t >= i} s_t at a_i
    for (int p = tid; p < k; p += MT)
        if (own[p] == -2) ws[p] = 0.0;
    for (int i = tid; i < K; i += MT) {
        int q = ndp[i];
        double P = 1.0;
        for (;;) {
            const int pq = pv[q];
            ws[q] = (pq >= 0 ? cs[pq] : 1.0) * P;
            own[q] = i;
            if (pq < 0) break;
            P *= sn[pq];
            q = pq;
        }
    }
    __syncthreads();
    // columns of U: items [0, K) are the roots, [K, k) the deflated positions
    double* lam = (ob ? LamB : LamA) + o;
    double* fo = (ob ? FrB : FrA) + o;
    double* lo_ = (ob ? LrB : LrA) + o;
    double* u = U + nd.offu;
    for (int t = tid; t < k; t += MT) {
        double fs = 0.0, ls = 0.0, ev;
        if (t < K) {
            const double dor = dn[org[t]], tt = tau[t];
            ev = dor + tt;
            double nrm = 0.0;
            for (int i = 0; i < K; ++i) {
                const double x = zh[i] / ((dn[i] - dor) - tt);
                nrm += x * x;
            }
            const double inv = 1.0 / sqrt(nrm);
            for (int p = 0; p < k; ++p) {
                const int ow = own[p];
                const double x = ow >= 0 ? zh[ow] / ((dn[ow] - dor) - tt) * inv * ws[p] : 0.0;
                const int row = src[p];
                u[(int64_t)row * k + t] = x;
                fs += f1x[row] * x;
                ls += l2x[row] * x;
            }
        } else {
            const int p0 = org[t];
            ev = ds[p0];
            for (int p = 0; p < k; ++p) u[(int64_t)src[p] * k + t] = 0.0;
            const int q1 = nx[p0];
            if (q1 < 0) {
                const int row = src[p0];
                u[(int64_t)row * k + t] = 1.0;
                fs = f1x[row];
                ls = l2x[row];
            } else {
                // c_t v_t - s_t e_{a_t+1}, v_t[a_i] = c_{i-1} prod_{i <= u < t} s_u
                const double ct = cs[p0], st = sn[p0];
                {
                    const int row = src[q1];
                    u[(int64_t)row * k + t] = -st;
                    fs -= f1x[row] * st;
                    ls -= l2x[row] * st;
                }
                int q = p0;
                double P = 1.0;
                for (;;) {
                    const int pq = pv[q];
                    const double x = ct * (pq >= 0 ? cs[pq] : 1.0) * P;
                    const int row = src[q];
                    u[(int64_t)row * k + t] = x;
                    fs += f1x[row] * x;
                    ls += l2x[row] * x;
                    if (pq < 0) break;
                    P *= sn[pq];
                    q = pq;
                }
            }
        }
        lam[t] = ev;
        fo[t] = fs;
        lo_[t] = ls;
    }
}

// ----------------------------------------------------------------- apply
// Out[r, lo + c] = sum_t In[r, lo + t] F[t, c] over one block of one level,
// F = U (forward, leaves first) or U^T (reverse, top first), on 64 x 64
// output tiles.  Rows are stored column-major with leading dimension R
// (forward: the 2 nc core rows, R = 2 nc; reverse: the nc density rows).
// Forward: level l reads parity (l + 1) & 1 and writes l & 1, so the top
// level ends in buffer 0; reverse: level l reads (depth + 1 + l) & 1, so the
// leaf level ends in buffer 0.
constexpr int kAT = 64, kAK = 16;

template <bool REV>
__global__ void __launch_bounds__(256) k_dc_apply(const SubDesc* __restrict__ desc, const DcTile* __restrict__ tiles,
                                                  const double* __restrict__ U, double* __restrict__ buf0,
                                                  double* __restrict__ buf1) {
    __shared__ double sA[kAK][kAT];
    __shared__ double sB[kAK][kAT + 1];
    const DcTile tl = tiles[blockIdx.x];
    const SubDesc sd = desc[tl.sub];
    const int R = REV ? sd.nc : 2 * sd.nc, k = tl.k;
    const int pin = REV ? ((sd.dc_depth + 1 + tl.level) & 1) : ((tl.level + 1) & 1);
    // forward: buffers 0 / 1 are two arrays; reverse: two halves of one
    const int64_t base = 2 * sd.offc;
    const int64_t half = (int64_t)sd.nc * sd.ld;
    const double* X = REV ? buf0 + base + (pin ? half : 0) : (pin ? buf1 : buf0) + base;
    double* Y = REV ? buf0 + base + (pin ? 0 : half) : (pin ? buf0 : buf1) + base;
    const double* u = U + tl.offu;
    const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int t0 = 0; t0 < k; t0 += kAK) {
        for (int e = threadIdx.x; e < kAT * kAK; e += 256) {
            const int rr = e & (kAT - 1), tt = e >> 6;
            const int r = tl.r0 + rr, t = t0 + tt;
            sA[tt][rr] = (r < R && t < k) ? X[(int64_t)(tl.lo + t) * R + r] : 0.0;
        }
        for (int e = threadIdx.x; e < kAT * kAK; e += 256) {
            int tt, cc;
            if (REV) {
                tt = e & (kAK - 1);
                cc = e >> 4;
            } else {
                cc = e & (kAT - 1);
                tt = e >> 6;
            }
            const int t = t0 + tt, c = tl.c0 + cc;
            double v = 0.0;
            if (t < k && c < k) v = REV ? u[(int64_t)c * k + t] : u[(int64_t)t * k + c];
            sB[tt][cc] = v;
        }
        __syncthreads();
#pragma unroll
        for (int tt = 0; tt < kAK; ++tt) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sA[tt][tr + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sB[tt][tc + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = tl.c0 + tc + 16 * j;
        if (c >= k) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = tl.r0 + tr + 16 * i;
            if (r < R) Y[(int64_t)(tl.lo + c) * R + r] = acc[i][j];
        }
    }
}

}  // namespace

// ----------------------------------------------------------------- host

static int dc_set_lds(gdm_ctx* ctx, const void* fn, size_t bytes) {
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

int gdm_dc_depth(int n, int leaf) {
    int L = 0;
    while (((int64_t)n + (1LL << L) - 1) >> L > leaf) ++L;
    return L;
}

extern "C" int gdm_set_fp64_options(gdm_ctx* ctx, int leaf_rows) {
    if (!ctx) return GDM_E_ARG;
    if (leaf_rows < 8 || leaf_rows > kLeafMax)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_set_fp64_options: leaf_rows %d outside [8, %d]", leaf_rows, kLeafMax);
    ctx->fp64_leaf = leaf_rows;
    return GDM_OK;
}

int gdm_dc_plan(gdm_ctx* ctx) {
    Plan& P = ctx->plan;
    const int ns = P.n_sub;
    P.dc_nodes.clear();
    P.dc_tiles.clear();
    int maxL = 0;
    for (int s = 0; s < ns; ++s) {
        if (P.n[s] > kDcMaxRows)
            return gdm_fail(ctx, GDM_E_ARG, "gdm_plan: subgraph %d has %d orbitals; the FP64 path takes at most %d", s,
                            P.n[s], kDcMaxRows);
        P.desc[s].dc_depth = gdm_dc_depth(P.n[s], ctx->fp64_leaf);
        maxL = std::max(maxL, P.desc[s].dc_depth);
    }
    P.dc_max_depth = maxL;
    // factor offsets, per subgraph and level
    std::vector<std::vector<int64_t>> uoff(ns);
    int64_t totu = 0;
    for (int s = 0; s < ns; ++s) {
        const int n = P.n[s], L = P.desc[s].dc_depth;
        uoff[s].assign(L + 1, 0);
        for (int l = L; l >= 0; --l) {
            uoff[s][l] = totu;
            for (int i = 0; i < (1 << l); ++i) {
                const int64_t kk = dc_bound(n, l, i + 1) - dc_bound(n, l, i);
                totu += kk * kk;
            }
        }
    }
    P.dc_totu = totu;
    auto blk_off = [&](int s, int l, int i) {
        int64_t off = uoff[s][l];
        for (int q = 0; q < i; ++q) {
            const int64_t kk = dc_bound(P.n[s], l, q + 1) - dc_bound(P.n[s], l, q);
            off += kk * kk;
        }
        return off;
    };
    // leaves, then merges by round (round r: level depth - r), largest subgraphs first
    P.dc_round.assign(maxL + 2, 0);
    int kmax = 0;
    for (int r = 0; r <= maxL; ++r) {
        P.dc_round[r] = (int)P.dc_nodes.size();
        for (int q = 0; q < ns; ++q) {
            const int s = P.order[q], n = P.n[s], L = P.desc[s].dc_depth;
            if (r > L) continue;
            const int l = L - r;
            for (int i = 0; i < (1 << l); ++i) {
                DcNode nd{};
                nd.sub = s;
                nd.lo = dc_bound(n, l, i);
                nd.hi = dc_bound(n, l, i + 1);
                nd.mid = r == 0 ? nd.hi : dc_bound(n, l + 1, 2 * i + 1);
                nd.level = l;
                nd.offu = blk_off(s, l, i);
                if (r > 0) kmax = std::max(kmax, nd.hi - nd.lo);
                P.dc_nodes.push_back(nd);
            }
        }
    }
    P.dc_round[maxL + 1] = (int)P.dc_nodes.size();
    P.dc_merge_lds = (size_t)kMergeBytesPerRow * (size_t)std::max(kmax, 1);
    // product tiles: forward round r = depth - level, reverse round r = level
    auto add_tiles = [&](int s, int l, int rows) {
        const int n = P.n[s];
        for (int i = 0; i < (1 << l); ++i) {
            const int lo = dc_bound(n, l, i), k = dc_bound(n, l, i + 1) - lo;
            const int64_t off = blk_off(s, l, i);
            for (int c0 = 0; c0 < k; c0 += kAT)
                for (int r0 = 0; r0 < rows; r0 += kAT) {
                    DcTile t{};
                    t.sub = s;
                    t.lo = lo;
                    t.k = k;
                    t.level = l;
                    t.r0 = r0;
                    t.c0 = c0;
                    t.offu = off;
                    P.dc_tiles.push_back(t);
                }
        }
    };
    P.dc_fwd.assign(maxL + 2, 0);
    for (int r = 0; r <= maxL; ++r) {
        P.dc_fwd[r] = (int)P.dc_tiles.size();
        for (int q = 0; q < ns; ++q) {
            const int s = P.order[q], L = P.desc[s].dc_depth;
            if (r <= L) add_tiles(s, L - r, 2 * P.nc[s]);
        }
    }
    P.dc_fwd[maxL + 1] = (int)P.dc_tiles.size();
    P.dc_rev.assign(maxL + 2, 0);
    for (int r = 0; r <= maxL; ++r) {
        P.dc_rev[r] = (int)P.dc_tiles.size();
        for (int q = 0; q < ns; ++q) {
            const int s = P.order[q], L = P.desc[s].dc_depth;
            if (r <= L) add_tiles(s, r, P.nc[s]);
        }
    }
    P.dc_rev[maxL + 1] = (int)P.dc_tiles.size();
    // device copies
    bool ok = true;
    const size_t nb = sizeof(DcNode) * P.dc_nodes.size();
    const size_t tb = sizeof(DcTile) * P.dc_tiles.size();
    const size_t toff = (nb + 255) / 256 * 256;
    P.dc_tiles_off = toff;
    char* lst = (char*)gdm_buf(ctx, BUF_DCLIST, toff + tb, &ok);
    gdm_buf(ctx, BUF_DCU, sizeof(double) * (size_t)std::max<int64_t>(totu, 1), &ok);
    gdm_buf(ctx, BUF_DCAUX, sizeof(double) * 7 * (size_t)P.totv, &ok);
    gdm_buf(ctx, BUF_DCIDX, sizeof(int32_t) * 2 * (size_t)P.totv, &ok);
    gdm_buf(ctx, BUF_QC2, sizeof(double) * 2 * (size_t)P.totc, &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_plan: divide-and-conquer workspace allocation failed");
    GDM_HIP(ctx, hipMemcpyAsync(lst, P.dc_nodes.data(), nb, hipMemcpyHostToDevice, ctx->stream));
    GDM_HIP(ctx, hipMemcpyAsync(lst + toff, P.dc_tiles.data(), tb, hipMemcpyHostToDevice, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    int rc = dc_set_lds(ctx, (const void*)k_dc_merge<kMergeThreads>, P.dc_merge_lds);
    if (rc) return rc;
    return dc_set_lds(ctx, (const void*)k_dc_merge<kMergeThreadsFew>, P.dc_merge_lds);
}

// Eigenvalues (parity-0 buffer = the plan's eigenvalue array) and factors.
int gdm_dc_solve(gdm_ctx* ctx) {
    Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const DcNode* nodes = (const DcNode*)ctx->b[BUF_DCLIST].p;
    double* aux = (double*)ctx->b[BUF_DCAUX].p;
    const int64_t tv = P.totv;
    double* LamA = (double*)ctx->b[BUF_LAM].p;
    double *LamB = aux, *FrA = aux + tv, *FrB = aux + 2 * tv, *LrA = aux + 3 * tv, *LrB = aux + 4 * tv;
    double *Cs = aux + 5 * tv, *Sn = aux + 6 * tv;
    int32_t* idx = (int32_t*)ctx->b[BUF_DCIDX].p;
    double* U = (double*)ctx->b[BUF_DCU].p;
    const double* Dg = (const double*)ctx->b[BUF_D].p;
    const double* Eg = (const double*)ctx->b[BUF_E].p;
    {
        GDM_TIMED(ctx, "dc_leaf");
        const int nl = P.dc_round[1] - P.dc_round[0];
        hipLaunchKernelGGL(k_dc_leaf, dim3(nl), dim3(kLeafMax), 0, ctx->stream, desc, nodes, Dg, Eg, LamA, LamB, FrA,
                           FrB, LrA, LrB, U, ctx->d_status);
        GDM_LAUNCH_CHECK(ctx);
    }
    GDM_TIMED(ctx, "dc_merge");
    for (int r = 1; r <= P.dc_max_depth; ++r) {
        const int a = P.dc_round[r], b = P.dc_round[r + 1];
        if (b <= a) continue;
        // a round with fewer merges than CUs takes 1024 threads per merge (the
        // secular roots, weights and factor columns spread over more lanes)
        if (b - a < ctx->n_cu)
            hipLaunchKernelGGL((k_dc_merge<kMergeThreadsFew>), dim3(b - a), dim3(kMergeThreadsFew), P.dc_merge_lds,
                               ctx->stream, desc, nodes + a, Eg, LamA, LamB, FrA, FrB, LrA, LrB, Cs, Sn, idx, idx + tv, U);
        else
            hipLaunchKernelGGL((k_dc_merge<kMergeThreads>), dim3(b - a), dim3(kMergeThreads), P.dc_merge_lds,
                               ctx->stream, desc, nodes + a, Eg, LamA, LamB, FrA, FrB, LrA, LrB, Cs, Sn, idx, idx + tv, U);
        GDM_LAUNCH_CHECK(ctx);
    }
    return GDM_OK;
}

// Forward: the core rows in BUF_QC / BUF_QC2 times V_T (result in BUF_QC);
// reverse: the density rows in the halves of BUF_QC2 times V_T^T (result in
// the first half).
int gdm_dc_apply(gdm_ctx* ctx, int reverse) {
    Plan& P = ctx->plan;
    const SubDesc* desc = (const SubDesc*)ctx->b[BUF_DESC].p;
    const DcTile* tiles = (const DcTile*)((const char*)ctx->b[BUF_DCLIST].p + P.dc_tiles_off);
    const double* U = (const double*)ctx->b[BUF_DCU].p;
    double* G = (double*)ctx->b[BUF_QC].p;
    double* G2 = (double*)ctx->b[BUF_QC2].p;
    const std::vector<int>& rounds = reverse ? P.dc_rev : P.dc_fwd;
    GDM_TIMED(ctx, reverse ? "dc_apply_rev" : "dc_apply");
    for (int r = 0; r <= P.dc_max_depth; ++r) {
        const int a = rounds[r], b = rounds[r + 1];
        if (b <= a) continue;
        if (reverse)
            hipLaunchKernelGGL(k_dc_apply<true>, dim3(b - a), dim3(256), 0, ctx->stream, desc, tiles + a, U, G2,
                               (double*)nullptr);
        else
            hipLaunchKernelGGL(k_dc_apply<false>, dim3(b - a), dim3(256), 0, ctx->stream, desc, tiles + a, U, G, G2);
        GDM_LAUNCH_CHECK(ctx);
    }
    return GDM_OK;
}
