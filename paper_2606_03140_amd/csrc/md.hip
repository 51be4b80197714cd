// Integrator of extended-Lagrangian Born-Oppenheimer molecular dynamics
// (Shadow MD section: the nuclear equation of motion NEQ and the harmonic
// equation HW of the extended charges n, integrated with a modified velocity
// Verlet scheme with weak dissipation):
//
//   nuclei:  v += dt/2 a(F), R += dt v, (forces at R, n), v += dt/2 a(F);
//   charges: n_{t+1} = 2 n_t - n_{t-1} + kappa K (q[n_t] - n_t)
//                      + alpha sum_{k=0..5} c_k n_{t-k},
//
// kappa = dt^2 w^2, the kernel K = c I or K = -J^-1 supplied by the caller
// (the low-rank Krylov approximation), and the dissipation coefficients of
// Niklasson et al., J. Chem. Phys. 130, 214109 (2009) for K = 5 (kappa 1.82,
// alpha 0.018, c_k = -6, 14, -8, -3, 4, -1).  Units: A, fs, eV, amu.
#include "gdm_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr double kAccel = 0.00964853321;   // A/fs^2 per eV/(A amu)
constexpr double kKeEv = 103.6426965;      // eV per amu A^2/fs^2

__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    return red[0];
}

// v += h a(F) (h = dt/2); then R += dt v when drift; per-block kinetic energy
__global__ void __launch_bounds__(kThreads) k_verlet(int n, const int32_t* __restrict__ species, double m0, double m1,
                                                    double h, double dt, const double* __restrict__ F,
                                                    double* __restrict__ vel, double* __restrict__ pos,
                                                    double* __restrict__ part) {
    __shared__ double red[kThreads];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    double ke = 0.0;
    if (i < n) {
        const double m = species[i] == 0 ? m0 : m1;
        const double c = h * kAccel / m;
        double v2 = 0.0;
        for (int x = 0; x < 3; ++x) {
            const double v = vel[3 * i + x] + c * F[3 * i + x];
            vel[3 * i + x] = v;
            if (pos) pos[3 * i + x] += dt * v;
            v2 += v * v;
        }
        ke = 0.5 * kKeEv * m * v2;
    }
    const double s = block_sum(ke, red);
    if (part && threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) k_sum(int nb, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[kThreads];
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) a += part[i];
    const double s = block_sum(a, red);
    if (threadIdx.x == 0) out[0] = s;
}

// n_{t+1} from the history hist[k * n + i] = n_{t-k} (k = 0..5) and the
// driving term kc (q - n_t), or kc delta when delta is given; the history
// shifts by one in place (each thread owns its element)
__global__ void __launch_bounds__(kThreads) k_xl_charges(int n, const double* __restrict__ q,
                                                        const double* __restrict__ delta,
                                                        double* __restrict__ hist, double kc, double alpha,
                                                        double* __restrict__ n_out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double c[6] = {-6.0, 14.0, -8.0, -3.0, 4.0, -1.0};
    double h[6];
    for (int k = 0; k < 6; ++k) h[k] = hist[(int64_t)k * n + i];
    double diss = 0.0;
    for (int k = 0; k < 6; ++k) diss += c[k] * h[k];
    const double drive = delta ? delta[i] : q[i] - h[0];
    const double nn = 2.0 * h[0] - h[1] + kc * drive + alpha * diss;
    for (int k = 5; k > 0; --k) hist[(int64_t)k * n + i] = h[k - 1];
    hist[i] = nn;
    if (n_out) n_out[i] = nn;
}

// out = a x + b y (out may alias x or y: each element is read before it is written)
__global__ void __launch_bounds__(kThreads) k_axpby(int n, double a, const double* x, double b, const double* y,
                                                   double* out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) out[i] = a * x[i] + b * y[i];
}

}  // namespace

extern "C" int gdm_md_verlet(gdm_ctx* ctx, int32_t n, const int32_t* species, const double mass[2], double dt,
                             const double* F, double* vel, double* pos, double* kinetic) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !species || !mass || !F || !vel || !(mass[0] > 0.0) || !(mass[1] > 0.0) || !std::isfinite(dt))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_md_verlet: bad argument");
    const int nb = (n + kThreads - 1) / kThreads;
    double* part = nullptr;
    if (kinetic) {
        bool ok = true;
        part = (double*)gdm_buf(ctx, BUF_MIXPART, sizeof(double) * nb, &ok);
        if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_md_verlet: workspace allocation failed");
    }
    hipLaunchKernelGGL(k_verlet, dim3(nb), dim3(kThreads), 0, ctx->stream, n, species, mass[0], mass[1], 0.5 * dt, dt,
                       F, vel, pos, part);
    GDM_LAUNCH_CHECK(ctx);
    if (kinetic) {
        hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, ctx->stream, nb, part, kinetic);
        GDM_LAUNCH_CHECK(ctx);
    }
    return GDM_OK;
}

extern "C" int gdm_xlbomd_charges(gdm_ctx* ctx, int32_t n, const double* q, const double* delta, double* hist,
                                  double kappa_c, double alpha, double* n_out) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || (!q && !delta) || !hist || !std::isfinite(kappa_c) || !std::isfinite(alpha))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_xlbomd_charges: bad argument");
    hipLaunchKernelGGL(k_xl_charges, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, ctx->stream, n, q, delta,
                       hist, kappa_c, alpha, n_out);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}

extern "C" int gdm_axpby(gdm_ctx* ctx, int32_t n, double a, const double* x, double b, const double* y,
                         double* out) {
    if (!ctx) return GDM_E_ARG;
    if (n <= 0 || !x || !y || !out) return gdm_fail(ctx, GDM_E_ARG, "gdm_axpby: bad argument");
    hipLaunchKernelGGL(k_axpby, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, ctx->stream, n, a, x, b, y,
                       out);
    GDM_LAUNCH_CHECK(ctx);
    return GDM_OK;
}
