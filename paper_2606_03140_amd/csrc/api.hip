// Context, workspace planning and the C ABI entry points of the solve path.
#include "gdm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

int gdm_cutoff_graph(gdm_ctx* ctx, const gdm_system* sys, double cutoff, int32_t* row_ptr, int32_t* col,
                     int64_t cap, int64_t* nnz_out);
int gdm_dm_graph(gdm_ctx* ctx, const gdm_system* sys, int mode, double alpha, double tau, const gdm_subgraphs* prev,
                 const double* D_core, const int32_t* nbr_row_ptr, const int32_t* nbr_col,
                 const int32_t* union_row_ptr, const int32_t* union_col, int32_t* row_ptr, int32_t* col, int64_t cap,
                 int64_t* nnz_out);

int gdm_fail(gdm_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

int gdm_hip(gdm_ctx* ctx, hipError_t e, const char* what) {
    return gdm_fail(ctx, GDM_E_HIP, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
}

void gdm_buf_release(gdm_ctx* ctx, int slot) {
    DevBuf& b = ctx->b[slot];
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

void* gdm_buf(gdm_ctx* ctx, int slot, size_t bytes, bool* ok) {
    DevBuf& b = ctx->b[slot];
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return b.p;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    // grow with headroom so that repeated plans of similar size do not reallocate
    size_t want = bytes + bytes / 8;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        *ok = false;
        return nullptr;
    }
    b.bytes = want;
    return b.p;
}

extern "C" int gdm_create(gdm_ctx** out, int device, void* hip_stream) {
    if (!out) return GDM_E_ARG;
    *out = nullptr;
    gdm_ctx* ctx = new (std::nothrow) gdm_ctx();
    if (!ctx) return GDM_E_HIP;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&ctx->d_status, sizeof(int)) != hipSuccess) {
        delete ctx;
        return GDM_E_HIP;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        ctx->n_cu = ncu;
    if (hipMemsetAsync(ctx->d_status, 0, sizeof(int), ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        (void)hipFree(ctx->d_status);
        delete ctx;
        return GDM_E_HIP;
    }
    *out = ctx;
    return GDM_OK;
}

extern "C" int gdm_destroy(gdm_ctx* ctx) {
    if (!ctx) return GDM_E_ARG;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (auto& b : ctx->b)
        if (b.p) (void)hipFree(b.p);
    for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    delete ctx;
    return GDM_OK;
}

extern "C" int gdm_set_stream(gdm_ctx* ctx, void* hip_stream) {
    if (!ctx) return GDM_E_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return GDM_OK;
}

extern "C" const char* gdm_last_error(const gdm_ctx* ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

static int status_to_code(gdm_ctx* ctx, int st) {
    if (st == 0) return GDM_OK;
    if (st & GDM_STATUS_NOT_PD) return gdm_fail(ctx, GDM_E_NOT_PD, "a subgraph overlap matrix is not positive definite");
    if (st & GDM_STATUS_CAPACITY) return gdm_fail(ctx, GDM_E_CAPACITY, "a device-side record exceeded its capacity");
    if (st & GDM_STATUS_NOT_CONVERGED) return gdm_fail(ctx, GDM_E_NOT_CONVERGED,
                                                         "an iteration did not converge (mixed path: the inverse-"
                                                         "overlap factor needs more Newton-Schulz iterations, "
                                                         "gdm_set_mixed_options ns_z)");
    if (st & GDM_STATUS_NO_BRACKET) return gdm_fail(ctx, GDM_E_NO_BRACKET, "electron count outside the bracket");
    if (st & GDM_STATUS_NAN) return gdm_fail(ctx, GDM_E_NAN, "NaN produced");
    if (st & GDM_STATUS_PARTITION)
        return gdm_fail(ctx, GDM_E_ARG, "an atom is not a core atom of exactly one subgraph of the set");
    return gdm_fail(ctx, GDM_E_STATE, "unknown device status %d", st);
}

extern "C" int gdm_check(gdm_ctx* ctx) {
    if (!ctx) return GDM_E_ARG;
    int st = 0;
    GDM_HIP(ctx, hipMemcpyAsync(&st, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (st) GDM_HIP(ctx, hipMemsetAsync(ctx->d_status, 0, sizeof(int), ctx->stream));
    return status_to_code(ctx, st);
}

static int check_system(gdm_ctx* ctx, const gdm_system* sys, const char* who) {
    if (!sys || !sys->pos || !sys->species || !sys->orb_ptr || sys->n_atoms <= 0)
        return gdm_fail(ctx, GDM_E_ARG, "%s: system has null arrays or no atoms", who);
    for (int a = 0; a < 3; ++a)
        if (!(sys->box[a] > 0.0) || !(sys->inv_box[a] > 0.0))
            return gdm_fail(ctx, GDM_E_ARG, "%s: box edges must be positive", who);
    return GDM_OK;
}

extern "C" int gdm_build_graph(gdm_ctx* ctx, const gdm_system* sys, int mode, double cutoff, double alpha,
                               double tau, const gdm_subgraphs* prev, const double* D_core,
                               const int32_t* nbr_row_ptr, const int32_t* nbr_col, const int32_t* union_row_ptr,
                               const int32_t* union_col, int32_t* row_ptr, int32_t* col, int64_t cap,
                               int64_t* nnz_out) {
    if (!ctx) return GDM_E_ARG;
    int rc = check_system(ctx, sys, "gdm_build_graph");
    if (rc) return rc;
    if (!row_ptr || !col || !nnz_out || cap < 0) return gdm_fail(ctx, GDM_E_ARG, "gdm_build_graph: null output");
    if (mode == GDM_GRAPH_CUTOFF) {
        if (!(cutoff > 0.0)) return gdm_fail(ctx, GDM_E_ARG, "gdm_build_graph: cutoff must be positive");
        for (int a = 0; a < 3; ++a)
            if (sys->box[a] <= 2.0 * cutoff)
                return gdm_fail(ctx, GDM_E_ARG, "gdm_build_graph: box edge %g must exceed twice the cutoff",
                                sys->box[a]);
        return gdm_cutoff_graph(ctx, sys, cutoff, row_ptr, col, cap, nnz_out);
    }
    if (mode == GDM_GRAPH_DM || mode == GDM_GRAPH_ADAPTIVE) {
        if (!prev || !D_core || !(tau > 0.0))
            return gdm_fail(ctx, GDM_E_ARG, "gdm_build_graph: DM modes need prev, D_core and tau > 0");
        if (mode == GDM_GRAPH_ADAPTIVE && (!nbr_row_ptr || !nbr_col || !(alpha > 0.0)))
            return gdm_fail(ctx, GDM_E_ARG, "gdm_build_graph: adaptive mode needs the neighbour CSR and alpha > 0");
        if ((union_row_ptr == nullptr) != (union_col == nullptr))
            return gdm_fail(ctx, GDM_E_ARG, "gdm_build_graph: union graph needs both arrays");
        return gdm_dm_graph(ctx, sys, mode, alpha, tau, prev, D_core, nbr_row_ptr, nbr_col, union_row_ptr, union_col,
                            row_ptr, col, cap, nnz_out);
    }
    return gdm_fail(ctx, GDM_E_ARG, "gdm_build_graph: unknown mode %d", mode);
}

// ------------------------------------------------------------------ plan

static int round_up(int v, int m) { return (v + m - 1) / m * m; }

static int plan_impl(gdm_ctx* ctx, const gdm_subgraphs* sg, int precision) {
    if (!sg || sg->n_sub <= 0 || !sg->atom_ptr || !sg->atoms || !sg->n_core || !sg->h_norb || !sg->h_ncore_orb)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_plan: incomplete subgraph set");
    if (precision != GDM_FP64_EIG && !gdm_is_mixed(precision))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_plan: unknown precision %d", precision);
    const int ns = sg->n_sub;
    Plan& P = ctx->plan;
    P = Plan();
    P.precision = precision;
    P.n_sub = ns;
    P.n.assign(sg->h_norb, sg->h_norb + ns);
    P.nc.assign(sg->h_ncore_orb, sg->h_ncore_orb + ns);
    std::vector<int32_t> aptr(ns + 1), ncore(ns);
    GDM_HIP(ctx, hipMemcpyAsync(aptr.data(), sg->atom_ptr, sizeof(int32_t) * (ns + 1), hipMemcpyDeviceToHost,
                                ctx->stream));
    GDM_HIP(ctx, hipMemcpyAsync(ncore.data(), sg->n_core, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    P.desc.resize(ns);
    for (int s = 0; s < ns; ++s) {
        const int n = P.n[s], nc = P.nc[s];
        if (n <= 0 || nc <= 0 || nc > n)
            return gdm_fail(ctx, GDM_E_ARG, "gdm_plan: subgraph %d has n=%d nc=%d", s, n, nc);
        if (n > 8192) return gdm_fail(ctx, GDM_E_ARG, "gdm_plan: subgraph %d has %d orbitals (> 8192)", s, n);
        SubDesc& d = P.desc[s];
        d.n = n;
        d.nc = nc;
        d.ld = gdm_is_mixed(precision) ? round_up(n, 64) : round_up(n, 16);
        d.natoms = aptr[s + 1] - aptr[s];
        d.ncore_atoms = ncore[s];
        d.atom0 = aptr[s];
        d.off2 = P.tot2;
        d.offv = P.totv;
        d.offc = P.totc;
        d.offd = P.totd;
        d.offe = P.tote;
        d.offt = P.tott;
        P.tot2 += (int64_t)d.ld * d.ld;
        P.totv += d.ld;
        P.totc += (int64_t)nc * d.ld;
        P.totd += (int64_t)nc * n;
        P.tote += n;
        P.tott += 4096LL * ((n + 63) / 64);   // T factors of the reflector blocks (and, before them, L_JJ^-1)
        P.max_n = std::max(P.max_n, n);
        P.max_nc = std::max(P.max_nc, nc);
        P.max_natoms = std::max(P.max_natoms, d.natoms);
    }
    // release the other solver's exclusive workspace, so that switching
    // solvers on one context holds one solver's arena, not both
    static const int kFp64Only[] = {BUF_TAU, BUF_D, BUF_E, BUF_LAM, BUF_W, BUF_DCU, BUF_DCAUX,
                                    BUF_DCIDX, BUF_DCLIST, BUF_QC, BUF_QC2, BUF_HT, BUF_MU,
                                    BUF_MUPART, BUF_TRDP};
    static const int kMixedOnly[] = {BUF_X_F, BUF_X_HI, BUF_X_LO, BUF_GERSH, BUF_TR, BUF_NDBL, BUF_TILES,
                                     BUF_HIST_HI, BUF_HIST_LO, BUF_RESP, BUF_MSTATE};
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (precision == GDM_FP64_EIG)
        for (int s : kMixedOnly) gdm_buf_release(ctx, s);
    else
        for (int s : kFp64Only) gdm_buf_release(ctx, s);
    bool ok = true;
    void* desc = gdm_buf(ctx, BUF_DESC, sizeof(SubDesc) * ns, &ok);
    if (precision == GDM_FP64_EIG) {
        gdm_buf(ctx, BUF_A, sizeof(double) * P.tot2, &ok);
        gdm_buf(ctx, BUF_S, sizeof(double) * P.tot2, &ok);
        gdm_buf(ctx, BUF_L, sizeof(double) * P.tot2, &ok);
        for (int slot : {BUF_TAU, BUF_D, BUF_E, BUF_LAM, BUF_W}) gdm_buf(ctx, slot, sizeof(double) * P.totv, &ok);
        gdm_buf(ctx, BUF_ORDER, sizeof(int32_t) * ns, &ok);        // longest first
        gdm_buf(ctx, BUF_QC, sizeof(double) * 2 * P.totc, &ok);
        gdm_buf(ctx, BUF_HT, sizeof(double) * (size_t)std::max<int64_t>(P.tott, 1), &ok);
        gdm_buf(ctx, BUF_CC, sizeof(double) * P.totc, &ok);
        gdm_buf(ctx, BUF_MU, sizeof(double) * 8, &ok);
        gdm_buf(ctx, BUF_MUPART, sizeof(double) * 256 * (size_t)ns, &ok);
        // tile sums of the tridiagonalisation's product, per subgraph
        // 64 T (T + 1) doubles with T = ceil(ld / 64), below ld^2/64 + 3 ld + 128
        gdm_buf(ctx, BUF_TRDP, sizeof(double) * (size_t)(P.tot2 / 64 + 3 * P.totv + 128LL * ns), &ok);
        // workgroups take the subgraphs in decreasing size (ties by index)
        P.order.resize(ns);
        for (int s = 0; s < ns; ++s) P.order[s] = s;
        std::stable_sort(P.order.begin(), P.order.end(), [&](int a, int b) { return P.n[a] > P.n[b]; });
        if (ok) {
            int rc = gdm_dc_plan(ctx);
            if (rc) return rc;
            rc = gdm_fp64_plan_lds(ctx);
            if (rc) return rc;
        }
    } else {
        int rc = gdm_mixed_plan(ctx);
        if (rc) return rc;
    }
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_plan: workspace allocation failed");
    GDM_HIP(ctx, hipMemcpyAsync(desc, P.desc.data(), sizeof(SubDesc) * ns, hipMemcpyHostToDevice, ctx->stream));
    if (precision == GDM_FP64_EIG) {
        GDM_HIP(ctx, hipMemcpyAsync(ctx->b[BUF_ORDER].p, P.order.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice,
                                    ctx->stream));
    }
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    P.generation++;
    return GDM_OK;
}

extern "C" int gdm_plan(gdm_ctx* ctx, const gdm_subgraphs* sg, int precision) {
    if (!ctx) return GDM_E_ARG;
    ctx->solved = false;
    const int rc = plan_impl(ctx, sg, precision);
    if (rc) ctx->plan = Plan();      // a failed plan leaves no plan: the solve calls report GDM_E_STATE
    return rc;
}

static int check_plan(gdm_ctx* ctx, const gdm_subgraphs* sg, int precision, const char* who) {
    const Plan& P = ctx->plan;
    if (!sg || sg->n_sub != P.n_sub || P.n_sub <= 0)
        return gdm_fail(ctx, GDM_E_STATE, "%s: subgraph set does not match the plan (call gdm_plan)", who);
    if (precision != P.precision)
        return gdm_fail(ctx, GDM_E_STATE, "%s: precision %d differs from the planned %d", who, precision, P.precision);
    return GDM_OK;
}

extern "C" int gdm_find_mu(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg, const int32_t* row_ptr,
                           const int32_t* col, int64_t nnz, const double* H, const double* S, double n_electrons,
                           double kT, int precision, double mu_guess, double tol_N, double* mu_out, double* n_out) {
    if (!ctx) return GDM_E_ARG;
    int rc = check_system(ctx, sys, "gdm_find_mu");
    if (rc) return rc;
    if ((rc = check_plan(ctx, sg, precision, "gdm_find_mu"))) return rc;
    if (!row_ptr || (!col && nnz > 0) || !H || !mu_out || !n_out || !(kT > 0.0) || !(n_electrons > 0.0) ||
        !std::isfinite(n_electrons))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_find_mu: null argument or non-positive kT / electron count");
    double cap = 0.0;
    for (int s = 0; s < ctx->plan.n_sub; ++s) cap += 2.0 * ctx->plan.nc[s];
    if (n_electrons >= cap)
        return gdm_fail(ctx, GDM_E_NO_BRACKET, "gdm_find_mu: %g electrons do not fit in %g core spin-orbitals",
                        n_electrons, cap);
    ctx->solved = false;
    (void)hipGetLastError();   // a stale error of an earlier, unrelated call must not be blamed here
    if (precision == GDM_FP64_EIG)
        rc = gdm_fp64_find_mu(ctx, sys, sg, row_ptr, col, nnz, H, S, n_electrons, kT, mu_out, n_out);
    else
        rc = gdm_mixed_find_mu(ctx, sys, sg, row_ptr, col, nnz, H, S, n_electrons, kT, mu_guess, tol_N, mu_out,
                               n_out);
    if (rc) return rc;
    if (ctx->mu_out_device) {
        // enqueued only: mu and N are written on the stream, and a count or
        // NaN failure is left in the status word for gdm_check
        ctx->solved = true;
        ctx->solved_precision = precision;
        ctx->mu_solved = NAN;
        ctx->kT_solved = kT;
        return GDM_OK;
    }
    if ((rc = gdm_check(ctx))) return rc;
    if (!std::isfinite(*mu_out) || !std::isfinite(*n_out)) return gdm_fail(ctx, GDM_E_NAN, "gdm_find_mu: NaN result");
    const double tol = precision == GDM_FP64_EIG ? 1e-6 * std::max(1.0, n_electrons)
                                                 : std::max(tol_N, 1e-7 * n_electrons);
    if (std::fabs(*n_out - n_electrons) > tol)
        return gdm_fail(ctx, GDM_E_NO_BRACKET, "gdm_find_mu: electron count %.12g, wanted %.12g", *n_out,
                        n_electrons);
    ctx->solved = true;
    ctx->solved_precision = precision;
    ctx->mu_solved = *mu_out;
    ctx->kT_solved = kT;
    return GDM_OK;
}

extern "C" int gdm_set_mu_outputs(gdm_ctx* ctx, int device) {
    if (!ctx) return GDM_E_ARG;
    if (device != 0 && device != 1) return gdm_fail(ctx, GDM_E_ARG, "gdm_set_mu_outputs: device must be 0 or 1");
    ctx->mu_out_device = device;
    return GDM_OK;
}

extern "C" int gdm_subgraph_density(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, double kT, int precision,
                                    double* D_core, double* eig_out) {
    if (!ctx) return GDM_E_ARG;
    int rc;
    if ((rc = check_plan(ctx, sg, precision, "gdm_subgraph_density"))) return rc;
    if (!D_core || !(kT > 0.0) || !std::isfinite(mu))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_subgraph_density: null output or bad mu / kT");
    if (!ctx->solved || ctx->solved_precision != precision)
        return gdm_fail(ctx, GDM_E_STATE, "gdm_subgraph_density: call gdm_find_mu first");
    if (precision == GDM_FP64_EIG) return gdm_fp64_density(ctx, sg, mu, nullptr, kT, D_core, eig_out, 0);
    if (eig_out) return gdm_fail(ctx, GDM_E_ARG, "gdm_subgraph_density: eigenvalues exist only for FP64_EIG");
    // the expansion holds X at (mu_pass, kT_solved); other points are reached
    // by the first-order term only, inside its linear range
    if (std::fabs(kT - ctx->kT_solved) > 1e-12 * ctx->kT_solved)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_subgraph_density: kT %.17g differs from gdm_find_mu's %.17g (mixed path)",
                        kT, ctx->kT_solved);
    double mu_pass = 0.0;
    if ((rc = gdm_mixed_pass_mu(ctx, &mu_pass))) return rc;
    if (!(std::fabs(mu - mu_pass) <= kT))
        return gdm_fail(ctx, GDM_E_ARG,
                        "gdm_subgraph_density: mu %.12g is more than kT from the expansion's %.12g (mixed path: "
                        "first-order range)", mu, mu_pass);
    ctx->mixed_mu_pass = mu_pass;
    return gdm_mixed_density(ctx, sg, mu, nullptr, kT, D_core);
}

extern "C" int gdm_subgraph_density_dmu(gdm_ctx* ctx, const gdm_subgraphs* sg, const double* mu_device, double kT,
                                        int precision, double* D_core) {
    if (!ctx) return GDM_E_ARG;
    int rc;
    if ((rc = check_plan(ctx, sg, precision, "gdm_subgraph_density_dmu"))) return rc;
    if (!D_core || !mu_device || !(kT > 0.0))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_subgraph_density_dmu: null argument or bad kT");
    if (!ctx->solved || ctx->solved_precision != precision)
        return gdm_fail(ctx, GDM_E_STATE, "gdm_subgraph_density_dmu: call gdm_find_mu first");
    if (precision == GDM_FP64_EIG) return gdm_fp64_density(ctx, sg, 0.0, mu_device, kT, D_core, nullptr, 0);
    if (std::fabs(kT - ctx->kT_solved) > 1e-12 * ctx->kT_solved)
        return gdm_fail(ctx, GDM_E_ARG,
                        "gdm_subgraph_density_dmu: kT %.17g differs from gdm_find_mu's %.17g (mixed path)", kT,
                        ctx->kT_solved);
    return gdm_mixed_density(ctx, sg, 0.0, mu_device, kT, D_core);
}

extern "C" int gdm_subgraph_edm(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, double kT, double* W_core) {
    if (!ctx) return GDM_E_ARG;
    int rc;
    if ((rc = check_plan(ctx, sg, GDM_FP64_EIG, "gdm_subgraph_edm"))) return rc;
    if (!W_core || !(kT > 0.0) || !std::isfinite(mu))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_subgraph_edm: null output or bad mu / kT");
    if (!ctx->solved || ctx->solved_precision != GDM_FP64_EIG)
        return gdm_fail(ctx, GDM_E_STATE, "gdm_subgraph_edm: call gdm_find_mu (FP64_EIG) first");
    return gdm_fp64_density(ctx, sg, mu, nullptr, kT, W_core, nullptr, 1);
}

extern "C" int gdm_band_energy(gdm_ctx* ctx, const gdm_subgraphs* sg, double mu, double kT, double* omega_out) {
    if (!ctx) return GDM_E_ARG;
    int rc;
    if ((rc = check_plan(ctx, sg, GDM_FP64_EIG, "gdm_band_energy"))) return rc;
    if (!omega_out || !(kT > 0.0) || !std::isfinite(mu))
        return gdm_fail(ctx, GDM_E_ARG, "gdm_band_energy: null output or bad mu / kT");
    if (!ctx->solved || ctx->solved_precision != GDM_FP64_EIG)
        return gdm_fail(ctx, GDM_E_STATE, "gdm_band_energy: call gdm_find_mu (FP64_EIG) first");
    bool ok = true;
    double* dev = (double*)gdm_buf(ctx, BUF_ESUM, 64, &ok);
    if (!ok) return gdm_fail(ctx, GDM_E_HIP, "gdm_band_energy: workspace allocation failed");
    if ((rc = gdm_fp64_band_energy(ctx, mu, kT, dev))) return rc;
    GDM_HIP(ctx, hipMemcpyAsync(omega_out, dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GDM_OK;
}

extern "C" int gdm_mulliken_charges(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                                    const int32_t* row_ptr, const int32_t* col, int64_t nnz, const double* S,
                                    const double* D_core, const double n0[2], double* q_out) {
    if (!ctx) return GDM_E_ARG;
    int rc = check_system(ctx, sys, "gdm_mulliken_charges");
    if (rc) return rc;
    if (!sg || sg->n_sub != ctx->plan.n_sub || !row_ptr || (!col && nnz > 0) || !D_core || !n0 || !q_out)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_mulliken_charges: null argument or subgraph set differs from plan");
    return gdm_launch_mulliken(ctx, sys, sg, row_ptr, col, nnz, S, D_core, n0, q_out);
}

extern "C" int gdm_set_response(gdm_ctx* ctx, int max_doublings) {
    if (!ctx) return GDM_E_ARG;
    if (max_doublings < 0 || max_doublings > 40)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_set_response: max_doublings %d outside 0..40", max_doublings);
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->mixed_rec_cap = max_doublings;
    ctx->mixed_rec_nd = -1;
    return gdm_mixed_response_alloc(ctx);
}

extern "C" int gdm_density_response(gdm_ctx* ctx, const gdm_system* sys, const gdm_subgraphs* sg,
                                    const int32_t* row_ptr, const int32_t* col, int64_t nnz, const double* S,
                                    const double* dV, double* dq_out, double* dmu_out) {
    if (!ctx) return GDM_E_ARG;
    int rc = check_system(ctx, sys, "gdm_density_response");
    if (rc) return rc;
    if (!gdm_is_mixed(ctx->plan.precision))
        return gdm_fail(ctx, GDM_E_STATE, "gdm_density_response: the plan is not a mixed-precision plan");
    if ((rc = check_plan(ctx, sg, ctx->plan.precision, "gdm_density_response"))) return rc;
    if (!row_ptr || (!col && nnz > 0) || !dV || !dq_out)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_density_response: null argument");
    if (!ctx->solved || ctx->solved_precision != ctx->plan.precision)
        return gdm_fail(ctx, GDM_E_STATE, "gdm_density_response: call gdm_find_mu (mixed precision) first");
    if ((rc = gdm_mixed_response(ctx, sys, sg, row_ptr, col, nnz, S, dV, dq_out, dmu_out))) return rc;
    return gdm_check(ctx);
}

extern "C" int gdm_profile(gdm_ctx* ctx, int enable) {
    if (!ctx) return GDM_E_ARG;
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (enable) {
        if (ctx->prof_pool.empty()) {
            ctx->prof_pool.resize(2 * 65536);
            for (auto& e : ctx->prof_pool) GDM_HIP(ctx, hipEventCreate(&e));
        }
        ctx->prof.clear();
    }
    ctx->prof_on = enable != 0;
    return GDM_OK;
}

extern "C" int gdm_profile_query(gdm_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches) {
    if (!ctx) return GDM_E_ARG;
    if (!kernel || !total_ms || !launches) return gdm_fail(ctx, GDM_E_ARG, "gdm_profile_query: null argument");
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double tot = 0.0;
    int64_t n = 0;
    for (const auto& r : ctx->prof) {
        if (std::strcmp(r.name, kernel) != 0) continue;
        float ms = 0.f;
        GDM_HIP(ctx, hipEventElapsedTime(&ms, r.start, r.stop));
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return GDM_OK;
}
