// Cost-balanced core partition, for re-partitioning when the halos have
// grown (Determining the Subgraphs: a new core partitioning restores
// efficiency, Fig. graph_partition f; Scalability section: the cost of a
// subgraph grows as its size cubed, so uneven halos unbalance the work).
//
// The paper partitions with community detection; this library's stand-ins
// are the spatial grid (gdm_grid_cores) and, here, weighted recursive
// coordinate bisection of the molecules: a set of molecules that must form
// k cores is sorted along its widest axis and cut where the running weight
// reaches k1/k of its total (k1 = k/2), and both sides recurse.  A molecule's
// weight is the number of its atoms plus their graph degrees, so cores shrink
// where the density-matrix graph is dense and their subgraphs (core plus
// one-hop halo) come out of similar size.  Host code: the partition is
// computed once per re-partitioning event, off the per-step path.
#include "gdm_internal.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace {

// x - L floor(x / L) with a separate multiply and subtract (no fused
// contraction), so the wrapped position is the same on every host
#pragma clang fp contract(off)
double wrap(double x, double L, double inv_L) {
    const double k = std::floor(x * inv_L);
    const double s = L * k;
    return x - s;
}
#pragma clang fp contract(on)

struct Rcb {
    const double* xyz;
    const double* w;
    int32_t* part;
    std::vector<int32_t> idx;

    void split(int lo, int hi, int k, int first) {
        if (k == 1) {
            for (int i = lo; i < hi; ++i) part[idx[i]] = first;
            return;
        }
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = lo; i < hi; ++i)
            for (int a = 0; a < 3; ++a) {
                mn[a] = std::min(mn[a], xyz[3 * idx[i] + a]);
                mx[a] = std::max(mx[a], xyz[3 * idx[i] + a]);
            }
        int ax = 0;
        for (int a = 1; a < 3; ++a)
            if (mx[a] - mn[a] > mx[ax] - mn[ax]) ax = a;
        std::sort(idx.begin() + lo, idx.begin() + hi, [&](int32_t p, int32_t q) {
            const double xp = xyz[3 * p + ax], xq = xyz[3 * q + ax];
            return xp < xq || (xp == xq && p < q);
        });
        const int k1 = k / 2;
        double tot = 0.0;
        for (int i = lo; i < hi; ++i) tot += w[idx[i]];
        const double target = tot * (double)k1 / (double)k;
        // cut s in [lo + k1, hi - (k - k1)] (every core keeps a molecule) with
        // the running weight closest to the target
        int s = lo + k1;
        double run = 0.0;
        for (int i = lo; i < s; ++i) run += w[idx[i]];
        double best = std::fabs(run - target);
        int bs = s;
        for (; s < hi - (k - k1); ++s) {
            run += w[idx[s]];
            const double d = std::fabs(run - target);
            if (d < best) {
                best = d;
                bs = s + 1;
            }
        }
        split(lo, bs, k1, first);
        split(bs, hi, k - k1, first + k1);
    }
};

}  // namespace

extern "C" int gdm_rcb_partition(const double* xyz, const double* weight, int32_t n, int32_t n_parts,
                                 int32_t* part) {
    if (!xyz || !part || n <= 0 || n_parts < 1 || n_parts > n) return GDM_E_ARG;
    std::vector<double> ones;
    if (!weight) {
        ones.assign(n, 1.0);
        weight = ones.data();
    }
    for (int32_t i = 0; i < n; ++i)
        if (!(weight[i] > 0.0) || !std::isfinite(weight[i]) || !std::isfinite(xyz[3 * i]) ||
            !std::isfinite(xyz[3 * i + 1]) || !std::isfinite(xyz[3 * i + 2]))
            return GDM_E_ARG;
    Rcb r{xyz, weight, part, std::vector<int32_t>(n)};
    std::iota(r.idx.begin(), r.idx.end(), 0);
    r.split(0, n, n_parts, 0);
    return GDM_OK;
}

extern "C" int gdm_balanced_cores(gdm_ctx* ctx, const gdm_system* sys, const int32_t* row_ptr, int32_t n_cores,
                                  int32_t* core_of_atom) {
    if (!ctx) return GDM_E_ARG;
    if (!sys || !sys->pos || !sys->anchor || sys->n_atoms <= 0 || !core_of_atom)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_balanced_cores: null argument or empty system");
    const int n = sys->n_atoms;
    std::vector<double> pos(3 * (size_t)n);
    std::vector<int32_t> anchor(n), rp;
    GDM_HIP(ctx, hipMemcpyAsync(pos.data(), sys->pos, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, ctx->stream));
    GDM_HIP(ctx, hipMemcpyAsync(anchor.data(), sys->anchor, sizeof(int32_t) * n, hipMemcpyDeviceToHost, ctx->stream));
    if (row_ptr) {
        rp.resize(n + 1);
        GDM_HIP(ctx, hipMemcpyAsync(rp.data(), row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, ctx->stream));
    }
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    // molecules: atoms that anchor themselves; wrapped anchor positions
    std::vector<int32_t> mol(n, -1);
    std::vector<double> xyz, w;
    for (int a = 0; a < n; ++a) {
        if (anchor[a] < 0 || anchor[a] >= n)
            return gdm_fail(ctx, GDM_E_ARG, "gdm_balanced_cores: atom %d has anchor %d", a, anchor[a]);
        if (anchor[a] == a) {
            mol[a] = (int32_t)w.size();
            for (int c = 0; c < 3; ++c) xyz.push_back(wrap(pos[3 * a + c], sys->box[c], sys->inv_box[c]));
            w.push_back(0.0);
        }
    }
    for (int a = 0; a < n; ++a) {
        const int m = mol[anchor[a]];
        if (m < 0) return gdm_fail(ctx, GDM_E_ARG, "gdm_balanced_cores: anchor of atom %d is not its own anchor", a);
        w[m] += 1.0 + (row_ptr ? (double)(rp[a + 1] - rp[a]) : 0.0);
    }
    const int nm = (int)w.size();
    if (n_cores < 1 || n_cores > nm)
        return gdm_fail(ctx, GDM_E_ARG, "gdm_balanced_cores: %d cores for %d molecules", n_cores, nm);
    std::vector<int32_t> part(nm), core(n);
    const int rc = gdm_rcb_partition(xyz.data(), w.data(), nm, n_cores, part.data());
    if (rc) return gdm_fail(ctx, rc, "gdm_balanced_cores: partition failed");
    for (int a = 0; a < n; ++a) core[a] = part[mol[anchor[a]]];
    GDM_HIP(ctx, hipMemcpyAsync(core_of_atom, core.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, ctx->stream));
    GDM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GDM_OK;
}
