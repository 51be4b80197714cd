// Mixed-precision recursive Fermi-operator expansion (placeholder until built).
#include "gdm_internal.h"

int gdm_mixed_plan(gdm_ctx* ctx) { return gdm_fail(ctx, GDM_E_STATE, "mixed path not available"); }
int gdm_mixed_find_mu(gdm_ctx* ctx, const gdm_system*, const gdm_subgraphs*, const int32_t*, const int32_t*, int64_t,
                      const double*, const double*, double, double, double, double, double*, double*) {
    return gdm_fail(ctx, GDM_E_STATE, "mixed path not available");
}
int gdm_mixed_density(gdm_ctx* ctx, const gdm_subgraphs*, double, double, double*) {
    return gdm_fail(ctx, GDM_E_STATE, "mixed path not available");
}
