// Entry points whose implementation is not in this build yet: they fail
// loudly with PDMRG_EINVAL.
#include "internal.hpp"

using namespace pdmrg;

static int not_built(const char *name) {
    set_last_error(std::string(name) + ": not implemented in this build");
    return PDMRG_EINVAL;
}

extern "C" {
int mps_alloc(pdmrg_ctx *, int, const pdmrg_phys *, int32_t, const pdmrg_bond *, pdmrg_mps **) {
    return not_built("mps_alloc");
}
int mps_set_site(pdmrg_mps *, int, const double *, int64_t) { return not_built("mps_set_site"); }
int mps_bond(const pdmrg_mps *, int, int32_t *, int32_t *, int32_t *, int32_t) { return not_built("mps_bond"); }
int mps_get_site(pdmrg_mps *, int, double *, int64_t) { return not_built("mps_get_site"); }
int sweep(pdmrg_ctx *, pdmrg_mps *, const pdmrg_mpo *, const pdmrg_sweep_params *, pdmrg_sweep_report *) {
    return not_built("sweep");
}
int mps_energy(pdmrg_ctx *, pdmrg_mps *, const pdmrg_mpo *, double *) { return not_built("mps_energy"); }
void mps_free(pdmrg_mps *) {}
}
