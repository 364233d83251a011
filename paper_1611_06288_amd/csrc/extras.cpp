// Entry points whose implementation lands in later files; they report
// PFC_ERR_INVALID_ARG with a message until then.
#include "runtime_internal.h"

namespace pfc {

pfc_status mixed_init(pfc_handle *H) {
    H->err = "mixed precision is not available in this build";
    return PFC_ERR_INVALID_ARG;
}

pfc_status mixed_step(pfc_handle *H, const double *, const double *, double *, double *, double *,
                      pfc_step_info *) {
    H->err = "mixed precision is not available in this build";
    return PFC_ERR_INVALID_ARG;
}

// Algorithmic HBM bytes per launch of the finest-level kernels (FP64):
// a full red-black sweep must read u (3 fields), f (3) and phi^k (1) and
// write u (3): 80 B per point; each half-sweep launch is credited half.
double algorithmic_bytes(const pfc_handle *H, int kernel) {
    const double P = (double)H->lev[0].P;
    switch (kernel) {
        case PFC_KERNEL_SMOOTH0: return 40.0 * P;
        case PFC_KERNEL_RESIDUAL0: return 62.0 * P;
        case PFC_KERNEL_PROLONG0: return 54.0 * P;
        case PFC_KERNEL_NORM0: return 56.0 * P;
        default: return 0.0;
    }
}

}  // namespace pfc

extern "C" {

pfc_status pfc_adjoint_step(pfc_handle *h, const double *, const double *, const double *,
                            const double *, double *, double *, double *, double, int32_t *) {
    if (h) h->err = "adjoint is not available in this build";
    return PFC_ERR_INVALID_ARG;
}

pfc_status pfc_batch_create(int32_t, const pfc_config *, void *, pfc_batch **out) {
    if (out) *out = nullptr;
    return PFC_ERR_INVALID_ARG;
}
pfc_status pfc_batch_destroy(pfc_batch *) { return PFC_ERR_INVALID_ARG; }
pfc_status pfc_batch_set_state(pfc_batch *, int32_t, const double *, const double *, const double *,
                               const double *) {
    return PFC_ERR_INVALID_ARG;
}
pfc_status pfc_batch_get_state(pfc_batch *, int32_t, double *, double *, double *, double *) {
    return PFC_ERR_INVALID_ARG;
}
pfc_status pfc_batch_run(pfc_batch *, int32_t, pfc_step_info *) { return PFC_ERR_INVALID_ARG; }

}  // extern "C"
