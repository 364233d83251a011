// Entry points not yet implemented; they report PFC_ERR_INVALID_ARG.
#include "runtime_internal.h"



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
