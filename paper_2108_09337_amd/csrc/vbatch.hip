// Batched small factorizations (placeholder entry points).
#include "internal.h"

extern "C" {

cdf_status_t cdf_vbatch_plan_create(cdf_handle_t h, int, const int *, const int *, cdf_dtype_t,
                                    cdf_vbatch_plan_t *) {
    return h ? CDF_ERR_UNSUPPORTED : CDF_ERR_INVALID_ARG;
}
cdf_status_t cdf_vbatch_run(cdf_handle_t h, cdf_vbatch_plan_t, void *const *, const int *, int *const *, int *) {
    return h ? CDF_ERR_UNSUPPORTED : CDF_ERR_INVALID_ARG;
}
cdf_status_t cdf_vbatch_plan_destroy(cdf_vbatch_plan_t) { return CDF_ERR_UNSUPPORTED; }

}  // extern "C"
