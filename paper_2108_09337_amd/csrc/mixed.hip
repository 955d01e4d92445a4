// Mixed-precision solvers (placeholder entry points, filled in below).
#include "internal.h"

extern "C" {

cdf_status_t cdf_dgesv_mixed(cdf_handle_t h, cdf_update_prec_t, int, int, const double *, int, const double *,
                             int, double *, int, int, int *, double *, int *) {
    return h ? CDF_ERR_UNSUPPORTED : CDF_ERR_INVALID_ARG;
}
cdf_status_t cdf_dposv_mixed(cdf_handle_t h, cdf_update_prec_t, int, int, const double *, int, const double *,
                             int, double *, int, int, int *, double *, int *) {
    return h ? CDF_ERR_UNSUPPORTED : CDF_ERR_INVALID_ARG;
}
cdf_status_t cdf_quantize(cdf_handle_t h, cdf_update_prec_t, int, int, const float *, int, int, int, void *, int,
                          int *) {
    return h ? CDF_ERR_UNSUPPORTED : CDF_ERR_INVALID_ARG;
}
cdf_status_t cdf_lowp_update(cdf_handle_t h, cdf_update_prec_t, int, int, int, const void *, int, const int *,
                             const void *, int, const int *, float *, int) {
    return h ? CDF_ERR_UNSUPPORTED : CDF_ERR_INVALID_ARG;
}
int cdf_update_tile(cdf_update_prec_t) { return 128; }

}  // extern "C"
