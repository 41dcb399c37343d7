// Entry points whose kernels are not written yet.
#include "common.h"

extern "C" {
evd_status_t evd_dorgsb_work_size(evd_ctx_t, int64_t, int64_t, size_t *) { return EVD_ERR_NOT_IMPLEMENTED; }
evd_status_t evd_dorgsb(evd_ctx_t, int64_t, int64_t, const double *, int64_t, const double *, double *, int64_t,
                        void *, size_t) { return EVD_ERR_NOT_IMPLEMENTED; }
evd_status_t evd_dbcback(evd_ctx_t, int64_t, int64_t, int64_t, const double *, const double *, double *,
                         int64_t) { return EVD_ERR_NOT_IMPLEMENTED; }
evd_status_t evd_dsyevd_work_size(evd_ctx_t, char, char, int64_t, int64_t, size_t *) { return EVD_ERR_NOT_IMPLEMENTED; }
evd_status_t evd_dsyevd(evd_ctx_t, char, char, int64_t, double *, int64_t, double *, void *, size_t, int32_t *)
{ return EVD_ERR_NOT_IMPLEMENTED; }
}
