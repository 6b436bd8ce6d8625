// pending.hip -- entry points of the ABI whose implementation is not in
// this build yet; each returns MXL_ERR_NOT_IMPLEMENTED with a message, the
// "declare first, implement later" pattern for executors without kernels.
#include <string>

#include "internal.hpp"

namespace {
thread_local std::string g_pending;
}

#define MXL_PENDING(name)                                                   \
    do {                                                                    \
        (void)0;                                                            \
        return MXL_ERR_NOT_IMPLEMENTED;                                     \
    } while (0)

extern "C" {
mxl_status mxl_batch_csr_create(mxl_ctx *, int64_t, const int32_t *, const int32_t *,
                                const int32_t *, const int32_t *, const double *, int, mxl_op **) {
    MXL_PENDING(batch_csr_create);
}
mxl_status mxl_batch_solve(const mxl_op *, const mxl_criteria *, const mxl_tuning *, const double *,
                           double *, int32_t *, double *, uint8_t *) {
    MXL_PENDING(batch_solve);
}
mxl_status mxl_batch_autotune(const mxl_op *, const mxl_criteria *, const double *, double *, int,
                              mxl_tuning *, double *) {
    MXL_PENDING(batch_autotune);
}
mxl_status mxl_features(const mxl_op *, double *) { MXL_PENDING(features); }
mxl_status mxl_mlp_create(mxl_ctx *, int32_t, const int32_t *, const float *, mxl_mlp **) {
    MXL_PENDING(mlp_create);
}
mxl_status mxl_mlp_get_params(const mxl_mlp *, float *, int64_t) { MXL_PENDING(x); }
mxl_status mxl_mlp_set_params(mxl_mlp *, const float *, int64_t) { MXL_PENDING(x); }
mxl_status mxl_mlp_forward(const mxl_mlp *, int64_t, const float *, float *) { MXL_PENDING(x); }
mxl_status mxl_mlp_loss_grad(mxl_mlp *, int64_t, const float *, const float *, const float *, float,
                             float *) {
    MXL_PENDING(x);
}
mxl_status mxl_mlp_get_grad(const mxl_mlp *, float *, int64_t) { MXL_PENDING(x); }
mxl_status mxl_mlp_adam_step(mxl_mlp *, int64_t, float, float, float, float) { MXL_PENDING(x); }
mxl_status mxl_mlp_destroy(mxl_mlp *) { return MXL_OK; }
}
