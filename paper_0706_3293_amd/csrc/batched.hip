// Batched persistent Lanczos (placeholder until the persistent kernel lands).
#include "hm_internal.h"

using hm::fail;

extern "C" {

int hm_lanczos_batched_workspace(int32_t, const hm_basis *, int32_t, int32_t, size_t *) {
    return fail(HM_EINVAL, "batched Lanczos not available in this build");
}

int hm_lanczos_batched(int32_t, const hm_basis *, const double *const *, const double *const *,
                       int32_t, int32_t, double, void *, size_t, double *, double *, double *,
                       int32_t *, void *) {
    return fail(HM_EINVAL, "batched Lanczos not available in this build");
}

}  // extern "C"
