// Spin-1/2 block kernel for H x (placeholder until the block kernel lands).
#include "device_common.h"
#include "hm_internal.h"

namespace hm {

bool half_supported(const Basis *) { return false; }

int hx_half_grid(const Basis *) { return 1; }

int launch_hx_half(const Basis *, const Couplings *, int, const HxPass &, hipStream_t) {
    return fail(HM_EINVAL, "spin-1/2 block kernel not available");
}

}  // namespace hm
