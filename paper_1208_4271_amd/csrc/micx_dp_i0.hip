// micx_dp_i0.hip -- DP kernel instances for count-row classes YR=2, YR=3.
#include "micx_dp_kernel.h"
#include "micx_dp_shapes.h"

namespace micx {

dp_kernel_t dp_pick_0(int NL, int YR, int T) {
    MICX_NL_LIST(MICX_CASE, 2)
    MICX_NL_LIST(MICX_CASE, 3)
    return nullptr;
}

}  // namespace micx
