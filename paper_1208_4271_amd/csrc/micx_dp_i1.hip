// micx_dp_i1.hip -- DP kernel instances for count-row classes YR=4, YR=5.
#include "micx_dp_kernel.h"
#include "micx_dp_shapes.h"

namespace micx {

dp_kernel_t dp_pick_1(int NL, int YR, int T) {
    MICX_NL_LIST(MICX_CASE, 4)
    MICX_NL_LIST(MICX_CASE, 5)
    return nullptr;
}

}  // namespace micx
