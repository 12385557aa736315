// micx_dp_u32_i1.hip -- DP kernel instances (uint32_t values) for count-row classes YR=4, YR=5.
#include "micx_dp_kernel.h"

#define MICX_GR false
#define MICX_V uint32_t
#include "micx_dp_shapes.h"

namespace micx {

dp_kernel_t dp_pick_u32_1(int NL, int YR, int T) {
    MICX_NL_BIG(MICX_CASE3, 4)
    MICX_NL_BIG(MICX_CASE3, 5)
    MICX_NL_LIST(MICX_CASE, 4)
    MICX_NL_LIST(MICX_CASE, 5)
    return nullptr;
}

}  // namespace micx
