// micx_dp_u32_i3.hip -- DP kernel instances (uint32_t values) for count-row classes YR=10, YR=12, YR=16, YR=20, YR=24, YR=32, YR=40, YR=0.
#include "micx_dp_kernel.h"

#define MICX_GR false
#define MICX_V uint32_t
#include "micx_dp_shapes.h"

namespace micx {

dp_kernel_t dp_pick_u32_3(int NL, int YR, int T) {
    MICX_NL_SMALL(MICX_CASE, 10)
    MICX_NL_SMALL(MICX_CASE, 12)
    MICX_NL_SMALL(MICX_CASE1, 16)
    MICX_NL_TINY(MICX_CASE1, 20)
    MICX_NL_TINY(MICX_CASE1, 24)
    MICX_NL_TINY(MICX_CASE1, 32)
    MICX_NL_TINY(MICX_CASE1, 40)
    MICX_NL_LIST(MICX_CASE1, 0)
    MICX_CASE1(0, 0)
    return nullptr;
}

}  // namespace micx
