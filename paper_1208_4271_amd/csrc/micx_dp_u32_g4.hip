// micx_dp_u32_g4.hip -- DP kernel instances taking batch-stream item descriptors (uint32_t values) for wide row counts
// (YR = 10..40) with 10-24 layers per pass, and YR = 20..40 with 5-8.
#include "micx_dp_kernel.h"

#define MICX_GR true
#define MICX_V uint32_t
#include "micx_dp_shapes.h"

namespace micx {

dp_kernel_t dp_pickg_u32_4(int NL, int YR, int T) {
    MICX_NL_MID(MICX_CASE1, 10)
    MICX_NL_MID(MICX_CASE1, 12)
    MICX_NL_MID(MICX_CASE1, 16)
    MICX_NL_MID(MICX_CASE1, 20)
    MICX_NL_MID(MICX_CASE1, 24)
    MICX_NL_MID(MICX_CASE1, 32)
    MICX_NL_MID(MICX_CASE1, 40)
    MICX_NL_58(MICX_CASE1, 20)
    MICX_NL_58(MICX_CASE1, 24)
    MICX_NL_58(MICX_CASE1, 32)
    MICX_NL_58(MICX_CASE1, 40)
    return nullptr;
}

}  // namespace micx
