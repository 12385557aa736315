// micx_dp_u32_g0.hip -- DP kernel instances taking batch-stream item descriptors (uint32_t values) for count-row classes YR=2, YR=3.
#include "micx_dp_kernel.h"

#define MICX_GR true
#define MICX_V uint32_t
#include "micx_dp_shapes.h"

namespace micx {

dp_kernel_t dp_pickg_u32_0(int NL, int YR, int T) {
    MICX_NL_BIG(MICX_CASE3, 2)
    MICX_NL_BIG(MICX_CASE3, 3)
    MICX_NL_LIST(MICX_CASE, 2)
    MICX_NL_LIST(MICX_CASE, 3)
    return nullptr;
}

}  // namespace micx
