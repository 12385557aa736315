// micx_dp_f64_i2.hip -- DP kernel instances (double values) for count-row classes YR=6, YR=7, YR=8.
#include "micx_dp_kernel.h"

#define MICX_GR false
#define MICX_V double
#include "micx_dp_shapes.h"

namespace micx {

dp_kernel_t dp_pick_f64_2(int NL, int YR, int T) {
    MICX_NL_LIST(MICX_CASE, 6)
    MICX_NL_LIST(MICX_CASE, 7)
    MICX_NL_LIST(MICX_CASE, 8)
    return nullptr;
}

}  // namespace micx
