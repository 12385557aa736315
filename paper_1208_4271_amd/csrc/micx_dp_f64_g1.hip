// micx_dp_f64_g1.hip -- DP kernel instances taking batch-stream item descriptors (double values) for count-row classes YR=4, YR=5.
#include "micx_dp_kernel.h"

#define MICX_GR true
#define MICX_V double
#include "micx_dp_shapes.h"

namespace micx {

dp_kernel_t dp_pickg_f64_1(int NL, int YR, int T) {
    MICX_NL_LIST(MICX_CASE, 4)
    MICX_NL_LIST(MICX_CASE, 5)
    return nullptr;
}

}  // namespace micx
