// micx_dp_co.hip -- cooperative instances of the DP kernel (one item per
// workgroup, see k_dp's CO flag) for the batch stream's largest items: passes
// of 24 layers, 2-5 count rows in registers, three targets per lane in 32-bit
// fixed point and one in FP64 (two would not fit the registers beside the
// cooperative state).
#include "micx_dp_kernel.h"

namespace micx {

dp_kernel_t dp_pick_co(bool fx, int NL, int YR, int T) {
    if (NL != 24) return nullptr;
    if (fx && T == 3) {
        switch (YR) {
            case 2: return k_dp<uint32_t, 24, 2, 3, true, false, true>;
            case 3: return k_dp<uint32_t, 24, 3, 3, true, false, true>;
            case 4: return k_dp<uint32_t, 24, 4, 3, true, false, true>;
            case 5: return k_dp<uint32_t, 24, 5, 3, true, false, true>;
        }
    }
    if (!fx && T == 1) {
        switch (YR) {
            case 2: return k_dp<double, 24, 2, 1, true, false, true>;
            case 3: return k_dp<double, 24, 3, 1, true, false, true>;
            case 4: return k_dp<double, 24, 4, 1, true, false, true>;
            case 5: return k_dp<double, 24, 5, 1, true, false, true>;
        }
    }
    return nullptr;
}

}  // namespace micx
