// micx_dp_co.hip -- cooperative instances of the DP kernel (one item per
// workgroup, see k_dp's CO flag) for the batch stream's largest items: passes
// of 24 layers, 2-8 count rows in registers; in 32-bit fixed point three
// targets per lane up to 5 rows and two up to 8, in FP64 one (two would not
// fit the registers beside the cooperative state).
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
    if (fx && T == 2) {
        switch (YR) {
            case 6: return k_dp<uint32_t, 24, 6, 2, true, false, true>;
            case 7: return k_dp<uint32_t, 24, 7, 2, true, false, true>;
            case 8: return k_dp<uint32_t, 24, 8, 2, true, false, true>;
        }
    }
    if (!fx && T == 1) {
        switch (YR) {
            case 2: return k_dp<double, 24, 2, 1, true, false, true>;
            case 3: return k_dp<double, 24, 3, 1, true, false, true>;
            case 4: return k_dp<double, 24, 4, 1, true, false, true>;
            case 5: return k_dp<double, 24, 5, 1, true, false, true>;
            case 6: return k_dp<double, 24, 6, 1, true, false, true>;
            case 7: return k_dp<double, 24, 7, 1, true, false, true>;
            case 8: return k_dp<double, 24, 8, 1, true, false, true>;
        }
    }
    return nullptr;
}

}  // namespace micx
