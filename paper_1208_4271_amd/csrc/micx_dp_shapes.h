// micx_dp_shapes.h -- the DP kernel shapes compiled into the library:
// NL (full layers per pass) x YR (count rows held in registers; 0 = read from
// LDS) x T (targets per lane), for the value type MICX_V of the including
// file.  Each micx_dp_{f64,u32}_i*.hip instantiates a slice; MICX_GR selects
// the instances that take per-item descriptors of a batch stream
// (micx_dp_{f64,u32}_g*.hip).
#pragma once

#include <type_traits>

namespace micx {

// Shapes with more than one target per lane are built only where the planner
// picks them (passes of 20 layers or more) and where their state fits the
// VGPRs: the shapes excluded here spill into accumulation registers, which
// the build rejects (from the compiler's resource report).  The planner
// steps down to fewer targets per lane where a shape is not built.
template <class V, int NL, int YR, int T, bool GR>
constexpr bool dp_built() {
    // one target per lane: every shape, except descriptor instances whose
    // label-run count scan (passes under 20 layers) and wide count rows
    // together spill (found by the build's spill check)
    if (T == 1) {
        if (!GR || NL < 10 || NL >= 20) return true;
        if (std::is_same<V, double>::value)
            return YR <= (NL <= 10 ? 32 : NL <= 12 ? 24 : NL <= 14 ? 16 : 12);
        return !(NL == 16 && YR == 24);
    }
    if (NL < 20) return false;
    if (std::is_same<V, double>::value) return T == 2 && (GR ? NL <= 24 : !(NL >= 36 && YR >= 4));
    if (T == 2) return true;
    return GR ? (NL <= 24 || (NL <= 28 && YR <= 3)) : true;
}

template <class V, int NL, int YR, int T, bool GR>
dp_kernel_t dp_inst() {
    if constexpr (dp_built<V, NL, YR, T, GR>()) return k_dp<V, NL, YR, T, GR>;
    else return nullptr;
}

}  // namespace micx

#define MICX_NL_LIST(X, YR) X(1, YR) X(2, YR) X(3, YR) X(4, YR) X(5, YR) X(6, YR) X(7, YR) X(8, YR) \
    X(10, YR) X(12, YR) X(14, YR) X(16, YR) X(20, YR) X(24, YR) X(28, YR) X(32, YR) X(36, YR)
#define MICX_NL_SMALL(X, YR) X(1, YR) X(2, YR) X(3, YR) X(4, YR) X(5, YR) X(6, YR) X(8, YR)
#define MICX_NL_TINY(X, YR) X(1, YR) X(2, YR) X(3, YR) X(4, YR)
#define MICX_CASE(NLv, YRv) \
    if (NL == NLv && YR == YRv) \
        return T == 1 ? micx::dp_inst<MICX_V, NLv, YRv, 1, MICX_GR>() : T == 2 ? micx::dp_inst<MICX_V, NLv, YRv, 2, MICX_GR>() : nullptr;
// three targets per lane: passes of >= 20 layers with few rows (32-bit form)
#define MICX_CASE3(NLv, YRv) \
    if (NL == NLv && YR == YRv && T == 3) return micx::dp_inst<MICX_V, NLv, YRv, 3, MICX_GR>();
#define MICX_NL_BIG(X, YR) X(20, YR) X(24, YR) X(28, YR) X(32, YR) X(36, YR)
// wide row counts (YR >= 10) with more layers per pass than the lists above
// hold: large grid bounds (n = 8000 at alpha 0.7-0.75 gives x >= 24 up to
// y = 35), one target per lane
#define MICX_NL_MID(X, YR) X(10, YR) X(12, YR) X(14, YR) X(16, YR) X(20, YR) X(24, YR)
#define MICX_NL_58(X, YR) X(5, YR) X(6, YR) X(7, YR) X(8, YR)
#define MICX_CASE1(NLv, YRv) \
    if (NL == NLv && YR == YRv) return T == 1 ? micx::dp_inst<MICX_V, NLv, YRv, 1, MICX_GR>() : nullptr;
