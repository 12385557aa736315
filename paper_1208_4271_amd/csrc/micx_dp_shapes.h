// micx_dp_shapes.h -- the DP kernel shapes compiled into the library:
// NL (full layers per pass) x YR (count rows held in registers; 0 = read from
// LDS) x T (targets per lane), for the value type MICX_V of the including
// file.  Each micx_dp_{f64,u32}_i*.hip instantiates a slice; MICX_GR selects
// the instances that take per-item descriptors of a batch stream
// (micx_dp_{f64,u32}_g*.hip).
#pragma once

#define MICX_NL_LIST(X, YR) X(1, YR) X(2, YR) X(3, YR) X(4, YR) X(5, YR) X(6, YR) X(7, YR) X(8, YR) \
    X(10, YR) X(12, YR) X(14, YR) X(16, YR) X(20, YR) X(24, YR) X(28, YR) X(32, YR) X(36, YR)
#define MICX_NL_SMALL(X, YR) X(1, YR) X(2, YR) X(3, YR) X(4, YR) X(5, YR) X(6, YR) X(8, YR)
#define MICX_NL_TINY(X, YR) X(1, YR) X(2, YR) X(3, YR) X(4, YR)
#define MICX_CASE(NLv, YRv) \
    if (NL == NLv && YR == YRv) \
        return T == 1 ? k_dp<MICX_V, NLv, YRv, 1, MICX_GR> : T == 2 ? k_dp<MICX_V, NLv, YRv, 2, MICX_GR> : nullptr;
// three targets per lane: passes of >= 20 layers with few rows (32-bit form)
#define MICX_CASE3(NLv, YRv) \
    if (NL == NLv && YR == YRv && T == 3) return k_dp<MICX_V, NLv, YRv, 3, MICX_GR>;
#define MICX_NL_BIG(X, YR) X(20, YR) X(24, YR) X(28, YR) X(32, YR) X(36, YR)
#define MICX_CASE1(NLv, YRv) \
    if (NL == NLv && YR == YRv) return T == 1 ? k_dp<MICX_V, NLv, YRv, 1, MICX_GR> : nullptr;
