// micx_dp.hip -- launch planning and dispatch of the OptimizeXAxis DP kernel
// (micx_dp_kernel.h) for one row count y at a time.
#include "micx_dp_kernel.h"

namespace micx {

dp_kernel_t dp_pick_0(int NL, int YR, int T);
dp_kernel_t dp_pick_1(int NL, int YR, int T);
dp_kernel_t dp_pick_2(int NL, int YR, int T);
dp_kernel_t dp_pick_3(int NL, int YR, int T);

// ------------------------------------------------------------------ dispatch

namespace {


dp_kernel_t pick(int NL, int YR, int T) {
    dp_kernel_t k = dp_pick_0(NL, YR, T);
    if (!k) k = dp_pick_1(NL, YR, T);
    if (!k) k = dp_pick_2(NL, YR, T);
    if (!k) k = dp_pick_3(NL, YR, T);
    return k;
}

bool have_shape(int NL, int YR) { return pick(NL, YR, 1) != nullptr; }

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

int round_up_in(int v, const int *set, int count, int otherwise) {
    for (int i = 0; i < count; i++)
        if (set[i] >= v) return set[i];
    return otherwise;
}

inline int align16(size_t b) { return (int)((b + 15) & ~(size_t)15); }

}  // namespace

// Shape of the DP launch for row count y (class yi).
DpPlan dp_plan(const Geometry &g, int n, int yi, int cus) {
    static const int NLS[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 36};
    static const int YRS[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 16, 20, 24, 32, 40};
    DpPlan p;
    const int y = yi + 2, x = g.B / y;
    const int kh = g.khat_host[yi];
    const int nf = std::max(x - 2, 1);                 // full layers (at least one shape)
    // tuning overrides: MICX_DP_NLCAP caps the layers per pass, MICX_DP_T
    // forces the targets per lane (1 or 2)
    const int nlcap = env_int("MICX_DP_NLCAP", 36);
    p.NL = round_up_in(std::min(nf, nlcap), NLS, 17, 36);
    p.YR = round_up_in(y, YRS, 14, 0);
    if (!have_shape(p.NL, p.YR)) p.YR = 0;
    p.T = (p.NL >= 5 && p.YR > 0 && p.YR <= 12) ? 2 : 1;
    const int tforce = env_int("MICX_DP_T", 0);
    if (tforce == 1 || (tforce == 2 && p.NL >= 5 && p.YR > 0 && p.YR <= 12)) p.T = tforce;
    const int NLP = (p.NL + 1) & ~1;
    p.KS = kh + 1;
    p.RS = (p.YR > 0 ? p.YR : y) + 1;
    p.x = x;
    p.slot = (size_t)x * (size_t)p.KS;                 // layers 0..x-1 (0 unused)
    const int lds_L = align16((size_t)(n + 1) * 8);
    const int lds_rec = align16((size_t)(kh + 1) * p.RS * 4);
    const int lds_pub = align16((size_t)NLP * 8);
    const int budget = 160 * 1024;
    p.WPB = 4;
    for (p.SB = 64; p.SB >= 8; p.SB >>= 1) {
        const int lds_stage = align16(std::max((size_t)p.SB * NLP * 8, (size_t)n));
        const int wave = align16((size_t)lds_stage + lds_pub + lds_rec);
        p.lds_L = lds_L;
        p.lds_stage = lds_stage;
        p.lds_pub = lds_pub;
        p.lds_wave = wave;
        p.lds = lds_L + p.WPB * wave;
        if (p.lds * 2 <= budget) break;     // two workgroups per CU
    }
    while (p.lds > budget && p.WPB > 1) {
        p.WPB--;
        p.lds = p.lds_L + p.WPB * p.lds_wave;
    }
    p.blocks_per_cu = std::max(1, budget / std::max(p.lds, 1));
    p.max_waves = cus * p.blocks_per_cu * p.WPB;
    return p;
}

hipError_t launch_dp(const RankTables &rt, const EquipTables &et, const Geometry &g,
                     PairSource ps, int npairs, const ItemBuffers &ib, const double *xlogx,
                     double *scratch, int yi, const DpPlan &p, int mode, hipStream_t s) {
    (void)mode;
    DpArgs a;
    a.n = rt.n; a.NY = g.NY; a.KSUM = g.KSUM; a.ASUM = g.ASUM;
    a.yi = yi; a.x = p.x; a.RS = p.RS; a.KS = p.KS;
    a.nitems = 2 * npairs; a.npairs = npairs; a.SB = p.SB; a.ps = ps;
    a.perm = rt.perm; a.grank = rt.grank; a.rowof = et.rowof; a.yhat = et.yhat;
    a.koff = g.koff; a.aoff = g.aoff;
    a.cbuf = ib.cbuf; a.sbuf = ib.sbuf; a.K = ib.K; a.src = ib.src; a.A = ib.A;
    a.xlogx = xlogx; a.scratch = scratch; a.slot = p.slot;
    a.lds_L = p.lds_L; a.lds_stage = p.lds_stage; a.lds_pub = p.lds_pub; a.lds_wave = p.lds_wave;
    dp_kernel_t k = pick(p.NL, p.YR, p.T);
    if (!k) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       p.lds);
    if (e != hipSuccess) return e;
    const int waves_needed = a.nitems;
    const int waves = std::min(waves_needed, p.max_waves);
    const int blocks = (waves + p.WPB - 1) / p.WPB;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * p.WPB), p.lds, s, a);
    return hipGetLastError();
}

}  // namespace micx
