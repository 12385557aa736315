// micx_dp.hip -- launch planning and dispatch of the OptimizeXAxis DP kernel
// (micx_dp_kernel.h) for one row count y at a time, and the fixed-point cost
// tables of the 32-bit form.
#include <math.h>

#include <mutex>

#include "micx_dp_kernel.h"

namespace micx {

dp_kernel_t dp_pick_f64_0(int NL, int YR, int T);
dp_kernel_t dp_pick_f64_1(int NL, int YR, int T);
dp_kernel_t dp_pick_f64_2(int NL, int YR, int T);
dp_kernel_t dp_pick_f64_3(int NL, int YR, int T);
dp_kernel_t dp_pick_u32_0(int NL, int YR, int T);
dp_kernel_t dp_pick_u32_1(int NL, int YR, int T);
dp_kernel_t dp_pick_u32_2(int NL, int YR, int T);
dp_kernel_t dp_pick_u32_3(int NL, int YR, int T);
dp_kernel_t dp_pickg_f64_0(int NL, int YR, int T);
dp_kernel_t dp_pickg_f64_1(int NL, int YR, int T);
dp_kernel_t dp_pickg_f64_2(int NL, int YR, int T);
dp_kernel_t dp_pickg_f64_3(int NL, int YR, int T);
dp_kernel_t dp_pickg_u32_0(int NL, int YR, int T);
dp_kernel_t dp_pickg_u32_1(int NL, int YR, int T);
dp_kernel_t dp_pickg_u32_2(int NL, int YR, int T);
dp_kernel_t dp_pickg_u32_3(int NL, int YR, int T);
dp_kernel_t dp_pick_f64_4(int NL, int YR, int T);
dp_kernel_t dp_pick_u32_4(int NL, int YR, int T);
dp_kernel_t dp_pickg_f64_4(int NL, int YR, int T);
dp_kernel_t dp_pickg_u32_4(int NL, int YR, int T);
dp_kernel_t dp_pick_co(bool fx, int NL, int YR, int T);

namespace {

// gr: the instances that take per-item descriptors (batch streams)
dp_kernel_t pick(bool fx, int NL, int YR, int T, bool gr = false) {
    typedef dp_kernel_t (*pick_t)(int, int, int);
    static const pick_t tab[2][2][5] = {
        {{dp_pick_f64_0, dp_pick_f64_1, dp_pick_f64_2, dp_pick_f64_3, dp_pick_f64_4},
         {dp_pick_u32_0, dp_pick_u32_1, dp_pick_u32_2, dp_pick_u32_3, dp_pick_u32_4}},
        {{dp_pickg_f64_0, dp_pickg_f64_1, dp_pickg_f64_2, dp_pickg_f64_3, dp_pickg_f64_4},
         {dp_pickg_u32_0, dp_pickg_u32_1, dp_pickg_u32_2, dp_pickg_u32_3, dp_pickg_u32_4}}};
    for (pick_t f : tab[gr ? 1 : 0][fx ? 1 : 0])
        if (dp_kernel_t k = f(NL, YR, T)) return k;
    return nullptr;
}

// a one-target instance of the shape exists in both forms (for the kernel
// family: descriptor instances or not)
bool have_shape(int NL, int YR, bool gr) {
    return pick(false, NL, YR, 1, gr) != nullptr && pick(true, NL, YR, 1, gr) != nullptr;
}

int round_up_in(int v, const int *set, int count, int otherwise) {
    for (int i = 0; i < count; i++)
        if (set[i] >= v) return set[i];
    return otherwise;
}

inline int align16(size_t b) { return (int)((b + 15) & ~(size_t)15); }

// T[j] = round(S * j ln j) mod 2^32 for one row-count class.
__global__ void k_fxtable(int n, double scale, const double *xlogx, uint32_t *tab) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j <= n) tab[j] = (uint32_t)(unsigned long long)__double2ll_rn(scale * xlogx[j]);
}

}  // namespace

// Shape of the DP launch for row count y (class yi).
//
// Fixed-point form (mode MICX_MODE_DP32): every candidate G_{l-1}(s) + h(s,t)
// is at most e_t ln(yhat) <= n ln y in exact arithmetic, so the scale
// S = floor(2^32 / (1.02 n ln max(y,2))) keeps the rounded sums below 2^32
// with a 2% margin.  Each column cost is off by at most (yhat+1)/2 units and
// a partition into at most l <= x columns by l(yhat+1)/2, so an entry M of
// the class is off by at most (y+1) x / (2 S n ln 2).  Classes whose bound
// exceeds the tolerance run in FP64.
namespace {

constexpr int kTuneSlots = 4096;
struct TuneEntry {
    DpTuneKey k;
    DpTune v;
    bool used;
};
TuneEntry g_tune[kTuneSlots];
int g_tune_n = 0;
std::mutex g_tune_mu;

bool same_key(const DpTuneKey &a, const DpTuneKey &b) {
    return a.fx == b.fx && a.nb == b.nb && a.y == b.y && a.x == b.x && a.khb == b.khb;
}

int ceil_log2(int v) {
    int b = 0;
    while ((1 << b) < v) b++;
    return b;
}

}  // namespace

DpTuneKey tune_key(bool fx, int n, int y, int x, int khat) {
    DpTuneKey k;
    k.fx = fx ? 1 : 0;
    k.nb = ceil_log2(n);
    k.y = y;
    k.x = x;
    k.khb = ceil_log2(khat + 1);
    return k;
}

void tune_set(const DpTuneKey &k, const DpTune &v) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (int i = 0; i < g_tune_n; i++)
        if (same_key(g_tune[i].k, k)) {
            g_tune[i].v = v;
            return;
        }
    if (g_tune_n < kTuneSlots) g_tune[g_tune_n++] = TuneEntry{k, v, true};
}

bool tune_get(const DpTuneKey &k, DpTune &v) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (int i = 0; i < g_tune_n; i++)
        if (same_key(g_tune[i].k, k)) {
            v = g_tune[i].v;
            return true;
        }
    return false;
}

void tune_clear() {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_n = 0;
}

int tune_count() {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    return g_tune_n;
}

void tune_entry(int i, DpTuneKey &k, DpTune &v) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    k = g_tune[i].k;
    v = g_tune[i].v;
}

// Each rounded cost h~(s,t) has 1 + yhat table terms, each within half a unit
// of S L[j], so a least sum over l columns is within l (yhat+1)/2 units of S
// times the exact least sum G_l.  The entry M[l][y] divides G_l / (S n) by
// ln min(l, yhat): its error is at most l (yhat+1) / (2 S n ln min(l, yhat)).
// The bound is the largest value of that over 2 <= l <= x and 2 <= yhat <= y
// (a row count with one row scores 0 whatever the DP returns).  For fixed
// yhat the largest l / ln min(l, yhat) is 2 / ln 2, m / ln m at
// m = min(x, yhat), or x / ln yhat when x > yhat; over yhat the products with
// (yhat + 1) peak at yhat = 2, at yhat = min(y, x - 1), or at yhat = y.
double dp32_bound(int n, int x, int y, double scale) {
    if (x < 2 || y < 2 || scale <= 0.0) return 0.0;
    const double c2 = 2.0 / log(2.0);
    auto lmax = [&](int yh) {   // max over 2 <= l <= x of l / ln min(l, yh)
        const int m = std::min(x, yh);
        double v = std::max(c2, (double)m / log((double)m));
        if (x > yh) v = std::max(v, (double)x / log((double)yh));
        return v;
    };
    double w = 3.0 * lmax(2);
    const int u = std::min(y, x - 1);
    if (u >= 2) w = std::max(w, (double)(u + 1) * lmax(u));
    w = std::max(w, (double)(y + 1) * lmax(y));
    return 0.5 * w / (scale * (double)n);
}

DpPlan dp_shape(const Geometry &g, int n, int yi, int mode, double tol, int nl_max, const DpTune *force,
                bool gr) {
    static const int NLS[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 36};
    static const int YRS[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 16, 20, 24, 32, 40};
    DpPlan p;
    const int y = yi + 2, x = g.B / y;
    const int kh = g.khat_host[yi];
    p.scale = floor(4294967296.0 / (1.02 * (double)n * log((double)std::max(y, 2))));
    p.bound = dp32_bound(n, x, y, p.scale);
    p.fx = mode == MICX_MODE_DP32 && p.bound <= tol && p.scale >= 1.0;
    const int vb = p.fx ? 4 : 8;                       // bytes per DP value
    const int PK = 16 / vb;
    const int nf = std::max(x - 2, 1);                 // full layers (at least one shape)
    // a tuned choice (micx_autotune) for this class, else the default rules
    DpTune tv;
    const bool tuned = force ? (tv = *force, true) : tune_get(tune_key(p.fx, n, y, x, kh), tv);
    const int nlcap = tuned && tv.nlcap > 0 ? std::min(tv.nlcap, nl_max) : nl_max;
    p.NL = round_up_in(std::min(nf, nlcap), NLS, 17, 36);
    p.YR = round_up_in(y, YRS, 14, 0);
    if (!have_shape(p.NL, p.YR, gr)) p.YR = 0;
    // more targets per lane pay off where a pass holds many layers (measured):
    // three in the 32-bit form with few rows, else two; one for smaller passes
    p.T = (p.NL >= 20 && p.YR > 0 && p.YR <= 12) ? 2 : 1;
    if (p.fx && p.NL >= 20 && p.YR > 0 && p.YR <= 5) p.T = 3;
    if (tuned && tv.T > 0) p.T = (tv.T == 1 || p.YR > 0) ? tv.T : 1;
    if (p.T == 3 && !p.fx) p.T = 2;                    // three targets per lane exist in 32 bits only
    p.wgs = tuned ? tv.wgs : 0;
    if (x == 2) {                                      // no full layer: the lean shape
        p.NL = 0;
        p.YR = 0;
        p.T = 1;
    }
    const int NLP = (p.NL + PK - 1) / PK * PK;
    p.KS = kh + 1;
    p.RS = rec_stride(p.YR, y);
    p.x = x;
    p.slot_bytes = (size_t)x * (size_t)p.KS * vb;      // layers 0..x-1 (0 unused)
    return p;
}

// Whether every row count's DP item fits the LDS of one compute unit with
// the smallest split (one wavefront, 8 staged sources), priced in FP64 (the
// 32-bit form falls back to FP64 per row count).
bool dp_fits(const Geometry &g, int n, const DpTune *force) {
    for (int yi = 0; yi < g.NY; yi++) {
        const DpPlan p = dp_shape(g, n, yi, MICX_MODE_FP64, 0.0, 36, force);
        const int NLP = (p.NL + 1) / 2 * 2;
        const size_t pairs = p.NL == 1 ? (size_t)3 * p.KS * 8 : 0;
        const size_t need = (size_t)align16((size_t)(n + 1) * 8) +
                            align16(std::max(std::max((size_t)8 * NLP * 8, (size_t)n), pairs)) +
                            align16((size_t)p.KS * p.RS * 4);
        if (need > 160 * 1024) return false;
    }
    return true;
}

DpPlan dp_plan(const Geometry &g, int n, int yi, int cus, int mode, double tol) {
    DpPlan p = dp_shape(g, n, yi, mode, tol);
    dp_fit_lds(p, n, (size_t)p.KS * p.RS * 4, cus);
    return p;
}

namespace {

// Fixed-size open-addressing memo: no heap allocation on any call path (the
// no-allocation entry point plans launches through here too).
struct OccEntry {
    const void *k;
    int device, threads, lds, occ;
};
constexpr int kOccSlots = 4096;
OccEntry g_occ[kOccSlots];
std::mutex g_occ_mu;

size_t occ_hash(const void *k, int device, int threads, int lds) {
    size_t h = (size_t)(uintptr_t)k * 0x9e3779b97f4a7c15ull;
    h ^= ((size_t)device * 0x85ebca6bu) ^ ((size_t)threads << 20) ^ (size_t)lds * 0xc2b2ae35u;
    return (h ^ (h >> 29)) & (kOccSlots - 1);
}

// Resident workgroups per CU for (kernel, workgroup size, LDS bytes) on the
// current device, asked of the runtime once and remembered.
int cached_occupancy(dp_kernel_t k, int threads, int lds) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(g_occ_mu);
    size_t h = occ_hash((const void *)k, device, threads, lds);
    for (int probe = 0; probe < kOccSlots; probe++, h = (h + 1) & (kOccSlots - 1)) {
        OccEntry &e = g_occ[h];
        if (e.k == (const void *)k && e.device == device && e.threads == threads && e.lds == lds) return e.occ;
        if (e.k == nullptr) {
            int occ = 0;
            if (ensure_lds_attr((const void *)k) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k, threads, lds) != hipSuccess)
                occ = 0;
            e = OccEntry{(const void *)k, device, threads, lds, occ};
            return occ;
        }
    }
    return 0;   // table full: no occupancy figure (the LDS cap alone applies)
}

// Kernels whose dynamic-LDS limit is set, per device (same memo scheme).
struct AttrEntry {
    const void *k;
    int device;
};
AttrEntry g_attr[kOccSlots];
std::mutex g_attr_mu;

}  // namespace

// Sets a kernel's dynamic-LDS limit to the whole 160 KB budget, once per
// kernel and device (the same value for every caller, so launches of one
// kernel from several threads agree).
hipError_t ensure_lds_attr(const void *k) {
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_attr_mu);
    size_t h = occ_hash(k, device, 0, 0);
    for (int probe = 0; probe < kOccSlots; probe++, h = (h + 1) & (kOccSlots - 1)) {
        AttrEntry &a = g_attr[h];
        if (a.k == k && a.device == device) return hipSuccess;
        if (a.k == nullptr) {
            e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e == hipSuccess) a = AttrEntry{k, device};
            return e;
        }
    }
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// LDS split of a DP launch: the L table (nmax+1 values), then per wavefront
// a staging buffer (SB sources x NLP layers, at least nmax bytes for the
// set-up flags) and the count records (rec_bytes).  SB and the wavefronts
// per workgroup shrink until two workgroups fit a CU (one at the least).
void dp_fit_lds(DpPlan &p, int nmax, size_t rec_bytes, int cus) {
    // fewer targets per lane where the shape is not built (see dp_built)
    while (p.T > 1 && !pick(p.fx, p.NL, p.YR, p.T, p.groups)) p.T--;
    const int vb = p.fx ? 4 : 8;
    const int PK = 16 / vb;
    const int NLP = (p.NL + PK - 1) / PK * PK;
    const int lds_L = align16((size_t)(nmax + 1) * vb);
    const int lds_rec = align16(rec_bytes);
    const int budget = 160 * 1024;
    p.WPB = 4;
    // workgroups per CU the staging split aims for: the tuned choice, else
    // four for one-target passes of 14 layers or more (their registers allow
    // four waves per SIMD; measured 7% faster than two), else two
    const int wgs = p.wgs > 0 ? p.wgs : ((p.T == 1 && p.NL >= 14) ? 4 : 2);
    // one-layer passes (x = 3) keep three arrays of KS values there instead
    const size_t pairs = p.NL == 1 ? (size_t)3 * p.KS * vb : 0;
    for (p.SB = 64;; p.SB >>= 1) {
        const int lds_stage = align16(std::max(std::max((size_t)p.SB * NLP * vb, (size_t)nmax), pairs));
        const int wave = align16((size_t)lds_stage + lds_rec);
        p.lds_L = lds_L;
        p.lds_stage = lds_stage;
        p.lds_wave = wave;
        p.lds = lds_L + p.WPB * wave;
        if (p.lds * wgs <= budget || p.SB == 8) break;
    }
    while (p.lds > budget && p.WPB > 1) {
        p.WPB--;
        p.lds = p.lds_L + p.WPB * p.lds_wave;
    }
    // resident workgroups per CU: the runtime's figure for this kernel (its
    // registers and LDS), capped by the LDS budget
    p.blocks_per_cu = std::max(1, budget / std::max(p.lds, 1));
    dp_kernel_t k = pick(p.fx, p.NL, p.YR, p.T, p.groups);
    const int occ = k ? cached_occupancy(k, 64 * p.WPB, p.lds) : 0;
    if (occ > 0) p.blocks_per_cu = std::min(p.blocks_per_cu, occ);
    p.max_waves = cus * p.blocks_per_cu * p.WPB;
}

bool dp_co_built(bool fx, int NL, int YR, int T) { return dp_pick_co(fx, NL, YR, T) != nullptr; }

// LDS of a cooperative launch: the table, the shared count records, the chunk
// flags and minima, the superclump flags (nmax bytes), then one staging buffer
// per wave.  Eight waves per workgroup where they fit, else four; the
// largest staging block that fits.
bool dp_fit_lds_co(DpPlan &p, int nmax, size_t rec_bytes, int cus) {
    // one completion flag per chunk of 64T targets: at most kCoChunks chunks
    if ((p.KS - 1 + 64 * p.T - 1) / (64 * p.T) > kCoChunks) return false;
    p.co = true;
    const int vb = p.fx ? 4 : 8;
    const int PK = 16 / vb;
    const int NLP = (p.NL + PK - 1) / PK * PK;
    const int budget = 160 * 1024;
    p.lds_L = align16((size_t)(nmax + 1) * vb);
    p.lds_rec = align16(rec_bytes);
    p.lds_flags = align16((size_t)nmax);
    const int fixed = p.lds_L + p.lds_rec + kCoMeta + p.lds_flags;
    // (the FP64 instances are built for four waves per workgroup)
    for (int w : {8, 4}) {
        if (w == 8 && !p.fx) continue;
        for (int sb : {32, 16, 8}) {
            const int stage = align16((size_t)sb * NLP * vb);
            if (fixed + w * stage <= budget) {
                p.WPB = w;
                p.SB = sb;
                p.lds_stage = stage;
                p.lds_wave = stage;
                p.lds = fixed + w * stage;
                dp_kernel_t k = dp_pick_co(p.fx, p.NL, p.YR, p.T);
                if (!k) return false;
                const int occ = cached_occupancy(k, 64 * p.WPB, p.lds);
                p.blocks_per_cu = std::max(1, std::min(budget / p.lds, occ > 0 ? occ : 1));
                p.max_waves = cus * p.blocks_per_cu;   // cooperative: workgroups, one item each
                return true;
            }
        }
    }
    return false;
}

hipError_t launch_fxtable(int n, const DpPlan &p, const double *xlogx, uint32_t *tab,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_fxtable, dim3((n + 256) / 256), dim3(256), 0, s, n, p.scale, xlogx, tab);
    return hipGetLastError();
}

hipError_t launch_dp(const RankTables &rt, const EquipTables &et, const Geometry &g,
                     PairSource ps, int npairs, const ItemBuffers &ib, const double *xlogx,
                     const uint32_t *fxtab, void *scratch, int yi, const DpPlan &p,
                     hipStream_t s, const int *ilist, const int *icount, int cap) {
    DpArgs a;
    a.n = rt.n; a.NY = g.NY; a.KSUM = g.KSUM; a.ASUM = g.ASUM;
    a.yi = yi; a.x = p.x; a.RS = p.RS; a.KS = p.KS;
    a.nitems = 2 * npairs; a.npairs = npairs; a.SB = p.SB; a.ps = ps;
    a.koff = g.koff; a.aoff = g.aoff;
    a.cbuf = ib.cbuf; a.sbuf = ib.sbuf; a.K = ib.K; a.src = ib.src; a.Yh = ib.Yh; a.A = ib.A;
    a.lab = ib.lab; a.lab_row = ib.lab_row; a.lab16 = ib.lab16;
    a.xlogx = xlogx; a.fxtab = fxtab; a.inv_scale = 1.0 / p.scale;
    a.scratch = scratch; a.slot_bytes = p.slot_bytes;
    a.lds_L = p.lds_L; a.lds_stage = p.lds_stage; a.lds_wave = p.lds_wave;
    a.groups = nullptr; a.gitems = nullptr; a.compat = g.compat;
    a.ilist = ilist; a.icount = icount; a.dbg = nullptr;
    if (ilist) a.nitems = std::min(a.nitems, cap);
    dp_kernel_t k = pick(p.fx, p.NL, p.YR, p.T);
    if (!k) return hipErrorInvalidValue;
    if (p.lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = ensure_lds_attr((const void *)k);
    if (e != hipSuccess) return e;
    const int waves_needed = a.nitems;
    const int waves = std::min(waves_needed, p.max_waves);
    const int blocks = (waves + p.WPB - 1) / p.WPB;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * p.WPB), p.lds, s, a);
    return hipGetLastError();
}

// The debug instances of the DP kernel (count tables only) for the two items
// of row count class yi of one pair: the label-run count scan of passes under
// 20 layers and the ballot scan of wider passes, each writing (khat+1)(y+1)
// ints per item (records of y+1 ints: e_t, then the rows' counts), to
// out[0..] and out[2*(khat+1)(y+1)..].
hipError_t launch_dp_debug(const RankTables &rt, const EquipTables &et, const Geometry &g, PairSource ps,
                           const ItemBuffers &ib, const double *xlogx, int yi, int cus, int *out,
                           hipStream_t s) {
    const dp_kernel_t ks[2] = {k_dp<double, 4, 0, 1, false, true>, k_dp<double, 24, 0, 1, false, true>};
    const int nls[2] = {4, 24};
    for (int v = 0; v < 2; v++) {
        DpPlan p = dp_shape(g, rt.n, yi, MICX_MODE_FP64, 0.0);
        p.NL = nls[v];
        p.YR = 0;
        p.T = 1;
        p.RS = rec_stride(0, yi + 2);
        dp_fit_lds(p, rt.n, (size_t)p.KS * p.RS * 4, cus);
        DpArgs a = {};
        a.n = rt.n; a.NY = g.NY; a.KSUM = g.KSUM; a.ASUM = g.ASUM;
        a.yi = yi; a.x = p.x; a.RS = p.RS; a.KS = p.KS;
        a.nitems = 2; a.npairs = 1; a.SB = p.SB; a.ps = ps;
        a.koff = g.koff; a.aoff = g.aoff;
        a.cbuf = ib.cbuf; a.sbuf = ib.sbuf; a.K = ib.K; a.src = ib.src; a.Yh = ib.Yh; a.A = ib.A;
        a.lab = ib.lab; a.lab_row = ib.lab_row; a.lab16 = ib.lab16;
        a.xlogx = xlogx; a.compat = g.compat;
        a.lds_L = p.lds_L; a.lds_stage = p.lds_stage; a.lds_wave = p.lds_wave;
        a.dbg = out + (size_t)v * 2 * p.KS * (yi + 3);
        if (p.lds > 160 * 1024) return hipErrorInvalidValue;
        hipError_t e = ensure_lds_attr((const void *)ks[v]);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(ks[v], dim3((2 + p.WPB - 1) / p.WPB), dim3(64 * p.WPB), p.lds, s, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_dp_items(const DpGroup *groups, const int *gitems, int nitems, int nmax,
                           const double *xlogx, const uint32_t *fxtab, void *scratch,
                           const DpPlan &p, int compat, hipStream_t s, const int *icount, int *status) {
    DpArgs a = {};
    a.compat = compat;
    a.n = nmax;
    a.nitems = nitems;
    a.SB = p.SB;
    a.groups = groups;
    a.gitems = gitems;
    a.xlogx = xlogx; a.fxtab = fxtab; a.inv_scale = p.fx ? 1.0 / p.scale : 0.0;
    a.scratch = scratch; a.slot_bytes = p.slot_bytes;
    a.lds_L = p.lds_L; a.lds_stage = p.lds_stage; a.lds_wave = p.lds_wave;
    a.ilist = nullptr; a.icount = icount;
    a.lds_rec = p.lds_rec; a.lds_flags = p.lds_flags; a.status = status;
    dp_kernel_t k = p.co ? dp_pick_co(p.fx, p.NL, p.YR, p.T) : pick(p.fx, p.NL, p.YR, p.T, true);
    if (!k) return hipErrorInvalidValue;
    if (p.lds > 160 * 1024) return hipErrorInvalidValue;
    if (p.co && !status) return hipErrorInvalidValue;
    hipError_t e = ensure_lds_attr((const void *)k);
    if (e != hipSuccess) return e;
    // cooperative: one item per workgroup; else one per wave
    const int waves = p.co ? std::min(nitems, p.max_waves) * p.WPB : std::min(nitems, p.max_waves);
    const int blocks = (waves + p.WPB - 1) / p.WPB;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * p.WPB), p.lds, s, a);
    return hipGetLastError();
}

}  // namespace micx
