// micx_noalloc.hip -- micx_score_noalloc: the single-pair score of
// micx_compute_score with inputs and outputs in device memory, for callers
// that cannot allocate (code under HIP graph capture, serving loops that
// forbid allocation).  Every buffer the kernels need beyond the caller's
// inputs and outputs lives in one file-scope device array, `scratch`, of
// MICX_NOALLOC_BYTES; each device holds its own copy until the process ends.
//
// The host code of the call allocates nothing: no hipMalloc/hipFree, no
// host heap (fixed-size arrays on the stack, the launch planner's fixed
// memo), no events.  Work is queued on the caller's stream and the call
// returns without waiting.  Calls that overlap on one device share its array
// and race: the caller orders them (one stream, or events).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "micx.h"
#include "micx_internal.h"

namespace micx {

namespace {

__device__ __align__(256) unsigned char scratch[MICX_NOALLOC_BYTES];

// The array's device address, per device.  In host code `scratch` names a
// host-side stand-in, not device memory: only these addresses reach kernels.
constexpr int kMaxDevices = 64;
void *g_scratch_addr[kMaxDevices];
std::mutex g_scratch_mu;

constexpr int kMaxRows = 512;    // row counts of one call held on the host stack

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Final status of a call for the caller's status word: MICX_OK, or the code
// of the device status word (bit 0: a NaN or infinity in the input).
__global__ void k_status_out(const int *status, int *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int s = *status;
        *out = s == 0 ? MICX_OK : ((s & 1) ? MICX_ENONFINITE : MICX_EDEVICE);
    }
}

}  // namespace

// Called by micx_ctx_create with `device` current: resolves the array's
// address on that device once.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return MICX_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[device]) return MICX_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MICX_EDEVICE;
    g_scratch_addr[device] = ptr;
    return MICX_OK;
}

}  // namespace micx

using namespace micx;

extern "C" int micx_score_noalloc(micx_ctx *ctx, const void *x_dev, const void *y_dev, int dtype,
                                  int n, const micx_param *param, int mode, double *stats_dev,
                                  double *mats_dev, int *status_dev, void *stream) {
    int device = 0, cus = 0, compat = 0;
    double tol = 0.0;
    if (!ctx || !x_dev || !y_dev || !stats_dev || !param) return MICX_EINVAL;
    ctx_params(ctx, &device, &cus, &compat, &tol);
    if (micx_check_param(param)) return MICX_EINVAL;
    const double alpha = param->alpha, c = param->c;
    if (mode != MICX_MODE_FP64 && mode != MICX_MODE_DP32) return MICX_EINVAL;
    if (dtype != MICX_F32 && dtype != MICX_F64 && dtype != MICX_I32) return MICX_EINVAL;
    if (n < 2) return MICX_EINVAL;
    if (n > MICX_MAX_N) return MICX_ETOOBIG;
    int B = micx_grid_bound(n, alpha);
    if (compat & MICX_COMPAT_BOUND_STRICT) B -= 1;
    if (B < 4) return MICX_ESMALLN;
    if (device < 0 || device >= kMaxDevices || !g_scratch_addr[device]) return MICX_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return MICX_EDEVICE;
    hipStream_t s = (hipStream_t)stream;

    // geometry on the host stack (the device gets its own from k_geometry)
    Geometry g;
    g.compat = compat;
    g.n = n;
    g.B = B;
    g.xmax = B / 2;
    g.NY = B / 2 - 1;
    g.W = g.NY;
    const int NY = g.NY;
    if (NY > kMaxRows) return MICX_ETOOBIG;
    int khat[kMaxRows];
    int KSUM = 0, ASUM = 0;
    for (int yi = 0; yi < NY; yi++) {
        const int x = B / (yi + 2);
        double kd = floor(c * (double)x);
        if (compat & MICX_COMPAT_KHAT_PLUS1) kd += 1.0;
        int kh = kd >= (double)n ? n : (int)kd;
        if (kh < 1) kh = 1;
        khat[yi] = kh;
        KSUM += end_slots(kh);
        ASUM += x - 1;
    }
    g.KSUM = KSUM;
    g.ASUM = ASUM;
    g.khat_host = khat;
    if (!dp_fits(g, n)) return MICX_ETOOBIG;

    // launch plans of every row count (and the FP64 plans of the recheck)
    DpPlan plans[kMaxRows];
    int nfx = 0;
    double bound = 0.0;
    size_t gbytes = 0;
    auto grid_bytes = [NY](const DpPlan &p) {
        const size_t waves = (size_t)std::min(p.max_waves, p.groups ? 2 * NY : 2);
        return (waves + p.WPB - 1) / p.WPB * p.WPB * p.slot_bytes;
    };
    for (int yi = 0; yi < NY; yi++) plans[yi] = dp_plan(g, n, yi, cus, mode, tol);
    // a 32-bit row count whose records of all rows would not fit beside the
    // FP64 table in the recheck's kernel runs in FP64 (as in micx_allpairs)
    for (int yi = 0; yi < NY; yi++) {
        if (!plans[yi].fx || B / (yi + 2) == 2) continue;
        auto a16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
        const size_t need = a16((size_t)(n + 1) * 8) + a16(std::max((size_t)8 * 8 * 8, (size_t)n)) +
                            a16((size_t)(khat[yi] + 1) * rec_stride(0, yi + 2) * 4);
        if (need > 160 * 1024) plans[yi] = dp_plan(g, n, yi, cus, MICX_MODE_FP64, 0.0);
    }
    // the row counts with x = 2 share the fixed-point scale of the largest y,
    // as in the other entry points (so that both give the same entries)
    int ylean = NY;
    while (ylean > 0 && B / (ylean + 1) == 2) ylean--;
    if (ylean < NY) {
        const double S = plans[NY - 1].scale;
        bool fx = plans[NY - 1].fx;
        for (int yi = ylean; yi < NY; yi++)
            if (dp32_bound(n, 2, yi + 2, S) > tol) fx = false;
        for (int yi = ylean; yi < NY; yi++) {
            if (fx) {
                plans[yi].scale = S;
                plans[yi].bound = dp32_bound(n, 2, yi + 2, S);
            } else if (plans[yi].fx) {
                plans[yi] = dp_plan(g, n, yi, cus, MICX_MODE_FP64, 0.0);
            }
        }
    }
    for (int yi = 0; yi < NY; yi++) {
        gbytes = std::max(gbytes, grid_bytes(plans[yi]));
        if (plans[yi].fx) {
            nfx++;
            bound = std::max(bound, plans[yi].bound);
        }
    }
    const bool recheck = nfx > 0;
    DpPlan gen;   // the FP64 recheck: a descriptor kernel that takes any row count
    if (recheck) {
        gen = dp_shape(g, n, 0, MICX_MODE_FP64, 0.0);
        gen.NL = 8;
        gen.YR = 0;
        gen.T = 1;
        gen.groups = true;
        size_t rec = 0, slot = 0;
        for (int yi = 0; yi < NY; yi++) {
            if (!plans[yi].fx) continue;   // only 32-bit classes queue items
            const size_t kh1 = (size_t)khat[yi] + 1;
            rec = std::max(rec, kh1 * (size_t)rec_stride(0, yi + 2) * 4);
            slot = std::max(slot, (size_t)(B / (yi + 2)) * kh1 * 8);
        }
        gen.slot_bytes = slot;
        dp_fit_lds(gen, n, rec, cus);
        gen.max_waves = gen.WPB;   // one workgroup: the queued items of one pair are few
        gbytes = std::max(gbytes, grid_bytes(gen));
    }

    // layout of the array
    const int esize = dtype == MICX_F64 ? 8 : 4;
    const int NYP = (NY + 7) / 8 * 8;
    const int lab16 = NY + 1 <= 256 ? 0 : 1;
    const size_t lab_row = (size_t)((n + 63) / 64 * 64) * (lab16 ? 2 : 1);
    const int nyw = (NY + 31) / 32;
    const size_t words = 1 + 2 + 2 * (size_t)nyw;   // status, recheck counters and flags
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        const size_t at = cur;
        cur += align256(bytes);
        return at;
    };
    const size_t o_words = take(words * 4);
    const size_t o_geo = take(4 * (size_t)NY * 4);
    const size_t o_X = take(2 * (size_t)n * esize);
    const size_t o_xlogx = take(((size_t)n + 1) * 8);
    const size_t o_perm = take(2 * (size_t)n * 4);
    const size_t o_gsize = take(2 * (size_t)n * 4);
    const size_t o_grank = take(2 * (size_t)n * 4);
    const size_t o_rowof = take(2 * (size_t)n * NYP * 2);
    const size_t o_yhat = take(2 * (size_t)NY * 4);
    const size_t o_cbuf = take(2 * (size_t)KSUM * 4);
    const size_t o_sbuf = take(2 * (size_t)KSUM * 4);
    const size_t o_K = take(2 * (size_t)NY * 4);
    const size_t o_k = take(2 * (size_t)NY * 4);
    const size_t o_src = take(2 * (size_t)NY * 4);
    const size_t o_Yh = take(2 * (size_t)NY * 4);
    const size_t o_A = take(2 * (size_t)ASUM * 8);
    const size_t o_lab = take(2 * (size_t)NY * lab_row);
    const size_t o_fx = take(nfx ? (size_t)NY * ((size_t)n + 1) * 4 : 0);
    const size_t o_ilist = take((size_t)NY * 2 * 3 * 4);
    const size_t o_plist = take(4);
    const size_t o_grp = take(sizeof(DpGroup));
    const size_t o_G = take(gbytes);
    if (cur > MICX_NOALLOC_BYTES) return MICX_ETOOBIG;

    unsigned char *base = (unsigned char *)g_scratch_addr[device];
    int *status = (int *)(base + o_words);
    int *geo = (int *)(base + o_geo);
    g.xcnt = geo;
    g.khat = geo + NY;
    g.koff = geo + 2 * NY;
    g.aoff = geo + 3 * NY;
    RankTables rt;
    rt.m = 2;
    rt.n = n;
    rt.perm = (int *)(base + o_perm);
    rt.gsize = (int *)(base + o_gsize);
    rt.grank = (int *)(base + o_grank);
    EquipTables et;
    et.NY = NY;
    et.NYP = NYP;
    et.rowof = (uint16_t *)(base + o_rowof);
    et.yhat = (int *)(base + o_yhat);
    et.RS = NY + 2;
    et.rowstart = nullptr;
    et.compat = compat;
    ItemBuffers ib;
    ib.cbuf = (int *)(base + o_cbuf);
    ib.sbuf = (int *)(base + o_sbuf);
    ib.K = (int *)(base + o_K);
    ib.k = (int *)(base + o_k);
    ib.src = (int *)(base + o_src);
    ib.Yh = (int *)(base + o_Yh);
    ib.A = (double *)(base + o_A);
    ib.lab = base + o_lab;
    ib.lab_row = lab_row;
    ib.lab16 = lab16;
    const double *xlogx = (const double *)(base + o_xlogx);
    uint32_t *fxtab = (uint32_t *)(base + o_fx);
    Recheck rc;
    if (recheck) {
        rc.band = 2.0 * bound + 1e-12;
        rc.icount = status + 1;
        rc.pcount = rc.icount + 1;
        rc.iflag = (unsigned *)(rc.pcount + 1);
        rc.nyw = nyw;
        rc.ilist = (int *)(base + o_ilist);
        rc.plist = (int *)(base + o_plist);
    }
    DpGroup *grp = (DpGroup *)(base + o_grp);
    PairSource ps;   // the one pair (0, 1) of the two gathered variables
    ps.pairs = nullptr;
    ps.p0 = 0;
    ps.m = 2;
    double *M = mats_dev, *Axy = mats_dev ? mats_dev + (size_t)NY * NY : nullptr;
    double *Ayx = mats_dev ? mats_dev + 2 * (size_t)NY * NY : nullptr;

#define NACHK(expr)                                    \
    do {                                               \
        if ((expr) != hipSuccess) return MICX_EDEVICE; \
    } while (0)
    NACHK(launch_zero(status, words, s));
    NACHK(launch_geometry(n, B, c, compat, NY, geo, s));
    NACHK(hipMemcpyAsync(base + o_X, x_dev, (size_t)n * esize, hipMemcpyDeviceToDevice, s));
    NACHK(hipMemcpyAsync(base + o_X + (size_t)n * esize, y_dev, (size_t)n * esize, hipMemcpyDeviceToDevice, s));
    NACHK(launch_xlogx(n, (double *)xlogx, s));
    NACHK(launch_rank(base + o_X, dtype, 2, n, rt, status, s));
    NACHK(launch_equip(rt, et, s));
    NACHK(launch_part(rt, et, g, ps, 1, ib, s));
    for (int yi = 0; yi < NY; yi++) {
        const uint32_t *tab = nullptr;
        if (plans[yi].fx) {
            uint32_t *tp = fxtab + (size_t)yi * ((size_t)n + 1);
            NACHK(launch_fxtable(n, plans[yi], xlogx, tp, s));
            tab = tp;
        }
        NACHK(launch_dp(rt, et, g, ps, 1, ib, xlogx, tab, base + o_G, yi, plans[yi], s));
    }
    NACHK(launch_stats(g, 1, ib, stats_dev, M, Axy, Ayx, s, recheck ? &rc : nullptr, nullptr, nullptr,
                       status));
    if (recheck) {
        DpGroup dg;
        dg.n = n;
        dg.NY = NY;
        dg.KSUM = KSUM;
        dg.ASUM = ASUM;
        dg.lab16 = lab16;
        dg.lab_row = lab_row;
        dg.xcnt = g.xcnt;
        dg.khat = g.khat;
        dg.koff = g.koff;
        dg.aoff = g.aoff;
        dg.Yh = ib.Yh;
        dg.cbuf = ib.cbuf;
        dg.sbuf = ib.sbuf;
        dg.K = ib.K;
        dg.src = ib.src;
        dg.lab = ib.lab;
        dg.A = ib.A;
        NACHK(launch_put_group(dg, grp, s));
        NACHK(launch_dp_items(grp, rc.ilist, 2 * NY, n, xlogx, nullptr, base + o_G, gen, compat, s, rc.icount));
        NACHK(launch_stats(g, 1, ib, stats_dev, M, Axy, Ayx, s, nullptr, rc.plist, rc.pcount, status));
    }
    if (status_dev) {
        hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, s, (const int *)status, status_dev);
        NACHK(hipGetLastError());
    }
#undef NACHK
    return MICX_OK;
}
