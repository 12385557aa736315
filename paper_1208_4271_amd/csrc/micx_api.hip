// micx_api.hip -- C ABI of the engine (declared in include/micx.h).
//
// Host code here validates arguments, derives the grid geometry (B, the row
// counts y, x(y) = floor(B/y), khat(y)), sizes the workspace and launches the
// kernels of micx_kernels.hip in order.  No step of the method runs on the
// host.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <unordered_map>
#include <thread>
#include <atomic>
#include <chrono>
#include <map>
#include <tuple>
#include <vector>

#include "micx.h"
#include "micx_internal.h"

using namespace micx;

namespace {

// Grow-only device buffer.  Every reallocation bumps the context's
// generation counter: launch graphs captured before it hold stale pointers.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    unsigned *gen = nullptr;
    int ensure(size_t bytes) {
        if (bytes <= cap) return MICX_OK;
        if (gen) (*gen)++;
        if (p) hipFree(p);
        p = nullptr;
        cap = 0;
        if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
            p = nullptr;
            return MICX_ENOMEM;
        }
        cap = bytes;
        return MICX_OK;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <class T> T *as() const { return (T *)p; }
};

// Arguments of an all-pairs call, the key of its captured graph.
struct GraphKey {
    const void *X = nullptr;
    int dtype = -1, m = 0, n = 0, mode = -1, compat = 0;
    double alpha = 0.0, c = 0.0, tol = 0.0;
    double *out = nullptr;
    bool operator==(const GraphKey &o) const {
        return X == o.X && dtype == o.dtype && m == o.m && n == o.n && mode == o.mode &&
               compat == o.compat && alpha == o.alpha && c == o.c && tol == o.tol && out == o.out;
    }
};

}  // namespace

struct micx_ctx {
    int device = 0;
    int cus = 256;
    unsigned gen = 0;         // workspace generation (see DevBuf)
    DevBuf perm, gsize, grank, rowof, yhat, rowstart, xlogx, status;
    DevBuf geo;        // xcnt | khat | koff | aoff
    DevBuf cbuf, sbuf, Kb, kb, srcb, yhb, A, scratch, pairs, input, out, dense;
    DevBuf counters, fxtab, lab;
    DevBuf moments;                    // micx_pearson: per-variable mean and 1/norm
    DevBuf bdata, boffs, bout, bidx;   // micx_batch: gathered variables, offsets, staged results
    double dp32_tol = 5e-7;   // half of the 1e-6 agreement required of the scores
    int compat = 0;           // MICX_COMPAT_* flags
    int profiling = 0;
    micx_profile prof = {};
    DevBuf rcwords, rclist, rcpairs;   // near-tie recheck: counters and item flags, item lists, pairs
    DevBuf rcmeta;                     // near-tie recheck of a batch pass: key offsets, key of each class
    DevBuf arena, gitems;              // micx_batch: per-pass group buffers, DP item lists
    DevBuf dbg;                        // micx_debug_tables: the DP's count table
    DevBuf grp;                        // the batch of a pair call as one group of the descriptor kernels
    DevBuf litems;                     // descriptors of the x = 2 row counts of a batch (one launch)
    DevBuf citems;                     // descriptors of one cooperative row count of a batch
    std::vector<hipStream_t> dstreams; // micx_batch: DP launches of different shapes run side by side
    // pinned host memory: the device status word of the last call, and a
    // staging ring for host-to-device copies of asynchronous calls
    int *hstatus = nullptr;
    hipStream_t last = nullptr;        // stream of the last pair call (micx_status waits on it)
    unsigned char *stage = nullptr;
    size_t stage_cap = 0, stage_off = 0;
    std::vector<hipStream_t> stage_streams;   // streams with copies out of the ring since its reset
    // launch graph of micx_allpairs: the last key, whether it ran once, its graph
    size_t batch_budget = 0;           // bytes of per-item buffers per batch (batch_pairs)
    int graphs = 1;
    GraphKey gkey;
    bool gseen = false;
    unsigned ggen = 0;
    hipGraphExec_t gexec = nullptr;
    micx_profile gprof = {};           // the profile of the captured call (restored on replay)
    hipStream_t cstream = nullptr;     // capture stream
    std::vector<DevBuf *> bufs() {
        return {&perm, &gsize, &grank, &rowof, &yhat, &rowstart, &xlogx, &status, &geo, &cbuf, &sbuf,
                &Kb, &kb, &srcb, &yhb, &A, &scratch, &pairs, &input, &out, &dense, &counters, &fxtab, &lab,
                &moments, &bdata, &boffs, &bout, &bidx, &rcwords, &rclist, &rcpairs, &rcmeta, &arena,
                &gitems, &dbg, &grp, &litems, &citems};
    }
};

#define HIPCHK(expr)                                   \
    do {                                               \
        if ((expr) != hipSuccess) return MICX_EDEVICE; \
    } while (0)
#define RETCHK(expr)                 \
    do {                             \
        int rc_ = (expr);            \
        if (rc_ != MICX_OK) return rc_; \
    } while (0)

extern "C" const char *micx_strerror(int code) {
    switch (code) {
        case MICX_OK: return "ok";
        case MICX_EINVAL: return "invalid argument";
        case MICX_ESMALLN: return "floor(n^alpha) < 4: the grid has no cell";
        case MICX_ENONFINITE: return "input holds NaN or infinity";
        case MICX_ENOMEM: return "out of memory";
        case MICX_EDEVICE: return "HIP runtime error or device status word set";
        case MICX_ETOOBIG: return "problem too large: n above MICX_MAX_N, or a DP item above one compute unit's LDS";
        default: return "unknown error";
    }
}

namespace {
const char *param_message(double alpha, double c) {
    if (!(alpha > 0.0 && alpha <= 1.0)) return "alpha must be in (0, 1]";
    if (!(c > 0.0) || !isfinite(c)) return "c must be > 0";
    return nullptr;
}
}  // namespace

extern "C" const char *micx_check_param(const micx_param *p) {
    if (!p) return "no parameter structure";
    return param_message(p->alpha, p->c);
}

extern "C" int micx_grid_bound(int n, double alpha) {
    return (int)floor(pow((double)n, alpha));
}

extern "C" int micx_ctx_create(micx_ctx **ctx, int device) {
    if (!ctx) return MICX_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MICX_EDEVICE;
    micx_ctx *c = new (std::nothrow) micx_ctx();
    if (!c) return MICX_ENOMEM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return MICX_EDEVICE;
    }
    c->cus = device_cus(device);
    for (DevBuf *b : c->bufs()) b->gen = &c->gen;
    // the no-allocation entry point's array: its address on this device
    const int rc = noalloc_init(device);
    if (rc != MICX_OK) {
        delete c;
        return rc;
    }
    if (hipHostMalloc((void **)&c->hstatus, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return MICX_ENOMEM;
    }
    *c->hstatus = 0;
    if (hipStreamCreateWithFlags(&c->cstream, hipStreamNonBlocking) != hipSuccess) {
        hipHostFree(c->hstatus);
        delete c;
        return MICX_EDEVICE;
    }
    *ctx = c;
    return MICX_OK;
}

namespace micx {
void ctx_params(const micx_ctx *ctx, int *device, int *cus, int *compat, double *tol) {
    *device = ctx->device;
    *cus = ctx->cus;
    *compat = ctx->compat;
    *tol = ctx->dp32_tol;
}
}  // namespace micx

extern "C" void micx_ctx_destroy(micx_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (DevBuf *b : c->bufs()) b->release();
    for (hipStream_t st : c->dstreams) hipStreamDestroy(st);
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->cstream) hipStreamDestroy(c->cstream);
    if (c->stage) hipHostFree(c->stage);
    if (c->hstatus) hipHostFree(c->hstatus);
    delete c;
}

namespace {

struct HostGeometry {
    Geometry g;
    std::vector<int> xcnt, khat, koff, aoff;
};

// Grid geometry for (n, B, c): row counts y = 2..floor(B/2), x(y) = floor(B/y),
// khat(y) = max(1, min(floor(c x(y)), n)) (Algorithm 2's bound; it never
// needs to exceed n, the largest possible clump count).
void make_geometry(int n, int B, double c, HostGeometry &hg, int compat = 0) {
    Geometry &g = hg.g;
    if (compat & MICX_COMPAT_BOUND_STRICT) B -= 1;   // cells with xy < B
    g.compat = compat;
    g.n = n;
    g.B = B;
    g.xmax = B / 2;
    g.NY = B / 2 - 1;
    g.W = g.NY;
    hg.xcnt.resize(g.NY);
    hg.khat.resize(g.NY);
    hg.koff.resize(g.NY);
    hg.aoff.resize(g.NY);
    int ks = 0, as = 0, kmax = 0, kymax = 0;
    for (int yi = 0; yi < g.NY; yi++) {
        const int y = yi + 2, x = B / y;
        double kd = floor(c * (double)x);
        if (compat & MICX_COMPAT_KHAT_PLUS1) kd += 1.0;
        int kh = kd >= (double)n ? n : (int)kd;
        if (kh < 1) kh = 1;
        hg.xcnt[yi] = x;
        hg.khat[yi] = kh;
        hg.koff[yi] = ks;
        hg.aoff[yi] = as;
        ks += end_slots(kh);
        as += x - 1;
        kmax = std::max(kmax, kh);
        kymax = std::max(kymax, (kh + 1) * y);
    }
    g.KSUM = ks;
    g.ASUM = as;
    g.KMAX = kmax;
    g.KYMAX = kymax;
    g.khat_host = hg.khat.data();
}

// The geometry's device copy, computed by a kernel from (n, B, c) with the
// host's arithmetic (no host staging, so the call stays asynchronous).
int upload_geometry(micx_ctx *ctx, HostGeometry &hg, hipStream_t s, double c) {
    const int NY = hg.g.NY;
    RETCHK(ctx->geo.ensure(sizeof(int) * 4 * (size_t)NY));
    int *d = ctx->geo.as<int>();
    HIPCHK(launch_geometry(hg.g.n, hg.g.B, c, hg.g.compat, NY, d, s));
    hg.g.xcnt = d;
    hg.g.khat = d + NY;
    hg.g.koff = d + 2 * NY;
    hg.g.aoff = d + 3 * NY;
    return MICX_OK;
}

// Host-to-device copy through the context's pinned staging ring, so that the
// caller's host memory may change as soon as the call returns.  The ring is
// reused once every stream that copied out of it has finished those copies.
int stage_copy(micx_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return MICX_OK;
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (ctx->stage_off + need > ctx->stage_cap) {
        for (hipStream_t st : ctx->stage_streams) HIPCHK(hipStreamSynchronize(st));
        ctx->stage_streams.clear();
        ctx->stage_off = 0;
        if (need > ctx->stage_cap) {
            if (ctx->stage) hipHostFree(ctx->stage);
            ctx->stage = nullptr;
            ctx->stage_cap = 0;
            const size_t cap = std::max(need, (size_t)64 << 20);
            if (hipHostMalloc((void **)&ctx->stage, cap, hipHostMallocDefault) != hipSuccess) return MICX_ENOMEM;
            ctx->stage_cap = cap;
        }
    }
    unsigned char *h = ctx->stage + ctx->stage_off;
    memcpy(h, src, bytes);
    ctx->stage_off += need;
    HIPCHK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
    if (std::find(ctx->stage_streams.begin(), ctx->stage_streams.end(), s) == ctx->stage_streams.end())
        ctx->stage_streams.push_back(s);
    return MICX_OK;
}

// Clears the call's device status word (a kernel: no memset node in graphs).
int begin_status(micx_ctx *ctx, hipStream_t s) {
    RETCHK(ctx->status.ensure(sizeof(int)));
    HIPCHK(launch_zero(ctx->status.p, 1, s));
    return MICX_OK;
}

// Queues the copy of the call's status word to pinned host memory, read by
// micx_status() after the stream has finished.
int end_status(micx_ctx *ctx, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(ctx->hstatus, ctx->status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    ctx->last = s;
    return MICX_OK;
}

int status_code(int st) { return st == 0 ? MICX_OK : ((st & 1) ? MICX_ENONFINITE : MICX_EDEVICE); }

int check_common(micx_ctx *ctx, int n, double alpha, double c, int mode) {
    if (!ctx) return MICX_EINVAL;
    if (param_message(alpha, c)) return MICX_EINVAL;
    if (mode != MICX_MODE_FP64 && mode != MICX_MODE_DP32) return MICX_EINVAL;
    if (n < 2) return MICX_EINVAL;
    if (n > MICX_MAX_N) return MICX_ETOOBIG;
    if (micx_grid_bound(n, alpha) - ((ctx->compat & MICX_COMPAT_BOUND_STRICT) ? 1 : 0) < 4)
        return MICX_ESMALLN;
    return MICX_OK;
}

// Per-variable stages: ranks and equipartitions, queued on s.  The rank
// kernel sets bit 0 of the call's status word on a NaN or infinity; the
// statistics kernels then write nothing (begin_status must have run).
int prepare_variables(micx_ctx *ctx, const void *X, int dtype, int m, int n, const Geometry &g,
                      bool want_rowstart, RankTables &rt, EquipTables &et, hipStream_t s) {
    const size_t mn = (size_t)m * n;
    RETCHK(ctx->perm.ensure(mn * sizeof(int)));
    RETCHK(ctx->gsize.ensure(mn * sizeof(int)));
    RETCHK(ctx->grank.ensure(mn * sizeof(int)));
    const int NYP = (g.NY + 7) / 8 * 8;
    RETCHK(ctx->rowof.ensure(mn * NYP * sizeof(uint16_t)));
    RETCHK(ctx->yhat.ensure((size_t)m * g.NY * sizeof(int)));
    RETCHK(ctx->xlogx.ensure((size_t)(n + 1) * sizeof(double)));
    RETCHK(ctx->status.ensure(sizeof(int)));
    rt.m = m;
    rt.n = n;
    rt.perm = ctx->perm.as<int>();
    rt.gsize = ctx->gsize.as<int>();
    rt.grank = ctx->grank.as<int>();
    et.NY = g.NY;
    et.NYP = NYP;
    et.compat = g.compat;
    et.rowof = ctx->rowof.as<uint16_t>();
    et.yhat = ctx->yhat.as<int>();
    et.RS = g.NY + 2;
    et.rowstart = nullptr;
    if (want_rowstart) {
        RETCHK(ctx->rowstart.ensure((size_t)m * g.NY * et.RS * sizeof(int)));
        et.rowstart = ctx->rowstart.as<int>();
    }
    int *status = ctx->status.as<int>();
    HIPCHK(launch_xlogx(n, ctx->xlogx.as<double>(), s));
    HIPCHK(launch_rank(X, dtype, m, n, rt, status, s));
    HIPCHK(launch_equip(rt, et, s));
    return MICX_OK;
}

// Row labels take one byte when every label fits (labels < yhat <= NY + 1),
// else two; a row of labels is padded to whole 64-point blocks.
int lab_bytes(const Geometry &g) { return g.NY + 1 <= 256 ? 1 : 2; }
size_t lab_row_bytes(const Geometry &g) { return (size_t)((g.n + 63) / 64 * 64) * lab_bytes(g); }

// Pairs per batch.  The per-item buffers of a batch (clump and superclump
// ends, row labels, scores, recheck lists) take up to a third of the device
// memory free at the first call, at most 96 GB: the benchmark workload
// (m = 1000, n = 1340: about 155 KB per pair) runs as one batch on a 288 GB
// MI355X.  The budget is fixed per context, so repeated calls reuse the
// buffers (and a captured graph stays valid).
int batch_pairs(micx_ctx *ctx, const Geometry &g, int64_t total) {
    static_assert(sizeof(size_t) >= 8, "64-bit sizes");
    const size_t per_pair = 2 * (2 * (size_t)g.KSUM * sizeof(int) + 3 * (size_t)g.NY * sizeof(int) +
                                 (size_t)g.ASUM * sizeof(double) + (size_t)g.NY * lab_row_bytes(g) +
                                 2 * (size_t)g.NY * sizeof(int) + 8);
    if (ctx->batch_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = (size_t)6 << 30;
        ctx->batch_budget = std::min(fr / 3, (size_t)96 << 30);
        ctx->batch_budget = std::max(ctx->batch_budget, (size_t)256 << 20);
    }
    size_t pb = ctx->batch_budget / (per_pair ? per_pair : 1);
    if (pb < 1) pb = 1;
    if (pb > (size_t)INT32_MAX / 4) pb = (size_t)INT32_MAX / 4;
    if ((int64_t)pb > total) pb = (size_t)total;
    return (int)pb;
}

int ensure_items(micx_ctx *ctx, const Geometry &g, int pb, ItemBuffers &ib) {
    const size_t npo = 2 * (size_t)pb;
    RETCHK(ctx->cbuf.ensure(npo * g.KSUM * sizeof(int)));
    RETCHK(ctx->sbuf.ensure(npo * g.KSUM * sizeof(int)));
    RETCHK(ctx->Kb.ensure(npo * g.NY * sizeof(int)));
    RETCHK(ctx->kb.ensure(npo * g.NY * sizeof(int)));
    RETCHK(ctx->srcb.ensure(npo * g.NY * sizeof(int)));
    RETCHK(ctx->yhb.ensure(npo * g.NY * sizeof(int)));
    RETCHK(ctx->A.ensure(npo * g.ASUM * sizeof(double)));
    ib.lab16 = lab_bytes(g) == 2;
    ib.lab_row = lab_row_bytes(g);
    RETCHK(ctx->lab.ensure(npo * g.NY * ib.lab_row));
    ib.lab = ctx->lab.as<unsigned char>();
    ib.cbuf = ctx->cbuf.as<int>();
    ib.sbuf = ctx->sbuf.as<int>();
    ib.K = ctx->Kb.as<int>();
    ib.k = ctx->kb.as<int>();
    ib.src = ctx->srcb.as<int>();
    ib.Yh = ctx->yhb.as<int>();
    ib.A = ctx->A.as<double>();
    return MICX_OK;
}

// Runs clumps, DP and statistics for npairs pairs in batches.  The DP runs
// one launch per row count y, each with its own kernel shape.
int run_pairs(micx_ctx *ctx, const RankTables &rt, const EquipTables &et, const Geometry &g,
              const int32_t *pairs_dev, int64_t npairs, int m, int mode, double *out_dev,
              double *M, double *Axy, double *Ayx, hipStream_t s) {
    const int pb = batch_pairs(ctx, g, npairs);
    const int n = rt.n;
    ItemBuffers ib;
    RETCHK(ensure_items(ctx, g, pb, ib));
    std::vector<DpPlan> plans(g.NY);
    size_t scratch = 0;
    auto grid_bytes = [&](const DpPlan &p, int64_t items) {
        const size_t waves = (size_t)std::min<int64_t>(p.max_waves, items);
        if (p.co) return waves * p.slot_bytes;   // one G table per workgroup
        return ((waves + p.WPB - 1) / p.WPB) * p.WPB * p.slot_bytes;
    };
    // the row counts with x = 2 (one layer at the last target only, the lean
    // shape) form one launch over all their items: the last classes, sharing
    // the smallest fixed-point scale among them (that of the largest y)
    int ylean = g.NY;
    while (ylean > 0 && g.B / (ylean + 1) == 2) ylean--;
    for (int yi = 0; yi < g.NY; yi++) plans[yi] = dp_plan(g, n, yi, ctx->cus, mode, ctx->dp32_tol);
    // the near-tie recheck re-runs queued items of 32-bit row counts in FP64
    // with all rows' counts read from LDS (below): a row count whose records
    // of all rows would not fit one CU's LDS beside the FP64 table runs in
    // FP64 from the start (only at the largest n and alpha)
    for (int yi = 0; yi < ylean; yi++) {
        if (!plans[yi].fx) continue;
        auto a16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
        const size_t need = a16((size_t)(n + 1) * 8) + a16(std::max((size_t)8 * 8 * 8, (size_t)n)) +
                            a16((size_t)(g.khat_host[yi] + 1) * rec_stride(0, yi + 2) * 4);
        if (need > 160 * 1024) plans[yi] = dp_plan(g, n, yi, ctx->cus, MICX_MODE_FP64, 0.0);
    }
    // row counts whose items hold thousands of superclumps (large n and
    // alpha) may run cooperatively, one item per workgroup, through the
    // descriptor instances.  One wave per item leaves a CU's LDS to a few
    // waves (each holds its own count records) and runs each item's passes
    // serially; a workgroup shares the records and runs the chunks of a pass
    // side by side, but only the staged part of a chunk overlaps (its own
    // triangle waits for the chunk before it), so a workgroup finishes an item
    // about min(waves, chunks/6) times sooner (fitted to the grid-bound
    // sweep: n = 8000 at alpha 0.7, 21 chunks per pass, gains 1.5x; at
    // alpha 0.6, 9 chunks, and at n = 2000-4000, alpha 0.7, 8-13 chunks, it
    // loses 1.3-1.5x).  The cooperative form is taken where that makes the
    // batch's rounds of items shorter.
    std::vector<char> coop(g.NY, 0);
    for (int yi = 0; yi < ylean; yi++) {
        if (plans[yi].KS < kCoopMinK) continue;
        const DpTune rule;
        DpPlan pc = dp_shape(g, n, yi, plans[yi].fx ? mode : MICX_MODE_FP64, ctx->dp32_tol, 24, &rule, true);
        if (!pc.fx && !dp_co_built(false, pc.NL, pc.YR, pc.T) && dp_co_built(false, pc.NL, pc.YR, 1)) pc.T = 1;
        if (!dp_co_built(pc.fx, pc.NL, pc.YR, pc.T)) continue;
        pc.groups = true;
        if (!dp_fit_lds_co(pc, n, (size_t)pc.KS * pc.RS * 4, ctx->cus)) continue;
        const double items = 2.0 * std::min<int64_t>(pb, npairs);
        const double chunks = ceil((double)(pc.KS - 1) / (64.0 * pc.T));
        const double speed = std::min((double)pc.WPB, chunks / 6.0);
        const double t_one = ceil(items / std::max(plans[yi].max_waves, 1));
        const double t_co = ceil(items / std::max(pc.max_waves, 1)) / std::max(speed, 1e-9);
        if (!(t_co < 0.9 * t_one)) continue;
        plans[yi] = pc;
        coop[yi] = 1;
    }
    bool any_coop = false;
    for (char c : coop) any_coop |= c != 0;
    if (any_coop) RETCHK(ctx->citems.ensure((size_t)2 * pb * 3 * sizeof(int)));
    DpPlan lean;
    std::vector<double> bnd(g.NY, 0.0);
    bool lean_fx = false;
    if (ylean < g.NY) {
        lean = dp_shape(g, n, g.NY - 1, mode, ctx->dp32_tol);
        lean_fx = lean.fx;
        size_t rec = 0, slot = 0;
        for (int yi = ylean; yi < g.NY; yi++) {
            const int y = yi + 2;
            bnd[yi] = dp32_bound(n, 2, y, lean.scale);
            if (bnd[yi] > ctx->dp32_tol) lean_fx = false;
            rec = std::max(rec, (size_t)(g.khat_host[yi] + 1) * (size_t)rec_stride(0, y) * 4);
        }
        if (!lean_fx) {
            lean = dp_shape(g, n, g.NY - 1, MICX_MODE_FP64, 0.0);
            for (int yi = ylean; yi < g.NY; yi++) bnd[yi] = 0.0;
        }
        for (int yi = ylean; yi < g.NY; yi++)
            slot = std::max(slot, (size_t)2 * (size_t)(g.khat_host[yi] + 1) * (lean_fx ? 4 : 8));
        lean.slot_bytes = slot;
        lean.groups = true;
        dp_fit_lds(lean, n, rec, ctx->cus);
        scratch = std::max(scratch, grid_bytes(lean, (int64_t)(g.NY - ylean) * 2 * pb));
        RETCHK(ctx->litems.ensure((size_t)(g.NY - ylean) * 2 * pb * 3 * sizeof(int)));
    }
    int nfx = 0;
    double bound = 0.0;
    for (int yi = 0; yi < g.NY; yi++) {
        if (yi < ylean) {
            scratch = std::max(scratch, grid_bytes(plans[yi], 2 * (int64_t)pb));
            if (plans[yi].fx) bnd[yi] = plans[yi].bound;
        }
        const bool fx = yi < ylean ? plans[yi].fx : lean_fx;
        nfx += fx ? 1 : 0;
        bound = std::max(bound, bnd[yi]);
    }
    // near-tie recheck of the 32-bit form (Recheck): the queued items run in
    // FP64 in one launch of a descriptor kernel that takes any row count
    // (eight layers per pass, counts read from LDS)
    const bool recheck = nfx > 0;
    Recheck rc;
    size_t rc_words = 0;
    DpPlan gen;
    const size_t icap = (size_t)g.NY * 2 * pb;
    if (recheck) {
        gen = dp_shape(g, n, 0, MICX_MODE_FP64, 0.0);
        gen.NL = 8;
        gen.YR = 0;
        gen.T = 1;
        gen.groups = true;
        size_t rec = 0, slot = 0;
        for (int yi = 0; yi < g.NY; yi++) {
            if (!(yi < ylean ? plans[yi].fx : lean_fx)) continue;   // only 32-bit classes queue items
            const size_t kh1 = (size_t)g.khat_host[yi] + 1;
            rec = std::max(rec, kh1 * (size_t)rec_stride(0, yi + 2) * 4);
            slot = std::max(slot, (size_t)(g.B / (yi + 2)) * kh1 * 8);
        }
        gen.slot_bytes = slot;
        dp_fit_lds(gen, n, rec, ctx->cus);
        scratch = std::max(scratch, grid_bytes(gen, (int64_t)icap));
        rc.band = 2.0 * bound + 1e-12;
        rc.nyw = (g.NY + 31) / 32;
        rc_words = 2 + (size_t)2 * pb * rc.nyw;
        RETCHK(ctx->rcwords.ensure(rc_words * sizeof(unsigned)));
        RETCHK(ctx->rclist.ensure(icap * 3 * sizeof(int)));
        RETCHK(ctx->rcpairs.ensure((size_t)pb * sizeof(int)));
        rc.icount = ctx->rcwords.as<int>();
        rc.pcount = rc.icount + 1;
        rc.iflag = (unsigned *)(rc.pcount + 1);
        rc.ilist = ctx->rclist.as<int>();
        rc.plist = ctx->rcpairs.as<int>();
    }
    RETCHK(ctx->scratch.ensure(scratch));
    RETCHK(ctx->grp.ensure(sizeof(DpGroup)));
    DpGroup *grp = ctx->grp.as<DpGroup>();
    // fixed-point cost tables of the row counts that run in 32 bits, in
    // launches of up to kFxBatch classes
    const size_t tabn = (size_t)n + 1;
    if (nfx) {
        RETCHK(ctx->fxtab.ensure((size_t)g.NY * tabn * sizeof(uint32_t)));
        FxScales sc;
        int cnt = 0;
        for (int yi = 0; yi <= g.NY; yi++) {
            const bool flush = yi == g.NY || cnt == kFxBatch;
            if (flush && cnt) {
                HIPCHK(launch_fxtables(n, sc, cnt, ctx->xlogx.as<double>(), ctx->fxtab.as<uint32_t>(), tabn, s));
                cnt = 0;
            }
            if (yi == g.NY) break;
            const bool fx = yi < ylean ? plans[yi].fx : (lean_fx && yi == g.NY - 1);
            if (!fx) continue;
            sc.scale[cnt] = yi < ylean ? plans[yi].scale : lean.scale;
            sc.cls[cnt] = yi;
            cnt++;
        }
    }
    std::vector<hipEvent_t> ev, ev_rc;
    unsigned long long *counters = nullptr;
    ctx->prof = micx_profile{};
    if (ctx->profiling) {
        RETCHK(ctx->counters.ensure(4 * sizeof(unsigned long long)));
        counters = ctx->counters.as<unsigned long long>();
        HIPCHK(launch_zero(counters, 8, s));
    }
    auto mark = [&](std::vector<hipEvent_t> &v) -> int {
        if (!ctx->profiling) return MICX_OK;
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        v.push_back(e);
        HIPCHK(hipEventRecord(e, s));
        return MICX_OK;
    };
    const int *status = ctx->status.as<int>();
    for (int64_t p0 = 0; p0 < npairs; p0 += pb) {
        const int np = (int)std::min<int64_t>(pb, npairs - p0);
        PairSource ps;
        ps.m = m;
        if (pairs_dev) {
            ps.pairs = pairs_dev + 2 * p0;
            ps.p0 = 0;
        } else {
            ps.pairs = nullptr;
            ps.p0 = p0;
        }
        // the batch as one group of the descriptor kernels
        DpGroup dg;
        dg.n = n;
        dg.NY = g.NY;
        dg.KSUM = g.KSUM;
        dg.ASUM = g.ASUM;
        dg.lab16 = ib.lab16;
        dg.lab_row = ib.lab_row;
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
        HIPCHK(launch_put_group(dg, grp, s));
        if (recheck) HIPCHK(launch_zero(ctx->rcwords.p, rc_words, s));
        HIPCHK(launch_part(rt, et, g, ps, np, ib, s));
        if (counters) HIPCHK(launch_work(et, g, ps, np, ib, counters, s));
        for (int yi = 0; yi < ylean; yi++) {
            const uint32_t *tab = plans[yi].fx ? ctx->fxtab.as<uint32_t>() + yi * tabn : nullptr;
            if (coop[yi]) {
                HIPCHK(launch_range_items(yi, 1, 2 * np, ctx->citems.as<int>(), s));
                RETCHK(mark(ev));
                HIPCHK(launch_dp_items(grp, ctx->citems.as<int>(), 2 * np, n, ctx->xlogx.as<double>(), tab,
                                       ctx->scratch.p, plans[yi], g.compat, s, nullptr, ctx->status.as<int>()));
                RETCHK(mark(ev));
                continue;
            }
            RETCHK(mark(ev));
            HIPCHK(launch_dp(rt, et, g, ps, np, ib, ctx->xlogx.as<double>(), tab,
                             ctx->scratch.p, yi, plans[yi], s));
            RETCHK(mark(ev));
        }
        if (ylean < g.NY) {
            HIPCHK(launch_range_items(ylean, g.NY - ylean, 2 * np, ctx->litems.as<int>(), s));
            RETCHK(mark(ev));
            const uint32_t *tab = lean_fx ? ctx->fxtab.as<uint32_t>() + (size_t)(g.NY - 1) * tabn : nullptr;
            HIPCHK(launch_dp_items(grp, ctx->litems.as<int>(), (g.NY - ylean) * 2 * np, n,
                                   ctx->xlogx.as<double>(), tab, ctx->scratch.p, lean, g.compat, s));
            RETCHK(mark(ev));
        }
        HIPCHK(launch_stats(g, np, ib, out_dev + 4 * p0, M, Axy, Ayx, s, recheck ? &rc : nullptr, nullptr,
                            nullptr, status));
        if (recheck) {
            // FP64 re-run of the queued items, then the flagged pairs'
            // statistics again from the updated entries
            RETCHK(mark(ev_rc));
            HIPCHK(launch_dp_items(grp, rc.ilist, (int)std::min<size_t>(icap, INT32_MAX), n,
                                   ctx->xlogx.as<double>(), nullptr, ctx->scratch.p, gen, g.compat, s,
                                   rc.icount));
            HIPCHK(launch_stats(g, np, ib, out_dev + 4 * p0, M, Axy, Ayx, s, nullptr, rc.plist, rc.pcount,
                                status));
            RETCHK(mark(ev_rc));
            if (ctx->profiling) {
                int h[2];
                HIPCHK(hipMemcpyAsync(h, rc.icount, sizeof(h), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                ctx->prof.recheck_items += h[0];
                ctx->prof.recheck_pairs += h[1];
            }
        }
    }
    if (ctx->profiling) {
        HIPCHK(hipStreamSynchronize(s));
        double ms = 0.0;
        for (size_t k = 0; k + 1 < ev.size(); k += 2) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
            ms += t;
        }
        for (hipEvent_t e : ev) hipEventDestroy(e);
        double rms = 0.0;
        for (size_t k = 0; k + 1 < ev_rc.size(); k += 2) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ev_rc[k], ev_rc[k + 1]));
            rms += t;
        }
        for (hipEvent_t e : ev_rc) hipEventDestroy(e);
        ctx->prof.recheck_ms = rms;
        unsigned long long h[4];
        HIPCHK(hipMemcpy(h, counters, sizeof(h), hipMemcpyDeviceToHost));
        ctx->prof.items = (int64_t)h[0];
        ctx->prof.dp_cells = (int64_t)h[1];
        ctx->prof.h_evals = (int64_t)h[2];
        ctx->prof.h_terms = (int64_t)h[3];
        ctx->prof.dp_ms = ms;
        ctx->prof.dp_launches = (int)(ev.size() / 2);
    }
    for (int yi = 0; yi < g.NY; yi++) {
        const bool fx = yi < ylean ? plans[yi].fx : lean_fx;
        if (fx) {
            ctx->prof.dp32_classes++;
            ctx->prof.dp32_bound = std::max(ctx->prof.dp32_bound, bnd[yi]);
        } else {
            ctx->prof.fp64_classes++;
        }
        ctx->prof.coop_classes += coop[yi] ? 1 : 0;
    }
    return MICX_OK;
}

int upload_pair_input(micx_ctx *ctx, const double *x, const double *y, int n, hipStream_t s) {
    RETCHK(ctx->input.ensure(2 * (size_t)n * sizeof(double)));
    double *d = ctx->input.as<double>();
    HIPCHK(hipMemcpyAsync(d, x, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d + n, y, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    RETCHK(ctx->pairs.ensure(2 * sizeof(int32_t)));
    const int32_t pr[2] = {0, 1};
    HIPCHK(hipMemcpyAsync(ctx->pairs.p, pr, sizeof(pr), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return MICX_OK;
}

}  // namespace

namespace {

// The work of one all-pairs call, queued on s.
int allpairs_work(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n, double alpha, double c,
                  int mode, double *out_dev, hipStream_t s) {
    HostGeometry hg;
    make_geometry(n, micx_grid_bound(n, alpha), c, hg, ctx->compat);
    RETCHK(begin_status(ctx, s));
    RETCHK(upload_geometry(ctx, hg, s, c));
    RankTables rt;
    EquipTables et;
    RETCHK(prepare_variables(ctx, X_dev, dtype, m, n, hg.g, false, rt, et, s));
    const int64_t npairs = (int64_t)m * (m - 1) / 2;
    RETCHK(run_pairs(ctx, rt, et, hg.g, nullptr, npairs, m, mode, out_dev, nullptr, nullptr, nullptr, s));
    return end_status(ctx, s);
}

void drop_graph(micx_ctx *ctx) {
    if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
}

}  // namespace

extern "C" int micx_allpairs(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n,
                             const micx_param *param, int mode, double *out_dev, void *stream) {
    if (!param) return MICX_EINVAL;
    const double alpha = param->alpha, c = param->c;
    RETCHK(check_common(ctx, n, alpha, c, mode));
    if (!X_dev || !out_dev || m < 2) return MICX_EINVAL;
    if (dtype != MICX_F32 && dtype != MICX_F64 && dtype != MICX_I32) return MICX_EINVAL;
    {
        HostGeometry hg;
        make_geometry(n, micx_grid_bound(n, alpha), c, hg, ctx->compat);
        if (!dp_fits(hg.g, n)) return MICX_ETOOBIG;
    }
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    GraphKey key;
    key.X = X_dev;
    key.dtype = dtype;
    key.m = m;
    key.n = n;
    key.mode = mode;
    key.compat = ctx->compat;
    key.alpha = alpha;
    key.c = c;
    key.tol = ctx->dp32_tol;
    key.out = out_dev;
    if (!ctx->graphs || ctx->profiling) {
        drop_graph(ctx);
        ctx->gseen = false;
        return allpairs_work(ctx, X_dev, dtype, m, n, alpha, c, mode, out_dev, s);
    }
    const bool same = ctx->gseen && key == ctx->gkey && ctx->ggen == ctx->gen;
    if (same && ctx->gexec) {
        // replay: the whole call is one graph launch (its profile is the
        // captured call's: the same launches over the same arguments)
        HIPCHK(hipGraphLaunch(ctx->gexec, s));
        ctx->last = s;
        ctx->prof = ctx->gprof;
        return MICX_OK;
    }
    drop_graph(ctx);
    if (!same) {
        // first call with these arguments: run it eagerly (it sizes the
        // workspace); the next one captures
        RETCHK(allpairs_work(ctx, X_dev, dtype, m, n, alpha, c, mode, out_dev, s));
        ctx->gkey = key;
        ctx->gseen = true;
        ctx->ggen = ctx->gen;
        return MICX_OK;
    }
    // second call: capture the work on the context's capture stream, after
    // the caller's stream has reached this point, then launch the graph on
    // the caller's stream
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(ctx->cstream, hipStreamCaptureModeRelaxed));
    const int rc = allpairs_work(ctx, X_dev, dtype, m, n, alpha, c, mode, out_dev, ctx->cstream);
    const hipError_t ec = hipStreamEndCapture(ctx->cstream, &graph);
    if (rc != MICX_OK || ec != hipSuccess || ctx->gen != ctx->ggen) {
        // the workspace moved during capture, or capture failed: run eagerly
        if (graph) hipGraphDestroy(graph);
        ctx->gseen = false;
        RETCHK(rc);
        return allpairs_work(ctx, X_dev, dtype, m, n, alpha, c, mode, out_dev, s);
    }
    const hipError_t ei = hipGraphInstantiate(&ctx->gexec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        ctx->gexec = nullptr;
        ctx->gseen = false;
        return allpairs_work(ctx, X_dev, dtype, m, n, alpha, c, mode, out_dev, s);
    }
    HIPCHK(hipGraphLaunch(ctx->gexec, s));
    ctx->last = s;
    ctx->gprof = ctx->prof;
    return MICX_OK;
}

extern "C" int micx_status(micx_ctx *ctx) {
    if (!ctx) return MICX_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->last));
    return status_code(*ctx->hstatus);
}

extern "C" int micx_set_graphs(micx_ctx *ctx, int enable) {
    if (!ctx) return MICX_EINVAL;
    ctx->graphs = enable ? 1 : 0;
    if (!enable) {
        drop_graph(ctx);
        ctx->gseen = false;
    }
    return MICX_OK;
}

extern "C" int micx_pearson(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n,
                            const int32_t *pairs_host, int64_t npairs, const double *stats_dev,
                            double *out_dev, void *stream) {
    if (!ctx || !X_dev || !out_dev || m < 2 || n < 2 || npairs < 1) return MICX_EINVAL;
    if (dtype != MICX_F32 && dtype != MICX_F64 && dtype != MICX_I32) return MICX_EINVAL;
    if (npairs > INT32_MAX) return MICX_EINVAL;
    if (!pairs_host && npairs != (int64_t)m * (m - 1) / 2) return MICX_EINVAL;
    if (pairs_host) {
        for (int64_t k = 0; k < 2 * npairs; k++)
            if (pairs_host[k] < 0 || pairs_host[k] >= m) return MICX_EINVAL;
    }
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    PairSource ps;
    ps.pairs = nullptr;
    ps.p0 = 0;
    ps.m = m;
    if (pairs_host) {
        RETCHK(ctx->pairs.ensure((size_t)npairs * 2 * sizeof(int32_t)));
        RETCHK(stage_copy(ctx, ctx->pairs.p, pairs_host, (size_t)npairs * 2 * sizeof(int32_t), s));
        ps.pairs = ctx->pairs.as<int32_t>();
    }
    RETCHK(ctx->moments.ensure((size_t)2 * m * sizeof(double)));
    double *mean = ctx->moments.as<double>();
    RETCHK(begin_status(ctx, s));
    HIPCHK(launch_pearson(X_dev, dtype, m, n, ps, (int)npairs, mean, mean + m, stats_dev, out_dev, s));
    return end_status(ctx, s);
}

extern "C" int micx_pairs(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n,
                          const int32_t *pairs_host, int64_t npairs, const micx_param *param, int mode,
                          double *out_dev, void *stream) {
    if (!param) return MICX_EINVAL;
    const double alpha = param->alpha, c = param->c;
    RETCHK(check_common(ctx, n, alpha, c, mode));
    if (!X_dev || !out_dev || !pairs_host || m < 2 || npairs < 1) return MICX_EINVAL;
    if (dtype != MICX_F32 && dtype != MICX_F64 && dtype != MICX_I32) return MICX_EINVAL;
    for (int64_t k = 0; k < 2 * npairs; k++)
        if (pairs_host[k] < 0 || pairs_host[k] >= m) return MICX_EINVAL;
    for (int64_t k = 0; k < npairs; k++)
        if (pairs_host[2 * k] == pairs_host[2 * k + 1]) return MICX_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HostGeometry hg;
    make_geometry(n, micx_grid_bound(n, alpha), c, hg, ctx->compat);
    if (!dp_fits(hg.g, n)) return MICX_ETOOBIG;
    RETCHK(begin_status(ctx, s));
    RETCHK(upload_geometry(ctx, hg, s, c));
    RETCHK(ctx->pairs.ensure((size_t)npairs * 2 * sizeof(int32_t)));
    RETCHK(stage_copy(ctx, ctx->pairs.p, pairs_host, (size_t)npairs * 2 * sizeof(int32_t), s));
    RankTables rt;
    EquipTables et;
    RETCHK(prepare_variables(ctx, X_dev, dtype, m, n, hg.g, false, rt, et, s));
    RETCHK(run_pairs(ctx, rt, et, hg.g, ctx->pairs.as<int32_t>(), npairs, m, mode, out_dev,
                     nullptr, nullptr, nullptr, s));
    return end_status(ctx, s);
}

namespace {

// One group of a batch stream: pairs that share (n, alpha, c).
struct BatchGroup {
    int n;
    double alpha, c, cost;
    std::vector<int64_t> idx;   // the caller's pair indices
    int64_t row0;               // first staged result row
    const HostGeometry *hg;     // the grid geometry of (n, alpha, c), made once per call
};

// Device layout of one group inside the batch arena (byte offsets).
struct GroupLayout {
    HostGeometry hg;
    int NYP = 0;
    size_t X, perm, gsize, grank, rowof, yhat, geo, pairs, offs;
    size_t cbuf, sbuf, K, k, src, Yh, lab, A;
    size_t lab_row = 0;
    int lab16 = 0;
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Assigns the arena offsets of a group: the parts the host fills (geometry,
// pair list, gather offsets) from *hc, the device-only parts from *dc.
void layout_offsets(const Geometry &g, size_t P, int esize, size_t &hc, size_t &dc, GroupLayout &L) {
    const size_t nv = 2 * P, n = (size_t)g.n, NY = (size_t)g.NY;
    L.NYP = (g.NY + 7) / 8 * 8;
    L.lab16 = lab_bytes(g) == 2;
    L.lab_row = lab_row_bytes(g);
    auto take = [](size_t &cur, size_t bytes) {
        const size_t at = cur;
        cur += align256(bytes);
        return at;
    };
    L.geo = take(hc, 4 * NY * 4);
    L.pairs = take(hc, nv * 4);
    L.offs = take(hc, nv * 8);
    L.X = take(dc, nv * n * esize);
    L.perm = take(dc, nv * n * 4);
    L.gsize = take(dc, nv * n * 4);
    L.grank = take(dc, nv * n * 4);
    L.rowof = take(dc, nv * n * L.NYP * 2);
    L.yhat = take(dc, nv * NY * 4);
    L.cbuf = take(dc, nv * g.KSUM * 4);
    L.sbuf = take(dc, nv * g.KSUM * 4);
    L.K = take(dc, nv * NY * 4);
    L.k = take(dc, nv * NY * 4);
    L.src = take(dc, nv * NY * 4);
    L.Yh = take(dc, nv * NY * 4);
    L.lab = take(dc, nv * NY * L.lab_row);
    L.A = take(dc, nv * g.ASUM * 8);
}

void layout_group(const BatchGroup &bg, int esize, size_t &hc, size_t &dc, GroupLayout &L) {
    L.hg = *bg.hg;
    L.hg.g.khat_host = L.hg.khat.data();
    layout_offsets(L.hg.g, bg.idx.size(), esize, hc, dc, L);
}

// Arena bytes of a group (both parts).
size_t group_bytes(const BatchGroup &bg, int esize) {
    GroupLayout L;
    size_t hc = 0, dc = 0;
    layout_offsets(bg.hg->g, bg.idx.size(), esize, hc, dc, L);
    return hc + dc;
}

// f(i) for every i in [0, n) on up to 16 host threads, taking `chunk`
// indices at a time (the batch stream's per-group planning: groups differ
// widely in their row counts).
template <class F>
void parallel_for(size_t n, size_t chunk, F &&f) {
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>(std::min<size_t>(hw, 16), (n + chunk - 1) / chunk);
    std::atomic<size_t> next{0};
    auto work = [&]() {
        for (;;) {
            const size_t lo = next.fetch_add(chunk);
            if (lo >= n) break;
            const size_t hi = std::min(n, lo + chunk);
            for (size_t i = lo; i < hi; i++) f(i);
        }
    };
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; t++) th.emplace_back(work);
    work();
    for (std::thread &t : th) t.join();
}

void add_profile(micx_profile &t, const micx_profile &p) {
    t.items += p.items;
    t.dp_cells += p.dp_cells;
    t.h_evals += p.h_evals;
    t.h_terms += p.h_terms;
    t.dp_ms += p.dp_ms;
    t.dp_launches += p.dp_launches;
    t.dp32_classes += p.dp32_classes;
    t.fp64_classes += p.fp64_classes;
    t.coop_classes += p.coop_classes;
    t.dp32_bound = std::max(t.dp32_bound, p.dp32_bound);
    t.recheck_pairs += p.recheck_pairs;
    t.recheck_items += p.recheck_items;
    t.recheck_ms += p.recheck_ms;
}

// DP launch key of a batch: kernel shape, plus the fixed-point scale bucket
// (classes whose scales lie within a factor 2 share one table).
inline size_t align16b(size_t b) { return (b + 15) & ~(size_t)15; }

struct DpKey {
    int fx, NL, YR, T, sb, grp;   // grp: part of a key split to fit the LDS
    int co;                       // cooperative launch (one item per workgroup)
    bool operator<(const DpKey &o) const {
        return std::tie(co, fx, NL, YR, T, sb, grp) < std::tie(o.co, o.fx, o.NL, o.YR, o.T, o.sb, o.grp);
    }
};

struct DpBucket {
    DpPlan plan;
    int nmax = 0, ksmax = 0;
    size_t rec = 0, slot = 0;
    double scale = 0.0, bound = 0.0;
    std::vector<std::pair<double, std::pair<int, int>>> classes;   // (cost, (group, yi))
    std::vector<int> items;
};

constexpr size_t kArenaBytes = (size_t)16 << 30;  // per pass over the stream (of 288 GB)

// The launch shape of one (group, row count) class of a batch pass in one
// numeric form.
struct ClassShape {
    DpKey key;          // grp: -1 (set when a key is split)
    int n, ks;          // samples, superclump slots + 1
    size_t rec, slot;   // count-record and G-table bytes per item
    double cost, scale, bound;
};

// Shapes of every class of a pass: s[off[i] + yi] for group i, in the
// requested form (s32: the 32-bit form where its bound allows, else FP64)
// and in FP64 (s64: the near-tie recheck and the classes a shared scale
// moves to FP64).
struct PassShapes {
    std::vector<size_t> off;
    std::vector<ClassShape> s32, s64;
};

// The default rules, passes of at most 24 layers: the descriptor kernels then
// keep two (FP64) or three (32-bit) targets per lane without spilling, which
// shortens the stream's largest items (measured: FP64 3.40 -> 2.95 s, DP32
// 2.29 -> 2.13 s on the 8,192-pair stream).  (Tuned choices are made for the
// all-pairs kernels.)
DpPlan class_plan(const Geometry &g, int n, int yi, int mode, double tol) {
    const DpTune rule;
    DpPlan p = dp_shape(g, n, yi, mode, tol, 24, &rule, true);
    if (p.KS >= kCoopMinK) {
        if (!p.fx && !dp_co_built(false, p.NL, p.YR, p.T) && dp_co_built(false, p.NL, p.YR, 1)) p.T = 1;
        p.co = dp_co_built(p.fx, p.NL, p.YR, p.T);
    }
    return p;
}

ClassShape class_shape(const DpPlan &p, int n) {
    ClassShape c;
    c.key = DpKey{p.fx ? 1 : 0, p.NL, p.YR, p.T, p.fx ? (int)floor(log2(p.scale)) : 0, -1, p.co ? 1 : 0};
    c.n = n;
    c.ks = p.KS;
    c.rec = (size_t)p.KS * p.RS * 4;
    c.slot = (size_t)p.x * p.KS * (p.fx ? 4 : 8);
    c.cost = (double)p.x * p.KS * p.KS;
    c.scale = p.scale;
    c.bound = p.bound;
    return c;
}

// Plans every class of groups[g0, g0 + lay.size()) on the host's threads.
void plan_pass_shapes(micx_ctx *ctx, const std::vector<BatchGroup> &groups, size_t g0,
                      const std::vector<GroupLayout> &lay, int mode, PassShapes &ps) {
    const size_t ng = lay.size();
    ps.off.assign(ng + 1, 0);
    for (size_t i = 0; i < ng; i++) ps.off[i + 1] = ps.off[i] + (size_t)lay[i].hg.g.NY;
    const bool fx = mode == MICX_MODE_DP32;
    ps.s64.resize(ps.off[ng]);
    ps.s32.resize(fx ? ps.off[ng] : 0);
    const double tol = ctx->dp32_tol;
    parallel_for(ng, 16, [&](size_t i) {
        const Geometry &g = lay[i].hg.g;
        const int n = groups[g0 + i].n;
        for (int yi = 0; yi < g.NY; yi++) {
            ps.s64[ps.off[i] + yi] = class_shape(class_plan(g, n, yi, MICX_MODE_FP64, 0.0), n);
            if (fx) ps.s32[ps.off[i] + yi] = class_shape(class_plan(g, n, yi, MICX_MODE_DP32, tol), n);
        }
    });
}

// A DpKey (grp -1) as one integer, for hashing.
uint64_t key_code(const DpKey &k) {
    return ((uint64_t)k.co << 40) | ((uint64_t)k.fx << 39) | ((uint64_t)(k.NL & 0xff) << 31) |
           ((uint64_t)(k.YR & 0xff) << 23) | ((uint64_t)(k.T & 0xff) << 15) | (uint64_t)(k.sb + 1024);
}

// Launch keys of a batch pass for one numeric form: every (group, row count)
// class goes to the launch of its kernel shape (and fixed-point scale
// bucket); a key whose largest table and largest count records together
// exceed the LDS is split, largest n first, into launches that fit (every
// class fits on its own).
void make_buckets(micx_ctx *ctx, const std::vector<BatchGroup> &groups, size_t g0,
                  const std::vector<GroupLayout> &lay, const PassShapes &ps, int mode,
                  std::map<DpKey, DpBucket> &buckets) {
    const size_t ng = lay.size();
    const bool fx = mode == MICX_MODE_DP32;
    const std::vector<ClassShape> &sh = fx ? ps.s32 : ps.s64;
    // class ids (off[i] + yi, plus total for the FP64 shape of a moved
    // class) by key, groups taken in order of decreasing n so that every
    // key's list is sorted by n
    const size_t total = ps.off[ng];
    std::vector<int> order(ng);
    for (size_t i = 0; i < ng; i++) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int u, int v) { return groups[g0 + u].n > groups[g0 + v].n; });
    std::vector<int> cgroup(total);   // group of each class
    for (size_t i = 0; i < ng; i++)
        for (size_t k = ps.off[i]; k < ps.off[i + 1]; k++) cgroup[k] = (int)i;
    std::unordered_map<uint64_t, int> kid;
    std::vector<DpKey> keys;
    std::vector<std::vector<size_t>> members;
    auto add = [&](const DpKey &key, size_t id) {
        auto it = kid.find(key_code(key));
        int k;
        if (it == kid.end()) {
            k = (int)keys.size();
            kid.emplace(key_code(key), k);
            keys.push_back(key);
            members.emplace_back();
        } else {
            k = it->second;
        }
        members[k].push_back(id);
    };
    for (int i : order)
        for (size_t k = ps.off[i]; k < ps.off[i + 1]; k++) add(sh[k].key, k);
    auto shape = [&](size_t id) -> const ClassShape & { return id < total ? sh[id] : ps.s64[id - total]; };
    if (fx) {
        // a 32-bit key's classes share one table at the smallest scale among
        // them (scales within a factor 2): a class whose bound at that scale
        // exceeds the tolerance moves to the FP64 key of its shape
        std::vector<int> touched;
        const size_t nk = keys.size();
        for (size_t k = 0; k < nk; k++) {
            if (!keys[k].fx) continue;
            double smin = 0.0;
            for (size_t id : members[k]) smin = smin == 0.0 ? sh[id].scale : std::min(smin, sh[id].scale);
            std::vector<size_t> keep, moved;
            keep.reserve(members[k].size());
            for (size_t id : members[k])
                (sh[id].bound * (sh[id].scale / smin) <= ctx->dp32_tol ? keep : moved).push_back(id);
            members[k].swap(keep);
            for (size_t id : moved) {   // (add may grow `members`)
                add(ps.s64[id].key, id + total);
                touched.push_back(kid[key_code(ps.s64[id].key)]);
            }
        }
        std::sort(touched.begin(), touched.end());
        touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
        for (int k : touched)
            std::stable_sort(members[k].begin(), members[k].end(),
                             [&](size_t u, size_t v) { return shape(u).n > shape(v).n; });
    }
    for (size_t k = 0; k < keys.size(); k++) {
        if (members[k].empty()) continue;
        const DpKey &key0 = keys[k];
        const int vb = key0.fx ? 4 : 8;
        const int NLP = (key0.NL + 16 / vb - 1) / (16 / vb) * (16 / vb);
        auto need = [&](int nmax, size_t rec, int ks) {
            if (key0.co)   // shared records and flags, four waves of eight staged sources
                return (size_t)align16b((size_t)(nmax + 1) * vb) + align16b(rec) + kCoMeta + align16b(nmax) +
                       4 * align16b((size_t)8 * NLP * vb);
            const size_t pairs = key0.NL == 1 ? (size_t)3 * ks * vb : 0;   // one-layer passes
            return (size_t)align16b((size_t)(nmax + 1) * vb) +
                   align16b(std::max(std::max((size_t)8 * NLP * vb, (size_t)nmax), pairs)) + align16b(rec);
        };
        int part = -1, nmax = 0, ks = 0;
        size_t rec = 0;
        for (size_t id : members[k]) {
            const ClassShape &c = shape(id);
            const int gi = cgroup[id < total ? id : id - total];
            const int yi = (int)((id < total ? id : id - total) - ps.off[gi]);
            if (part < 0 || need(nmax, std::max(rec, c.rec), std::max(ks, c.ks)) > 160 * 1024) {
                part++;
                nmax = c.n;
                rec = 0;
                ks = 0;
            }
            rec = std::max(rec, c.rec);
            ks = std::max(ks, c.ks);
            DpKey key = key0;
            key.grp = part;
            DpBucket &b = buckets[key];
            if (b.classes.empty())
                b.plan = class_plan(lay[gi].hg.g, c.n, yi, key0.fx ? MICX_MODE_DP32 : MICX_MODE_FP64,
                                    ctx->dp32_tol);
            b.nmax = std::max(b.nmax, c.n);
            b.ksmax = std::max(b.ksmax, c.ks);
            b.rec = std::max(b.rec, c.rec);
            b.slot = std::max(b.slot, c.slot);
            if (key0.fx) b.scale = b.scale == 0.0 ? c.scale : std::min(b.scale, c.scale);
            b.classes.push_back({c.cost, {gi, yi}});
        }
    }
    std::vector<DpBucket *> bl;
    for (auto &kv : buckets) bl.push_back(&kv.second);
    parallel_for(bl.size(), 1, [&](size_t i) {
        DpBucket &b = *bl[i];
        std::sort(b.classes.begin(), b.classes.end(),
                  [](const std::pair<double, std::pair<int, int>> &u,
                     const std::pair<double, std::pair<int, int>> &v) { return u.first > v.first; });
    });
    for (auto &kv : buckets) {
        DpBucket &b = kv.second;
        DpPlan &p = b.plan;
        p.scale = b.scale;
        p.slot_bytes = b.slot;
        p.groups = true;
        if (p.NL == 1) p.KS = b.ksmax;   // one-layer passes size their arrays by the largest item
        if (kv.first.co && dp_fit_lds_co(p, b.nmax, b.rec, ctx->cus)) continue;
        p.co = false;
        dp_fit_lds(p, b.nmax, b.rec, ctx->cus);
    }
}

// Scratch (G tables) of a set of DP launches spread round-robin over the DP
// streams: per stream, the largest need among the launches it runs.
size_t stream_scratch(const std::vector<std::pair<const DpPlan *, size_t>> &launches, int nstreams,
                      std::vector<size_t> &off) {
    std::vector<size_t> need(nstreams, 0);
    for (size_t k = 0; k < launches.size(); k++) {
        const DpPlan &p = *launches[k].first;
        const size_t waves = std::min<size_t>(launches[k].second, (size_t)p.max_waves);
        // one G table per wave, or per workgroup in a cooperative launch
        const size_t w = p.co ? waves : (waves + p.WPB - 1) / p.WPB * p.WPB;
        need[k % nstreams] = std::max(need[k % nstreams], w * p.slot_bytes);
    }
    size_t scr = 0;
    off.assign(nstreams, 0);
    for (int k = 0; k < nstreams; k++) {
        off[k] = scr;
        scr += align256(need[k]);
    }
    return scr;
}

constexpr int kDpStreams = 4;

// Runs groups[g0, g1) of a batch: per-group ranks, equipartitions and
// partitions, then one DP launch per key over all their items (spread over
// the context's DP streams), then per-group statistics into the staging rows.
int run_batch_pass(micx_ctx *ctx, const void *data_dev, int dtype, const micx_pair_desc *pairs_host,
                   std::vector<BatchGroup> &groups, size_t g0, size_t g1, int mode, hipStream_t s,
                   micx_profile &prof) {
    const int esize = dtype == MICX_F64 ? 8 : 4;
    const size_t ng = g1 - g0;
    std::vector<GroupLayout> lay(ng);
    size_t hc = 0, dc = 0;
    int nmax = 0;
    for (size_t i = 0; i < ng; i++) {
        layout_group(groups[g0 + i], esize, hc, dc, lay[i]);
        nmax = std::max(nmax, groups[g0 + i].n);
    }
    // block maps of the fused per-group stages (group, block inside the group)
    std::vector<int2> mvar, mequip, mpart, mstats;
    for (size_t i = 0; i < ng; i++) {
        const int P = (int)groups[g0 + i].idx.size(), nyb = (lay[i].hg.g.NY + 63) / 64;
        for (int v = 0; v < 2 * P; v++) mvar.push_back(make_int2((int)i, v));
        for (int b = 0; b < 2 * P * nyb; b++) mequip.push_back(make_int2((int)i, b));
        for (int b = 0; b < 2 * P * nyb; b++) mpart.push_back(make_int2((int)i, b));
        for (int p = 0; p < P; p += 64) mstats.push_back(make_int2((int)i, p));
    }
    const size_t tab_off = hc;                                      // DpGroup table
    hc += align256(ng * sizeof(DpGroup));
    const size_t gdev_off = hc;                                     // GroupDev table
    hc += align256(ng * sizeof(GroupDev));
    const size_t mvar_off = hc;
    hc += align256(mvar.size() * sizeof(int2));
    const size_t mequip_off = hc;
    hc += align256(mequip.size() * sizeof(int2));
    const size_t mpart_off = hc;
    hc += align256(mpart.size() * sizeof(int2));
    const size_t mstats_off = hc;
    hc += align256(mstats.size() * sizeof(int2));
    const size_t host_bytes = align256(hc);
    for (GroupLayout &L : lay)
        for (size_t *o : {&L.X, &L.perm, &L.gsize, &L.grank, &L.rowof, &L.yhat, &L.cbuf, &L.sbuf,
                          &L.K, &L.k, &L.src, &L.Yh, &L.lab, &L.A})
            *o += host_bytes;
    const size_t bytes = host_bytes + dc;
    RETCHK(ctx->arena.ensure(bytes));
    unsigned char *ar = ctx->arena.as<unsigned char>();
    // host-side inputs at the front of the arena: geometry, pair lists,
    // gather offsets, group table
    std::vector<unsigned char> blob(host_bytes, 0);
    std::vector<DpGroup> tab(ng);
    std::vector<GroupDev> gdev(ng);
    for (size_t i = 0; i < ng; i++) {
        const BatchGroup &bg = groups[g0 + i];
        GroupLayout &L = lay[i];
        const int NY = L.hg.g.NY;
        int *geo = (int *)(blob.data() + L.geo);
        std::copy(L.hg.xcnt.begin(), L.hg.xcnt.end(), geo);
        std::copy(L.hg.khat.begin(), L.hg.khat.end(), geo + NY);
        std::copy(L.hg.koff.begin(), L.hg.koff.end(), geo + 2 * NY);
        std::copy(L.hg.aoff.begin(), L.hg.aoff.end(), geo + 3 * NY);
        int32_t *pl = (int32_t *)(blob.data() + L.pairs);
        int64_t *of = (int64_t *)(blob.data() + L.offs);
        for (size_t p = 0; p < bg.idx.size(); p++) {
            pl[2 * p] = (int32_t)(2 * p);
            pl[2 * p + 1] = (int32_t)(2 * p + 1);
            of[2 * p] = pairs_host[bg.idx[p]].off_x;
            of[2 * p + 1] = pairs_host[bg.idx[p]].off_y;
        }
        Geometry &g = L.hg.g;
        g.xcnt = (int *)(ar + L.geo);
        g.khat = g.xcnt + NY;
        g.koff = g.xcnt + 2 * NY;
        g.aoff = g.xcnt + 3 * NY;
        DpGroup &t = tab[i];
        t.n = bg.n;
        t.NY = NY;
        t.KSUM = g.KSUM;
        t.ASUM = g.ASUM;
        t.lab16 = L.lab16;
        t.lab_row = L.lab_row;
        t.xcnt = g.xcnt;
        t.khat = g.khat;
        t.koff = g.koff;
        t.aoff = g.aoff;
        t.Yh = (const int *)(ar + L.Yh);
        t.cbuf = (const int *)(ar + L.cbuf);
        t.sbuf = (const int *)(ar + L.sbuf);
        t.K = (const int *)(ar + L.K);
        t.src = (const int *)(ar + L.src);
        t.lab = ar + L.lab;
        t.A = (double *)(ar + L.A);

        GroupDev &d = gdev[i];
        d.n = bg.n;
        d.NY = NY;
        d.NYP = L.NYP;
        d.KSUM = g.KSUM;
        d.ASUM = g.ASUM;
        d.B = g.B;
        d.W = g.W;
        d.nv = (int)(2 * bg.idx.size());
        d.npairs = (int)bg.idx.size();
        d.lab16 = L.lab16;
        d.lab_row = L.lab_row;
        d.offs = (const int64_t *)(ar + L.offs);
        d.X = ar + L.X;
        d.perm = (int *)(ar + L.perm);
        d.gsize = (int *)(ar + L.gsize);
        d.grank = (int *)(ar + L.grank);
        d.rowof = (uint16_t *)(ar + L.rowof);
        d.yhat = (int *)(ar + L.yhat);
        d.xcnt = g.xcnt;
        d.khat = g.khat;
        d.koff = g.koff;
        d.aoff = g.aoff;
        d.cbuf = (int *)(ar + L.cbuf);
        d.sbuf = (int *)(ar + L.sbuf);
        d.K = (int *)(ar + L.K);
        d.k = (int *)(ar + L.k);
        d.src = (int *)(ar + L.src);
        d.Yh = (int *)(ar + L.Yh);
        d.lab = ar + L.lab;
        d.A = (double *)(ar + L.A);
        d.pairs = (const int32_t *)(ar + L.pairs);
        d.out = ctx->bout.as<double>() + 4 * bg.row0;
        d.compat = ctx->compat;
    }
    memcpy(blob.data() + tab_off, tab.data(), ng * sizeof(DpGroup));
    memcpy(blob.data() + gdev_off, gdev.data(), ng * sizeof(GroupDev));
    memcpy(blob.data() + mvar_off, mvar.data(), mvar.size() * sizeof(int2));
    memcpy(blob.data() + mequip_off, mequip.data(), mequip.size() * sizeof(int2));
    memcpy(blob.data() + mpart_off, mpart.data(), mpart.size() * sizeof(int2));
    memcpy(blob.data() + mstats_off, mstats.data(), mstats.size() * sizeof(int2));
    RETCHK(stage_copy(ctx, ar, blob.data(), host_bytes, s));
    RETCHK(ctx->xlogx.ensure((size_t)(nmax + 1) * sizeof(double)));
    int *status = ctx->status.as<int>();
    HIPCHK(launch_xlogx(nmax, ctx->xlogx.as<double>(), s));
    unsigned long long *counters = nullptr;
    if (ctx->profiling) {
        RETCHK(ctx->counters.ensure(4 * sizeof(unsigned long long)));
        counters = ctx->counters.as<unsigned long long>();
        HIPCHK(launch_zero(counters, 8, s));
    }
    while ((int)ctx->dstreams.size() < kDpStreams) {
        hipStream_t st;
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        ctx->dstreams.push_back(st);
    }
    auto fork = [&]() -> int {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIPCHK(hipEventRecord(e, s));
        for (hipStream_t st : ctx->dstreams) HIPCHK(hipStreamWaitEvent(st, e, 0));
        HIPCHK(hipEventDestroy(e));
        return MICX_OK;
    };
    auto join = [&]() -> int {
        for (hipStream_t st : ctx->dstreams) {
            hipEvent_t e;
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            HIPCHK(hipEventRecord(e, st));
            HIPCHK(hipStreamWaitEvent(s, e, 0));
            HIPCHK(hipEventDestroy(e));
        }
        return MICX_OK;
    };
    // per-group stages, each one launch over all groups of the pass
    const GroupDev *gd = (const GroupDev *)(ar + gdev_off);
    HIPCHK(launch_gather_g(data_dev, esize, gd, (const int2 *)(ar + mvar_off), (int)mvar.size(), s));
    HIPCHK(launch_rank_g(gd, (const int2 *)(ar + mvar_off), (int)mvar.size(), nmax, dtype, status, s));
    HIPCHK(launch_equip_g(gd, (const int2 *)(ar + mequip_off), (int)mequip.size(), nmax, s));
    HIPCHK(launch_part_g(gd, (const int2 *)(ar + mpart_off), (int)mpart.size(), s));
    if (counters) {
        for (size_t i = 0; i < ng; i++) {
            GroupLayout &L = lay[i];
            ItemBuffers ib;
            ib.K = (int *)(ar + L.K);
            EquipTables et;
            et.NY = L.hg.g.NY;
            et.yhat = (int *)(ar + L.yhat);
            PairSource ps;
            ps.pairs = (const int32_t *)(ar + L.pairs);
            ps.p0 = 0;
            ps.m = (int)(2 * groups[g0 + i].idx.size());
            HIPCHK(launch_work(et, L.hg.g, ps, (int)groups[g0 + i].idx.size(), ib, counters, s));
        }
    }
    // DP keys: every (group, row count) class goes to the launch of its shape
    PassShapes shapes;
    plan_pass_shapes(ctx, groups, g0, lay, mode, shapes);
    std::map<DpKey, DpBucket> buckets;
    make_buckets(ctx, groups, g0, lay, shapes, mode, buckets);
    // keys run largest first (their longest items start at once), round-robin
    // over the DP streams
    std::vector<std::pair<const DpKey, DpBucket> *> keys;
    for (auto &kv : buckets) keys.push_back(&kv);
    size_t nitems = 0, tabs = 0;
    for (auto *kp : keys) {
        DpBucket &b = kp->second;
        for (auto &c : b.classes) {
            const int gi = c.second.first, yi = c.second.second;
            const int npo = (int)(2 * groups[g0 + gi].idx.size());
            for (int po = 0; po < npo; po++) {
                b.items.push_back(gi);
                b.items.push_back(yi);
                b.items.push_back(po);
            }
        }
        nitems += b.items.size() / 3;
        if (b.plan.fx) tabs++;
    }
    std::sort(keys.begin(), keys.end(), [](const std::pair<const DpKey, DpBucket> *u,
                                           const std::pair<const DpKey, DpBucket> *v) {
        return u->second.classes.front().first > v->second.classes.front().first;
    });
    // item lists and fixed-point tables, one region per key
    RETCHK(ctx->gitems.ensure(nitems * 3 * sizeof(int)));
    RETCHK(ctx->fxtab.ensure(std::max<size_t>(tabs, 1) * (size_t)(nmax + 1) * sizeof(uint32_t)));
    std::vector<int> allitems;
    allitems.reserve(nitems * 3);
    for (auto *kp : keys) allitems.insert(allitems.end(), kp->second.items.begin(), kp->second.items.end());
    RETCHK(stage_copy(ctx, ctx->gitems.p, allitems.data(), allitems.size() * sizeof(int), s));
    // near-tie recheck of the 32-bit form: FP64 launch keys over every class
    // of the pass, each with a device list of the items queued for it
    // (capacity: all items of its classes), per-item flag bits and the
    // flagged pairs (StreamRecheck)
    // (a class's bound at its bucket's shared scale: the bound scales as 1/S)
    auto shared_bound = [&](const DpBucket &b, const std::pair<int, int> &c) {
        const ClassShape &cs = shapes.s32[shapes.off[c.first] + c.second];
        return cs.bound * (cs.scale / b.plan.scale);
    };
    double bound = 0.0;
    for (auto &kv : buckets) {
        const DpBucket &b = kv.second;
        if (!b.plan.fx) continue;
        for (auto &c : b.classes) bound = std::max(bound, shared_bound(b, c.second));
    }
    const bool recheck = bound > 0.0;
    std::map<DpKey, DpBucket> rbuckets;
    std::vector<std::pair<const DpKey, DpBucket> *> rkeys;
    std::vector<int> rcap, rkoff, keyof;
    StreamRecheck srq;
    size_t rc_words = 0;
    int ptotal = 0;
    if (recheck) {
        make_buckets(ctx, groups, g0, lay, shapes, MICX_MODE_FP64, rbuckets);
        for (auto &kv : rbuckets) rkeys.push_back(&kv);
        std::vector<size_t> kbase(ng, 0);
        size_t nk = 0;
        for (size_t i = 0; i < ng; i++) {
            kbase[i] = nk;
            nk += lay[i].hg.g.NY;
        }
        keyof.assign(nk, -1);
        int koff = 0;
        for (size_t k = 0; k < rkeys.size(); k++) {
            int cap = 0;
            for (auto &c : rkeys[k]->second.classes) {
                keyof[kbase[c.second.first] + c.second.second] = (int)k;
                cap += (int)(2 * groups[g0 + c.second.first].idx.size());
            }
            rcap.push_back(cap);
            rkoff.push_back(koff);
            koff += cap;
        }
        size_t fw = 0;
        std::vector<size_t> fbase(ng);
        for (size_t i = 0; i < ng; i++) {
            fbase[i] = fw;
            ptotal += (int)groups[g0 + i].idx.size();
            fw += 2 * groups[g0 + i].idx.size() * (size_t)((lay[i].hg.g.NY + 31) / 32);
        }
        rc_words = rkeys.size() + 1 + fw;
        RETCHK(ctx->rcwords.ensure(rc_words * sizeof(unsigned)));
        RETCHK(ctx->rclist.ensure(std::max<size_t>((size_t)koff * 3, 1) * sizeof(int)));
        RETCHK(ctx->rcpairs.ensure((size_t)2 * ptotal * sizeof(int)));
        RETCHK(ctx->rcmeta.ensure((rkeys.size() + nk) * sizeof(int)));
        int *meta = ctx->rcmeta.as<int>();
        std::vector<int> hmeta(rkoff);
        hmeta.insert(hmeta.end(), keyof.begin(), keyof.end());
        RETCHK(stage_copy(ctx, meta, hmeta.data(), hmeta.size() * sizeof(int), s));
        srq.band = 2.0 * bound + 1e-12;
        srq.kcount = ctx->rcwords.as<int>();
        srq.pcount = srq.kcount + rkeys.size();
        srq.klist = ctx->rclist.as<int>();
        srq.koff = meta;
        srq.plist = ctx->rcpairs.as<int>();
        unsigned *flags = (unsigned *)(srq.pcount + 1);
        for (size_t i = 0; i < ng; i++) {
            gdev[i].iflag = flags + fbase[i];
            gdev[i].nyw = (lay[i].hg.g.NY + 31) / 32;
            gdev[i].keyof = meta + rkeys.size() + kbase[i];
        }
        RETCHK(stage_copy(ctx, ar + gdev_off, gdev.data(), ng * sizeof(GroupDev), s));
        HIPCHK(launch_zero(ctx->rcwords.p, rc_words, s));
    }
    // scratch per DP stream: the largest need among the keys it runs (main
    // and recheck launches run one after the other and share it)
    std::vector<size_t> scr_off, rscr_off;
    size_t scr;
    {
        std::vector<std::pair<const DpPlan *, size_t>> ml, rl;
        for (auto *kp : keys) ml.push_back({&kp->second.plan, kp->second.items.size() / 3});
        scr = stream_scratch(ml, kDpStreams, scr_off);
        for (size_t k = 0; k < rkeys.size(); k++) rl.push_back({&rkeys[k]->second.plan, (size_t)rcap[k]});
        scr = std::max(scr, stream_scratch(rl, kDpStreams, rscr_off));
    }
    RETCHK(ctx->scratch.ensure(std::max<size_t>(scr, 1)));
    RETCHK(fork());
    std::vector<hipEvent_t> ev;
    {
        int k = 0, t = 0;
        size_t off = 0;
        for (auto *kp : keys) {
            DpBucket &b = kp->second;
            hipStream_t st = ctx->dstreams[k % kDpStreams];
            const uint32_t *tab = nullptr;
            if (b.plan.fx) {
                uint32_t *tp = ctx->fxtab.as<uint32_t>() + (size_t)t * (nmax + 1);
                HIPCHK(launch_fxtable(b.nmax, b.plan, ctx->xlogx.as<double>(), tp, st));
                tab = tp;
                t++;
            }
            if (ctx->profiling) {
                hipEvent_t e0, e1;
                HIPCHK(hipEventCreate(&e0));
                HIPCHK(hipEventCreate(&e1));
                ev.push_back(e0);
                ev.push_back(e1);
                HIPCHK(hipEventRecord(e0, st));
            }
            const int nit = (int)(b.items.size() / 3);
            HIPCHK(launch_dp_items((const DpGroup *)(ar + tab_off), ctx->gitems.as<int>() + off, nit, b.nmax,
                                   ctx->xlogx.as<double>(), tab,
                                   ctx->scratch.as<unsigned char>() + scr_off[k % kDpStreams], b.plan,
                                   ctx->compat, st, nullptr, status));
            if (ctx->profiling) HIPCHK(hipEventRecord(ev.back(), st));
            off += b.items.size();
            k++;
        }
    }
    // statistics into the staging rows, once every DP key is done
    RETCHK(join());
    HIPCHK(launch_stats_g(gd, (const int2 *)(ar + mstats_off), (int)mstats.size(), s,
                          recheck ? &srq : nullptr, status));
    micx_profile pp{};
    if (recheck) {
        // FP64 re-run of the queued items, key by key, then the flagged pairs'
        // statistics again
        hipEvent_t r0 = nullptr, r1 = nullptr;
        if (ctx->profiling) {
            HIPCHK(hipEventCreate(&r0));
            HIPCHK(hipEventCreate(&r1));
            HIPCHK(hipEventRecord(r0, s));
        }
        RETCHK(fork());
        for (size_t k = 0; k < rkeys.size(); k++) {
            const DpBucket &b = rkeys[k]->second;
            HIPCHK(launch_dp_items((const DpGroup *)(ar + tab_off), srq.klist + 3 * (size_t)rkoff[k], rcap[k],
                                   b.nmax, ctx->xlogx.as<double>(), nullptr,
                                   ctx->scratch.as<unsigned char>() + rscr_off[k % kDpStreams], b.plan,
                                   ctx->compat, ctx->dstreams[k % kDpStreams], srq.kcount + k, status));
        }
        RETCHK(join());
        HIPCHK(launch_stats_g_list(gd, srq.plist, srq.pcount, ptotal, s, status));
        if (ctx->profiling) {
            HIPCHK(hipEventRecord(r1, s));
            std::vector<int> h(rkeys.size() + 1);
            HIPCHK(hipMemcpyAsync(h.data(), srq.kcount, h.size() * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (size_t k = 0; k < rkeys.size(); k++) pp.recheck_items += h[k];
            pp.recheck_pairs = h[rkeys.size()];
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, r0, r1));
            pp.recheck_ms = ms;
            hipEventDestroy(r0);
            hipEventDestroy(r1);
        }
    }
    if (ctx->profiling) {
        HIPCHK(hipStreamSynchronize(s));
        for (size_t k = 0; k + 1 < ev.size(); k += 2) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            pp.dp_ms += ms;
        }
        unsigned long long h[4];
        HIPCHK(hipMemcpy(h, counters, sizeof(h), hipMemcpyDeviceToHost));
        pp.items = (int64_t)h[0];
        pp.dp_cells = (int64_t)h[1];
        pp.h_evals = (int64_t)h[2];
        pp.h_terms = (int64_t)h[3];
        pp.dp_launches = (int)(ev.size() / 2);
    }
    for (hipEvent_t e : ev) hipEventDestroy(e);
    for (auto &kv : buckets) {
        const DpBucket &b = kv.second;
        for (auto &c : b.classes) {
            if (b.plan.fx) {
                pp.dp32_classes++;
                pp.dp32_bound = std::max(pp.dp32_bound, shared_bound(b, c.second));
            } else {
                pp.fp64_classes++;
            }
            pp.coop_classes += b.plan.co ? 1 : 0;
        }
    }
    add_profile(prof, pp);
    return MICX_OK;
}

}  // namespace

extern "C" int micx_batch(micx_ctx *ctx, const void *data_dev, int dtype,
                          const micx_pair_desc *pairs_host, int64_t npairs, int mode, double *out_dev,
                          void *stream) {
    if (!ctx || !data_dev || !pairs_host || !out_dev || npairs < 1) return MICX_EINVAL;
    if (dtype != MICX_F32 && dtype != MICX_F64 && dtype != MICX_I32) return MICX_EINVAL;
    const auto t_entry = std::chrono::steady_clock::now();
    for (int64_t k = 0; k < npairs; k++) {
        const micx_pair_desc &d = pairs_host[k];
        RETCHK(check_common(ctx, d.n, d.alpha, d.c, mode));
        if (d.off_x < 0 || d.off_y < 0) return MICX_EINVAL;
    }
    // pairs that share (n, alpha, c) share the grid geometry (made once per
    // key, on the host's threads); a group whose buffers would fill a large
    // part of the arena is split
    std::map<std::tuple<int, double, double>, std::vector<int64_t>> byKey;
    for (int64_t k = 0; k < npairs; k++)
        byKey[std::make_tuple(pairs_host[k].n, pairs_host[k].alpha, pairs_host[k].c)].push_back(k);
    std::vector<const std::pair<const std::tuple<int, double, double>, std::vector<int64_t>> *> kl;
    for (auto &kv : byKey) kl.push_back(&kv);
    std::vector<HostGeometry> kgeo(kl.size());
    std::vector<char> kfits(kl.size(), 0);
    parallel_for(kl.size(), 32, [&](size_t i) {
        const int n = std::get<0>(kl[i]->first);
        make_geometry(n, micx_grid_bound(n, std::get<1>(kl[i]->first)), std::get<2>(kl[i]->first), kgeo[i],
                      ctx->compat);
        const DpTune rule;   // the batch stream plans by the default rules
        kfits[i] = dp_fits(kgeo[i].g, n, &rule) ? 1 : 0;
    });
    for (char f : kfits)
        if (!f) return MICX_ETOOBIG;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int esize = dtype == MICX_F64 ? 8 : 4;
    std::vector<BatchGroup> groups;
    for (size_t ki = 0; ki < kl.size(); ki++) {
        const auto &kv = *kl[ki];
        BatchGroup g;
        g.n = std::get<0>(kv.first);
        g.alpha = std::get<1>(kv.first);
        g.c = std::get<2>(kv.first);
        g.hg = &kgeo[ki];
        g.idx = {kv.second.front()};
        const size_t per_pair = group_bytes(g, esize);   // upper bound per pair
        const size_t maxp = std::max<size_t>(1, kArenaBytes / 4 / std::max<size_t>(per_pair, 1));
        const double B = (double)micx_grid_bound(g.n, g.alpha);
        for (size_t i0 = 0; i0 < kv.second.size(); i0 += maxp) {
            BatchGroup part = g;
            part.idx.assign(kv.second.begin() + i0,
                            kv.second.begin() + std::min(kv.second.size(), i0 + maxp));
            part.cost = (double)part.idx.size() * (double)g.n * B * B * B * g.c * g.c;
            groups.push_back(std::move(part));
        }
    }
    // largest first, so the longest items start early in each pass
    std::sort(groups.begin(), groups.end(), [](const BatchGroup &a, const BatchGroup &b) { return a.cost > b.cost; });
    std::vector<int64_t> order;
    order.reserve(npairs);
    for (BatchGroup &g : groups) {
        g.row0 = (int64_t)order.size();
        order.insert(order.end(), g.idx.begin(), g.idx.end());
    }
    RETCHK(ctx->bout.ensure((size_t)npairs * 4 * sizeof(double)));
    RETCHK(ctx->bidx.ensure((size_t)npairs * sizeof(int64_t)));
    RETCHK(begin_status(ctx, s));
    micx_profile total{};
    for (size_t g0 = 0; g0 < groups.size();) {
        size_t g1 = g0, bytes = 0;
        while (g1 < groups.size()) {
            const size_t b = group_bytes(groups[g1], esize);
            if (g1 > g0 && bytes + b > kArenaBytes) break;
            bytes += b;
            g1++;
        }
        RETCHK(run_batch_pass(ctx, data_dev, dtype, pairs_host, groups, g0, g1, mode, s, total));
        g0 = g1;
    }
    RETCHK(stage_copy(ctx, ctx->bidx.p, order.data(), order.size() * sizeof(int64_t), s));
    HIPCHK(launch_scatter_rows(ctx->bout.as<double>(), ctx->bidx.as<int64_t>(), npairs, out_dev, s,
                               ctx->status.as<int>()));
    const int rc = end_status(ctx, s);
    total.host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_entry).count();
    ctx->prof = total;
    return rc;
}

extern "C" int micx_compute_score(micx_ctx *ctx, const micx_problem *problem, const micx_param *param,
                                  int mode, micx_score **out) {
    if (!problem || !param) return MICX_EINVAL;
    const int n = problem->n;
    const double *x = problem->x, *y = problem->y, alpha = param->alpha, c = param->c;
    RETCHK(check_common(ctx, n, alpha, c, mode));
    if (!x || !y || !out) return MICX_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = nullptr;
    HostGeometry hg;
    const int B = micx_grid_bound(n, alpha);
    make_geometry(n, B, c, hg, ctx->compat);
    if (!dp_fits(hg.g, n)) return MICX_ETOOBIG;
    RETCHK(begin_status(ctx, s));
    RETCHK(upload_geometry(ctx, hg, s, c));
    RETCHK(upload_pair_input(ctx, x, y, n, s));
    RankTables rt;
    EquipTables et;
    RETCHK(prepare_variables(ctx, ctx->input.p, MICX_F64, 2, n, hg.g, false, rt, et, s));
    const int W = hg.g.W;
    const size_t WW = (size_t)W * W;
    RETCHK(ctx->dense.ensure((4 + 3 * WW) * sizeof(double)));
    double *d = ctx->dense.as<double>();
    RETCHK(run_pairs(ctx, rt, et, hg.g, ctx->pairs.as<int32_t>(), 1, 2, mode, d, d + 4,
                     d + 4 + WW, d + 4 + 2 * WW, s));
    RETCHK(end_status(ctx, s));
    std::vector<double> h(4 + 3 * WW);
    HIPCHK(hipMemcpyAsync(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    RETCHK(status_code(*ctx->hstatus));
    micx_score *sc = (micx_score *)calloc(1, sizeof(micx_score));
    if (!sc) return MICX_ENOMEM;
    sc->n = n;
    sc->B = hg.g.B;
    sc->W = W;
    sc->M = (double *)malloc(WW * sizeof(double));
    sc->Axy = (double *)malloc(WW * sizeof(double));
    sc->Ayx = (double *)malloc(WW * sizeof(double));
    if (!sc->M || !sc->Axy || !sc->Ayx) {
        micx_free_score(sc);
        return MICX_ENOMEM;
    }
    memcpy(sc->stats, h.data(), 4 * sizeof(double));
    memcpy(sc->M, h.data() + 4, WW * sizeof(double));
    memcpy(sc->Axy, h.data() + 4 + WW, WW * sizeof(double));
    memcpy(sc->Ayx, h.data() + 4 + 2 * WW, WW * sizeof(double));
    *out = sc;
    return MICX_OK;
}

extern "C" int micx_set_profiling(micx_ctx *ctx, int enable) {
    if (!ctx) return MICX_EINVAL;
    ctx->profiling = enable ? 1 : 0;
    return MICX_OK;
}

extern "C" int micx_set_compat(micx_ctx *ctx, int flags) {
    const int all = MICX_COMPAT_TIE_STRICT | MICX_COMPAT_DESIRED_INT | MICX_COMPAT_COMBINE_INDEX |
                    MICX_COMPAT_NORM_BY_Y | MICX_COMPAT_BOUND_STRICT | MICX_COMPAT_KHAT_PLUS1;
    if (!ctx || (flags & ~all)) return MICX_EINVAL;
    ctx->compat = flags;
    return MICX_OK;
}

extern "C" int micx_set_dp32_tolerance(micx_ctx *ctx, double tol) {
    if (!ctx || !(tol > 0.0)) return MICX_EINVAL;
    ctx->dp32_tol = tol;
    return MICX_OK;
}

extern "C" double micx_dp32_bound(int n, int x, int y) {
    if (n < 1 || x < 2 || y < 2) return 0.0;
    const double S = floor(4294967296.0 / (1.02 * (double)n * log((double)y)));
    return dp32_bound(n, x, y, S);
}

extern "C" int micx_get_profile(micx_ctx *ctx, micx_profile *out) {
    if (!ctx || !out) return MICX_EINVAL;
    *out = ctx->prof;
    return MICX_OK;
}

extern "C" void micx_free_score(micx_score *s) {
    if (!s) return;
    free(s->M);
    free(s->Axy);
    free(s->Ayx);
    free(s);
}

extern "C" double micx_mic(const micx_score *s) { return s ? s->stats[0] : NAN; }
extern "C" double micx_mas(const micx_score *s) { return s ? s->stats[1] : NAN; }
extern "C" double micx_mev(const micx_score *s) { return s ? s->stats[2] : NAN; }

// MCN(eps): eps = 0 returns the value the device computed with the score.
// Other eps values scan the returned matrix: min log2(xy) over cells with
// M >= (1 - eps) MIC (Appendix A item 2).
extern "C" double micx_mcn(const micx_score *s, double eps) {
    if (!s) return NAN;
    if (eps == 0.0) return s->stats[3];
    const double thr = (1.0 - eps) * s->stats[0] - 1e-12;
    double best = INFINITY;
    for (int yy = 2; yy <= s->W + 1; yy++)
        for (int xx = 2; xx * yy <= s->B; xx++) {
            const double v = s->M[(size_t)(yy - 2) * s->W + (xx - 2)];
            if (v >= thr) best = std::min(best, log2((double)(xx * yy)));
        }
    return best;
}

namespace {

// Integer stages of one pair for the debug readbacks: geometry, ranks,
// equipartitions (with row starts) and partitions of both orientations,
// synchronised; MICX_ENONFINITE for NaN or infinite input.
int debug_stages(micx_ctx *ctx, const micx_problem *problem, const micx_param *param, int orient, int ry,
                 HostGeometry &hg, RankTables &rt, EquipTables &et, ItemBuffers &ib) {
    if (!problem || !param) return MICX_EINVAL;
    const int n = problem->n;
    const double alpha = param->alpha, c = param->c;
    RETCHK(check_common(ctx, n, alpha, c, MICX_MODE_FP64));
    const int B = micx_grid_bound(n, alpha);
    if (!problem->x || !problem->y) return MICX_EINVAL;
    if (orient != 0 && orient != 1) return MICX_EINVAL;
    if (ry < 2 || ry > B / 2) return MICX_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = nullptr;
    make_geometry(n, B, c, hg, ctx->compat);
    if (ry - 2 >= hg.g.NY) return MICX_EINVAL;
    if (!dp_fits(hg.g, n)) return MICX_ETOOBIG;
    RETCHK(begin_status(ctx, s));
    RETCHK(upload_geometry(ctx, hg, s, c));
    RETCHK(upload_pair_input(ctx, problem->x, problem->y, n, s));
    RETCHK(prepare_variables(ctx, ctx->input.p, MICX_F64, 2, n, hg.g, true, rt, et, s));
    RETCHK(ensure_items(ctx, hg.g, 1, ib));
    PairSource ps;
    ps.pairs = ctx->pairs.as<int32_t>();
    ps.m = 2;
    HIPCHK(launch_part(rt, et, hg.g, ps, 1, ib, s));
    RETCHK(end_status(ctx, s));
    HIPCHK(hipStreamSynchronize(s));
    return status_code(*ctx->hstatus);
}

}  // namespace

extern "C" int micx_debug_item(micx_ctx *ctx, const micx_problem *problem, const micx_param *param,
                               int orient, int ry, int *yhat, int *row_starts, int *k, int *K, int *ends) {
    if (!yhat || !row_starts || !k || !K || !ends) return MICX_EINVAL;
    HostGeometry hg;
    RankTables rt;
    EquipTables et;
    ItemBuffers ib;
    RETCHK(debug_stages(ctx, problem, param, orient, ry, hg, rt, et, ib));
    const Geometry &g = hg.g;
    const int yi = ry - 2;
    const int V = orient ? 0 : 1;   // row variable
    const size_t it = (size_t)orient * g.NY + yi;
    int yh = 0, kk = 0, KK = 0, src = 0;
    HIPCHK(hipMemcpy(&yh, et.yhat + (size_t)V * g.NY + yi, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&kk, ib.k + it, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&KK, ib.K + it, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&src, ib.src + it, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(row_starts, et.rowstart + ((size_t)V * g.NY + yi) * et.RS,
                     sizeof(int) * (size_t)(yh + 1), hipMemcpyDeviceToHost));
    const int *eb = (src ? ib.sbuf : ib.cbuf) + (size_t)orient * g.KSUM + hg.koff[yi];
    HIPCHK(hipMemcpy(ends, eb, sizeof(int) * (size_t)KK, hipMemcpyDeviceToHost));
    *yhat = yh;
    *k = kk;
    *K = KK;
    return MICX_OK;
}

extern "C" int micx_debug_tables(micx_ctx *ctx, const micx_problem *problem, const micx_param *param,
                                 int orient, int ry, int *group_start_x, int *group_start_y, int *counts) {
    if (!group_start_x || !group_start_y) return MICX_EINVAL;
    HostGeometry hg;
    RankTables rt;
    EquipTables et;
    ItemBuffers ib;
    RETCHK(debug_stages(ctx, problem, param, orient, ry, hg, rt, et, ib));
    const int n = problem->n;
    HIPCHK(hipMemcpy(group_start_x, rt.grank, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(group_start_y, rt.grank + n, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost));
    if (!counts) return MICX_OK;
    // the DP's own count table: a debug instance of the DP kernel writes the
    // table it builds in LDS for both items of the row count
    const Geometry &g = hg.g;
    const int yi = ry - 2;
    const size_t per = (size_t)(hg.khat[yi] + 1) * (size_t)(ry + 1);
    RETCHK(ctx->dbg.ensure(4 * per * sizeof(int)));
    PairSource ps;
    ps.pairs = ctx->pairs.as<int32_t>();
    ps.m = 2;
    HIPCHK(launch_dp_debug(rt, et, g, ps, ib, ctx->xlogx.as<double>(), yi, ctx->cus, ctx->dbg.as<int>(), nullptr));
    int yh = 0, KK = 0;
    const int V = orient ? 0 : 1;
    HIPCHK(hipMemcpy(&yh, et.yhat + (size_t)V * g.NY + yi, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&KK, ib.K + (size_t)orient * g.NY + yi, sizeof(int), hipMemcpyDeviceToHost));
    std::vector<int> tab(4 * per);
    HIPCHK(hipMemcpy(tab.data(), ctx->dbg.as<int>(), 4 * per * sizeof(int), hipMemcpyDeviceToHost));
    // the kernel's records: (K+1) rows of stride ry+1, e_t then the rows'
    // counts; the two count scans must agree
    const int *t0 = tab.data() + (size_t)orient * per, *t1 = tab.data() + (2 + (size_t)orient) * per;
    for (int t = 0; t <= KK; t++)
        for (int r = 0; r <= yh; r++)
            if (t0[(size_t)t * (ry + 1) + r] != t1[(size_t)t * (ry + 1) + r]) return MICX_EDEVICE;
    for (int t = 0; t <= KK; t++)
        for (int r = 0; r < yh; r++) counts[(size_t)t * yh + r] = t0[(size_t)t * (ry + 1) + 1 + r];
    return MICX_OK;
}

// ------------------------------------------------------------------ tuning

namespace {

struct TuneCand {
    DpTune tv;
    DpPlan p;
};

}  // namespace

extern "C" int micx_autotune(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n,
                             const micx_param *param, int mode, const char *cache_path, void *stream) {
    if (!param) return MICX_EINVAL;
    const double alpha = param->alpha, c = param->c;
    RETCHK(check_common(ctx, n, alpha, c, mode));
    if (!X_dev || m < 2) return MICX_EINVAL;
    if (dtype != MICX_F32 && dtype != MICX_F64 && dtype != MICX_I32) return MICX_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    HostGeometry hg;
    make_geometry(n, micx_grid_bound(n, alpha), c, hg, ctx->compat);
    const Geometry &g = hg.g;
    if (!dp_fits(g, n)) return MICX_ETOOBIG;
    // the sample: all pairs of the first (up to) 192 variables, enough items
    // per row count to fill the device several times over
    const int ms = std::min(m, 192);
    const int npairs = ms * (ms - 1) / 2;
    RETCHK(begin_status(ctx, s));
    RETCHK(upload_geometry(ctx, hg, s, c));
    RankTables rt;
    EquipTables et;
    RETCHK(prepare_variables(ctx, X_dev, dtype, ms, n, g, false, rt, et, s));
    ItemBuffers ib;
    RETCHK(ensure_items(ctx, g, npairs, ib));
    PairSource ps;
    ps.pairs = nullptr;
    ps.p0 = 0;
    ps.m = ms;
    HIPCHK(launch_part(rt, et, g, ps, npairs, ib, s));
    RETCHK(end_status(ctx, s));
    HIPCHK(hipStreamSynchronize(s));
    RETCHK(status_code(*ctx->hstatus));
    int ylean = g.NY;
    while (ylean > 0 && g.B / (ylean + 1) == 2) ylean--;
    const size_t tabn = (size_t)n + 1;
    RETCHK(ctx->fxtab.ensure((size_t)g.NY * tabn * sizeof(uint32_t)));
    RETCHK(ctx->counters.ensure(4 * sizeof(unsigned long long)));
    unsigned long long *sum = ctx->counters.as<unsigned long long>();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const DpTune rule;   // all zero: the default rules
    int rc = MICX_OK;
    for (int yi = 0; yi < ylean && rc == MICX_OK; yi++) {
        const DpPlan p0 = dp_shape(g, n, yi, mode, ctx->dp32_tol, 36, &rule);
        const uint32_t *tab = nullptr;
        if (p0.fx) {
            FxScales sc;
            sc.scale[0] = p0.scale;
            sc.cls[0] = yi;
            HIPCHK(launch_fxtables(n, sc, 1, ctx->xlogx.as<double>(), ctx->fxtab.as<uint32_t>(), tabn, s));
            tab = ctx->fxtab.as<uint32_t>() + yi * tabn;
        }
        // candidate shapes: targets per lane, layer cap, workgroups per CU;
        // distinct launches only (the planner steps down to built shapes)
        std::vector<TuneCand> cands;
        for (int T : {0, 1, 2, 3})
            for (int cap : {0, 36, 24, 16, 12})
                for (int wgs : {0, 1, 2, 4}) {
                    TuneCand tc;
                    tc.tv.T = T;
                    tc.tv.nlcap = cap;
                    tc.tv.wgs = wgs;
                    tc.p = dp_shape(g, n, yi, mode, ctx->dp32_tol, 36, &tc.tv);
                    dp_fit_lds(tc.p, n, (size_t)tc.p.KS * tc.p.RS * 4, ctx->cus);
                    if (tc.p.lds > 160 * 1024) continue;
                    bool dup = false;
                    for (const TuneCand &o : cands)
                        dup |= o.p.NL == tc.p.NL && o.p.YR == tc.p.YR && o.p.T == tc.p.T && o.p.SB == tc.p.SB &&
                               o.p.WPB == tc.p.WPB;
                    if (!dup) cands.push_back(tc);
                }
        double best_ms = 1e300;
        DpTune best;
        unsigned long long ref = 0;
        for (size_t k = 0; k < cands.size(); k++) {
            const DpPlan &p = cands[k].p;
            const size_t waves = (size_t)std::min<int64_t>(p.max_waves, 2 * (int64_t)npairs);
            RETCHK(ctx->scratch.ensure(((waves + p.WPB - 1) / p.WPB) * p.WPB * p.slot_bytes));
            HIPCHK(launch_dp(rt, et, g, ps, npairs, ib, ctx->xlogx.as<double>(), tab, ctx->scratch.p, yi, p, s));
            HIPCHK(hipEventRecord(e0, s));
            for (int r = 0; r < 2; r++)
                HIPCHK(launch_dp(rt, et, g, ps, npairs, ib, ctx->xlogx.as<double>(), tab, ctx->scratch.p, yi, p,
                                 s));
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(launch_zero(sum, 2, s));
            HIPCHK(launch_checksum(ib.A, 2 * npairs, g.ASUM, hg.aoff[yi], hg.xcnt[yi] - 1, sum, s));
            unsigned long long h = 0;
            HIPCHK(hipMemcpyAsync(&h, sum, sizeof(h), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            float ms_t = 0.f;
            HIPCHK(hipEventElapsedTime(&ms_t, e0, e1));
            if (k == 0) ref = h;
            else if (h != ref) {
                rc = MICX_EDEVICE;   // a launch shape changed the results: keep the rules
                break;
            }
            if (ms_t < best_ms) {
                best_ms = ms_t;
                best.T = p.T;
                best.nlcap = p.NL;
                best.wgs = cands[k].tv.wgs > 0 ? cands[k].tv.wgs : ((p.T == 1 && p.NL >= 14) ? 4 : 2);
            }
        }
        if (rc == MICX_OK)
            tune_set(tune_key(p0.fx, n, yi + 2, hg.xcnt[yi], hg.khat[yi]), best);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    RETCHK(rc);
    // captured graphs hold the old launch shapes
    drop_graph(ctx);
    ctx->gseen = false;
    if (cache_path) return micx_tune_save(cache_path);
    return MICX_OK;
}

extern "C" int micx_tune_save(const char *path) {
    if (!path) return MICX_EINVAL;
    FILE *f = fopen(path, "w");
    if (!f) return MICX_EINVAL;
    fprintf(f, "micx-tune 1 gfx950\n");
    const int cnt = tune_count();
    for (int i = 0; i < cnt; i++) {
        DpTuneKey k;
        DpTune v;
        tune_entry(i, k, v);
        fprintf(f, "%d %d %d %d %d %d %d %d\n", k.fx, k.nb, k.y, k.x, k.khb, v.T, v.nlcap, v.wgs);
    }
    fclose(f);
    return MICX_OK;
}

extern "C" int micx_tune_load(const char *path) {
    if (!path) return MICX_EINVAL;
    FILE *f = fopen(path, "r");
    if (!f) return MICX_EINVAL;
    char tag[32], arch[32];
    int ver = 0;
    if (fscanf(f, "%31s %d %31s", tag, &ver, arch) != 3 || strcmp(tag, "micx-tune") != 0 || ver != 1 ||
        strcmp(arch, "gfx950") != 0) {
        fclose(f);
        return MICX_EINVAL;
    }
    DpTuneKey k;
    DpTune v;
    while (fscanf(f, "%d %d %d %d %d %d %d %d", &k.fx, &k.nb, &k.y, &k.x, &k.khb, &v.T, &v.nlcap, &v.wgs) == 8)
        tune_set(k, v);
    fclose(f);
    return MICX_OK;
}

extern "C" int micx_tune_clear(void) {
    tune_clear();
    return MICX_OK;
}
