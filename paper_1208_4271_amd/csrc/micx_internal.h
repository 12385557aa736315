// micx_internal.h -- launch interface between the C ABI layer (micx_api.hip)
// and the device kernels (micx_kernels.hip).  Not installed; not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "micx.h"

namespace micx {

// Per-dataset ranking tables (one row of n entries per variable).
struct RankTables {
    int m = 0, n = 0;
    int *perm = nullptr;    // [v][i]: sample index at sorted position i
    int *gsize = nullptr;   // [v][p]: tie-group size at group-start position p, else 0
    int *grank = nullptr;   // [v][j]: sorted position of the start of sample j's tie group
};

// Per-(variable, row count) equipartition tables.
struct EquipTables {
    int NY = 0;             // number of row counts: y = 2 .. NY+1
    int NYP = 0;            // NY rounded up to a multiple of 8 (16-byte rows of rowof)
    uint16_t *rowof = nullptr;  // [v][p][y-2], NYP per p: 0-based row of the tie group starting at p
    int *yhat = nullptr;        // [v][y-2]: rows produced
    int *rowstart = nullptr;    // [v][y-2][r]: start position of row r (r = 0..yhat), may be null
    int RS = 0;                 // stride of rowstart per (v, y): NY + 2
    int compat = 0;             // MICX_COMPAT_* flags
};

// Grid geometry of one (n, alpha, c) configuration, computed on the host.
struct Geometry {
    int n = 0, B = 0, NY = 0, W = 0;   // NY = floor(B/2) - 1 row counts; W = NY
    int xmax = 0;                      // largest column count, floor(B/2)
    // per y-2 (device arrays):
    int *xcnt = nullptr;   // x(y) = floor(B/y)
    int *khat = nullptr;   // min(floor(c * x(y)), n)
    int *koff = nullptr;   // offsets of per-item end buffers inside one (pair, orientation)
    int *aoff = nullptr;   // offsets of per-item score rows inside one (pair, orientation)
    int KSUM = 0, ASUM = 0, KMAX = 0, KYMAX = 0;   // sums and maxima over y
    const int *khat_host = nullptr;                // khat per y-2 (host copy)
    int compat = 0;                                // MICX_COMPAT_* flags
};

// A launch-shape choice for one DP class, made by the autotuner
// (micx_autotune): targets per lane, cap on the layers per pass, workgroups
// per CU that the LDS split aims for.  0 leaves a field to the default rule.
struct DpTune {
    int T = 0, nlcap = 0, wgs = 0;
};
// Classes are keyed by their numeric form, n rounded up to a power of two,
// y, x and khat rounded up to a power of two.
struct DpTuneKey {
    int fx = 0, nb = 0, y = 0, x = 0, khb = 0;
};
DpTuneKey tune_key(bool fx, int n, int y, int x, int khat);
// Process-wide table of tuned choices (fixed size, no heap).
void tune_set(const DpTuneKey &k, const DpTune &v);
bool tune_get(const DpTuneKey &k, DpTune &v);
void tune_clear();
// The i-th entry (i < tune_count()), for saving.
int tune_count();
void tune_entry(int i, DpTuneKey &k, DpTune &v);

// Launch shape of the DP for one row count y.
struct DpPlan {
    bool fx = false;              // 32-bit fixed-point DP (else FP64)
    double scale = 0.0;           // fixed-point scale S
    double bound = 0.0;           // bound on |dM| of the fixed-point form for this class
    int NL = 0, YR = 0, T = 0;    // kernel template: layers per pass, rows in registers, targets per lane
    int x = 0, KS = 0, RS = 0;    // columns, G-table row stride, count-record stride
    int SB = 0, WPB = 0;          // sources staged per block, wavefronts per workgroup
    int lds = 0, lds_L = 0, lds_stage = 0, lds_wave = 0;
    int blocks_per_cu = 0, max_waves = 0;
    size_t slot_bytes = 0;        // G table bytes per wavefront
    bool groups = false;          // launched over batch-stream item descriptors
    int wgs = 0;                  // workgroups per CU the LDS split aims for (0: default rule)
    bool co = false;              // cooperative: one item per workgroup of WPB waves
    int lds_rec = 0, lds_flags = 0;   // cooperative: shared count records and superclump flags
};

// Per-batch item buffers.
struct ItemBuffers {
    int *cbuf = nullptr;   // clump ends, capacity khat per item
    int *sbuf = nullptr;   // superclump ends, capacity khat per item
    int *K = nullptr;      // (super)clumps used by the DP
    int *k = nullptr;      // clumps before merging
    int *src = nullptr;    // 0: DP columns are the clumps (cbuf), 1: the superclumps (sbuf)
    int *Yh = nullptr;     // rows yhat of the item's row variable (equipartition result)
    // Row labels of every point in column order, per (pair, orientation) and
    // row count: [item][y-2][p], lab_row bytes per row (n rounded up to 64
    // entries), one byte per label, two when some row count exceeds 255.
    unsigned char *lab = nullptr;
    size_t lab_row = 0;
    int lab16 = 0;
    double *A = nullptr;   // normalised scores, ASUM per (pair, orientation)
};

// Near-tie recheck of the 32-bit form.  Its entries are within a bound of
// the FP64 ones, which keeps MIC, MAS and MEV within tolerance but can change
// which cell MCN selects when cells lie within that bound of MIC (exact ties
// above all, which rounding at different fixed-point scales splits).  The
// statistics kernel flags such a pair and queues the items behind every cell
// within `band` of its MIC, per row count, for an FP64 re-run of their DP;
// the flagged pairs' statistics are then computed again.
struct Recheck {
    double band = 0.0;          // twice the largest entry bound plus the MCN slack; 0: no flags
    unsigned *iflag = nullptr;  // [pair*2+orientation][nyw]: one bit per row count, item queued
    int nyw = 0;                // 32-bit words per (pair, orientation)
    int *ilist = nullptr;       // queued items as descriptors (0, y-2, pair*2+orientation)
    int *icount = nullptr;      // number of queued items
    int *plist = nullptr;       // flagged pairs (batch-local index)
    int *pcount = nullptr;      // number of flagged pairs
};

// Pair source for a batch: either an explicit list (pairs != null) or the
// row-major upper triangle starting at global pair index p0.
struct PairSource {
    const int32_t *pairs = nullptr;   // device, 2 ints per pair
    int64_t p0 = 0;
    int m = 0;
};

// End slots of one row count inside a (pair, orientation)'s clump and
// superclump end buffers: khat rounded up to a multiple of four, so that every
// item's buffer starts on 16 bytes and the partition kernel can store its
// ends four at a time.
__host__ __device__ constexpr int end_slots(int khat) { return (khat + 3) & ~3; }

// Ints per superclump record of the DP's count table: e_t, then the rows'
// cumulative counts.  YR rows when the kernel keeps them in registers, else
// all y rows.  Padded to a multiple of four so that a record reads as 16-byte
// vectors (the padding holds zeros), except for YR = 2 and 4: records of 3
// ints gain nothing from vectors, and padding 5 to 8 cost the benchmark's
// y = 4 class a workgroup per CU (measured +11%).
__host__ __device__ constexpr bool rec_vector(int YR) { return YR != 2 && YR != 4; }
__host__ __device__ inline int rec_stride(int YR, int y) {
    if (YR > 0 && !rec_vector(YR)) return YR + 1;
    return ((YR > 0 ? YR : y) + 4) & ~3;
}

// One group of a batch stream on the device (pairs sharing n, alpha and c):
// its geometry and item buffers, for DP launches that mix groups.  The
// group's variables are rows 2i and 2i+1 for its pair i.
struct DpGroup {
    int n = 0, NY = 0, KSUM = 0, ASUM = 0, lab16 = 0, pad = 0;
    size_t lab_row = 0;
    const int *xcnt = nullptr, *khat = nullptr, *koff = nullptr, *aoff = nullptr;
    const int *Yh = nullptr;     // yhat per item
    const int *cbuf = nullptr, *sbuf = nullptr, *K = nullptr, *src = nullptr;
    const unsigned char *lab = nullptr;
    double *A = nullptr;
};

// One group of a batch pass for the per-group stages run as single launches
// over all groups (gather, rank, equipartition, partition, statistics).
struct GroupDev {
    int n = 0, NY = 0, NYP = 0, KSUM = 0, ASUM = 0, B = 0, W = 0, nv = 0, npairs = 0, lab16 = 0;
    size_t lab_row = 0;
    const int64_t *offs = nullptr;   // element offset of each variable in the packed data
    void *X = nullptr;               // gathered variables, nv x n
    int *perm = nullptr, *gsize = nullptr, *grank = nullptr;
    uint16_t *rowof = nullptr;
    int *yhat = nullptr;
    const int *xcnt = nullptr, *khat = nullptr, *koff = nullptr, *aoff = nullptr;
    int *cbuf = nullptr, *sbuf = nullptr, *K = nullptr, *k = nullptr, *src = nullptr, *Yh = nullptr;
    unsigned char *lab = nullptr;
    double *A = nullptr;
    const int32_t *pairs = nullptr;  // (2i, 2i+1) per pair
    double *out = nullptr;           // 4 doubles per pair
    int compat = 0;                  // MICX_COMPAT_* flags
    // near-tie recheck (see Recheck): one bit per (pair*2+orientation, y-2)
    // item, nyw words per (pair, orientation), and the FP64 recheck launch of
    // each row count (keyof[y-2])
    unsigned *iflag = nullptr;
    int nyw = 0;
    const int *keyof = nullptr;
};

// Near-tie recheck of a batch stream pass: per FP64 launch key k, the queued
// items (3 ints each: group, y-2, pair*2+orientation) at klist + 3*koff[k],
// kcount[k] of them; the flagged pairs as (group, pair) at plist, pcount of
// them.  band as in Recheck.
struct StreamRecheck {
    double band = 0.0;
    int *klist = nullptr;
    const int *koff = nullptr;
    int *kcount = nullptr;
    int *plist = nullptr;
    int *pcount = nullptr;
};

// Fused per-group stages: map[b] = (group, index of the block inside the
// group's own launch of that stage).
hipError_t launch_gather_g(const void *data, int esize, const GroupDev *G, const int2 *map, int blocks,
                           hipStream_t s);
hipError_t launch_rank_g(const GroupDev *G, const int2 *map, int blocks, int nmax, int dtype,
                         int *status, hipStream_t s);
hipError_t launch_equip_g(const GroupDev *G, const int2 *map, int blocks, int nmax, hipStream_t s);
hipError_t launch_part_g(const GroupDev *G, const int2 *map, int blocks, hipStream_t s);
hipError_t launch_stats_g(const GroupDev *G, const int2 *map, int blocks, hipStream_t s,
                          const StreamRecheck *flag = nullptr, const int *status = nullptr);
// statistics again for the flagged pairs of a pass (after the FP64 recheck)
hipError_t launch_stats_g_list(const GroupDev *G, const int *plist, const int *pcount, int cap,
                               hipStream_t s, const int *status = nullptr);


hipError_t launch_pearson(const void *X, int dtype, int m, int n, PairSource ps, int npairs,
                          double *mean, double *inorm, const double *stats, double *out, hipStream_t s);
hipError_t launch_rank(const void *X, int dtype, int m, int n, RankTables &rt, int *status,
                       hipStream_t s);
hipError_t launch_equip(const RankTables &rt, EquipTables &et, hipStream_t s);
hipError_t launch_part(const RankTables &rt, const EquipTables &et, const Geometry &g,
                       PairSource ps, int npairs, ItemBuffers &ib, hipStream_t s);
DpPlan dp_plan(const Geometry &g, int n, int yi, int cus, int mode, double tol);
// without the LDS split; nl_max caps the layers per pass; force (may be
// null) overrides the tuned table and the default rule
DpPlan dp_shape(const Geometry &g, int n, int yi, int mode, double tol, int nl_max = 36,
                const DpTune *force = nullptr, bool gr = false);
// The 32-bit form's a-priori bound on |dM| for the entries M[l][y], l <= x,
// at fixed-point scale S (rows yhat <= y, at least two; see micx_dp.hip).
double dp32_bound(int n, int x, int y, double scale);
// Every row count's DP item fits one CU's LDS (shapes by the tuned choices,
// or by `force` when given).
bool dp_fits(const Geometry &g, int n, const DpTune *force = nullptr);
void dp_fit_lds(DpPlan &p, int nmax, size_t rec_bytes, int cus);
// DP over items of several groups (see DpGroup): gitems holds 3 ints per item
// (group, y-2, pair*2+orientation); the plan's shape, scale and LDS split
// cover every item; scratch holds min(nitems, p.max_waves) G tables of
// p.slot_bytes.
// icount (device, may be null): only the first min(nitems, *icount) items.
hipError_t launch_dp_items(const DpGroup *groups, const int *gitems, int nitems, int nmax,
                           const double *xlogx, const uint32_t *fxtab, void *scratch,
                           const DpPlan &p, int compat, hipStream_t s, const int *icount = nullptr,
                           int *status = nullptr);
// Item descriptors (0, y-2, pair*2+orientation) of row counts yi_lo ..
// yi_lo+ncls-1, npo items each, class by class (a kernel).
hipError_t launch_range_items(int yi_lo, int ncls, int npo, int *items, hipStream_t s);
// Adds the bit patterns of one row count's entries (all items of a batch) to
// *sum (the autotuner's determinism check).
hipError_t launch_checksum(const double *A, int npo, int ASUM, int off, int cnt, unsigned long long *sum,
                           hipStream_t s);
// Writes one DpGroup into device memory (a kernel, so that captured graphs
// hold no host copies).
hipError_t launch_put_group(const DpGroup &g, DpGroup *dst, hipStream_t s);
// Fixed-point cost tables of several row-count classes in one launch:
// tab + cls[i] * stride gets round(scale[i] * j ln j), j = 0..n.
constexpr int kFxBatch = 64;
struct FxScales {
    double scale[kFxBatch];
    int cls[kFxBatch];
};
hipError_t launch_fxtables(int n, const FxScales &sc, int count, const double *xlogx, uint32_t *tab,
                           size_t stride, hipStream_t s);
hipError_t launch_fxtable(int n, const DpPlan &p, const double *xlogx, uint32_t *tab,
                          hipStream_t s);
// Cooperative DP instances: chunk completion flags per item (chunks of 64T
// targets, K <= MICX_MAX_N) and the bytes of the shared flags, per-wave
// minima and abort flag.
constexpr int kCoChunks = 128;
// Row-count classes whose items hold at least this many superclump slots
// (khat + 1) may run cooperatively, one item per workgroup: their one-wave
// time would otherwise bound a whole launch (batch stream) or leave a CU's
// LDS to a wave or two (all pairs at large n and alpha).
constexpr int kCoopMinK = 1024;
constexpr int kCoMeta = 4 * kCoChunks + 8 * 16 + 16;
// Cooperative DP (one item per workgroup) for the largest stream items:
// whether the shape has a cooperative instance, and its LDS split (WPB waves
// per workgroup, shared records of rec_bytes); launch_dp_items then runs it
// (status: the call's status word, bit 1 on a wait that gave up).
bool dp_co_built(bool fx, int NL, int YR, int T);
bool dp_fit_lds_co(DpPlan &p, int nmax, size_t rec_bytes, int cus);
// Debug instances of the DP kernel: the count tables of the two items of
// class yi of one pair, from both count scans (see micx_debug_tables).
hipError_t launch_dp_debug(const RankTables &rt, const EquipTables &et, const Geometry &g, PairSource ps,
                           const ItemBuffers &ib, const double *xlogx, int yi, int cus, int *out,
                           hipStream_t s);
// ilist/icount (device, may be null): run only the items ilist[0..*icount)
// (pair*2+orientation) of the class, at most `cap` of them.
hipError_t launch_dp(const RankTables &rt, const EquipTables &et, const Geometry &g,
                     PairSource ps, int npairs, const ItemBuffers &ib, const double *xlogx,
                     const uint32_t *fxtab, void *scratch, int yi, const DpPlan &p,
                     hipStream_t s, const int *ilist = nullptr, const int *icount = nullptr,
                     int cap = 0);
// Statistics of a batch.  flag (may be null): queue near-tied pairs and
// their items for the FP64 recheck.  plist/pcount (device, may be null): only
// the pairs plist[0..*pcount).  status (device, may be null): nothing is
// written while the call's status word is set.
hipError_t launch_stats(const Geometry &g, int npairs, const ItemBuffers &ib, double *out,
                        double *M, double *Axy, double *Ayx, hipStream_t s,
                        const Recheck *flag = nullptr, const int *plist = nullptr,
                        const int *pcount = nullptr, const int *status = nullptr);
// Clears nwords 32-bit words (a kernel, so that captured graphs hold no
// memset nodes).
hipError_t launch_zero(void *p, size_t nwords, hipStream_t s);
hipError_t launch_xlogx(int n, double *xlogx, hipStream_t s);
// Grid geometry of (n, B, c) into geo (4 NY ints: xcnt | khat | koff | aoff),
// computed on the device with the host's arithmetic; B already lowered by
// MICX_COMPAT_BOUND_STRICT.
hipError_t launch_geometry(int n, int B, double c, int compat, int NY, int *geo, hipStream_t s);
hipError_t launch_gather(const void *src, int esize, const int64_t *offs, int nv, int n, void *dst,
                         hipStream_t s);
// status (device, may be null): nothing is written while *status != 0
hipError_t launch_scatter_rows(const double *src, const int64_t *idx, int64_t rows, double *dst,
                               hipStream_t s, const int *status = nullptr);
// Accumulates the algorithmic work of a batch into counters[0..3]
// (items, dp_cells, h_evals, h_terms).
hipError_t launch_work(const EquipTables &et, const Geometry &g, PairSource ps, int npairs,
                       const ItemBuffers &ib, unsigned long long *counters, hipStream_t s);

int device_cus(int device);
// Sets a kernel's dynamic-LDS limit to the whole 160 KB, once per kernel and
// device.
hipError_t ensure_lds_attr(const void *k);

// A context's device, compute units, compatibility flags and DP32 tolerance.
void ctx_params(const micx_ctx *ctx, int *device, int *cus, int *compat, double *tol);
// Resolves the no-allocation scratch array's address on `device` (current).
int noalloc_init(int device);

}  // namespace micx
