/*
 * micx.h -- C ABI of the MI355X (gfx950) engine for the MINE statistics.
 *
 * The engine computes, for pairs of variables, the approximate
 * characteristic matrix M of the MINE family and the four statistics MIC,
 * MAS, MEV and MCN derived from it, following Albanese et al. 2012 ("minerva
 * and minepy: a C engine for the MINE suite", arXiv:1208.4271): its
 * Appendix A (implementation details, items 1-10), Algorithm 1
 * (GetClumpsPartition), Algorithm 2 (GetSuperclumpsPartition) and Sec. 2C
 * (grid bound B(n) = n^alpha).  The paper's engine exposes a dataset
 * structure, a parameter structure (alpha, c) and a returned score
 * structure from which four functions compute the statistics (Sec. 2,
 * "The MINE C engine and its wrappers"); this header keeps that shape and
 * adds an all-pairs call on an m x n matrix held in device memory.
 *
 * Every step of the computation runs in HIP kernels on the GPU.  Host code
 * only validates arguments, sizes the workspace and launches kernels.
 *
 * Conventions
 *  - Return codes: MICX_OK (0) or a negative MICX_E* code; micx_strerror()
 *    gives its message.  On error, outputs are left untouched.
 *  - Grid bound: B = floor(pow(n, alpha)) evaluated in FP64 on the host;
 *    cells (x, y) obey x, y >= 2 and x*y <= B (Appendix A item 1).  W =
 *    floor(B/2) - 1 is the side of the dense matrix layout used below.
 *  - Matrix layout: M[(y-2)*W + (x-2)] = M_{x,y}, the score of grids with x
 *    bins of the FIRST variable and y bins of the SECOND; entries with
 *    x*y > B are NaN.
 *  - Statistics: MIC = max M; MAS = max |M_{x,y} - M_{y,x}|; MEV = max of
 *    M over x = 2 or y = 2; MCN = min log2(x*y) over cells with
 *    M >= (1-eps) MIC (Appendix A item 2 sets eps = 0 and log base 2; the
 *    engine compares with an absolute slack of 1e-12).
 *  - Sample size: 2 <= n <= MICX_MAX_N.  Values must be finite.
 *  - Device: every call runs on the device the context was created for.
 */
#ifndef MICX_H
#define MICX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define MICX_OK           0
#define MICX_EINVAL      -1   /* bad argument: alpha not in (0,1], c <= 0, null pointer, m < 2, n < 2, bad dtype/mode */
#define MICX_ESMALLN     -2   /* floor(n^alpha) < 4: no grid cell exists */
#define MICX_ENONFINITE  -3   /* NaN or infinity in the input */
#define MICX_ENOMEM      -4   /* device or host allocation failed */
#define MICX_EDEVICE     -5   /* HIP runtime error or device status word set */
#define MICX_ETOOBIG     -6   /* n > MICX_MAX_N, or a DP item larger than one CU's LDS (large n with large alpha) */

/* Largest sample size: ranking sorts one variable inside one workgroup's LDS. */
#define MICX_MAX_N 8192

/* Element types of input matrices. */
#define MICX_F32 0
#define MICX_F64 1
#define MICX_I32 2

/* Numeric forms of the dynamic program (integer stages are identical).
 * MICX_MODE_DP32 runs the DP in 32-bit fixed point: column costs are scaled
 * by S and rounded through a table (T[j] = round(S j ln j)), sums are exact
 * integer arithmetic, and every matrix entry M[l][y] is then within
 * l (yhat+1) / (2 S n ln min(l, yhat)) of the exact one, S ~ 2^32 / (n ln y).
 * The library bounds that per row count y by its largest value over
 * 2 <= l <= x(y), 2 <= yhat <= y.  Row counts whose bound exceeds the tolerance (see
 * micx_set_dp32_tolerance, default 5e-7) run in FP64.  Scores, the
 * H(Q) term and all statistics are computed in FP64 in both forms. */
#define MICX_MODE_FP64  0   /* DP in FP64 */
#define MICX_MODE_DP32  1   /* DP in 32-bit fixed point with a per-class error bound, FP64 elsewhere */

/* Compatibility variants of readings the paper leaves open (micx_set_compat;
 * default 0 = the readings this library takes).  Each reproduces a variant
 * the paper discusses:
 *   TIE_STRICT     EquipartitionYAxis closes a row on '>' instead of '>='
 *                  (App. A item 3 with a strict comparison);
 *   DESIRED_INT    the desired row size is cast to an integer (App. A
 *                  item 3's integer variable);
 *   COMBINE_INDEX  the two orientations are combined at equal
 *                  (equipartitioned, optimised) index, not equal grid shape;
 *   NORM_BY_Y      entries are normalised by ln min(x, y), the requested
 *                  rows, instead of ln min(x, yhat) (App. A item 4);
 *   BOUND_STRICT   cells satisfy xy < B instead of xy <= B (App. A item 1);
 *   KHAT_PLUS1     up to khat + 1 superclumps (App. A item 7's behaviour). */
#define MICX_COMPAT_TIE_STRICT     1
#define MICX_COMPAT_DESIRED_INT    2
#define MICX_COMPAT_COMBINE_INDEX  4
#define MICX_COMPAT_NORM_BY_Y      8
#define MICX_COMPAT_BOUND_STRICT  16
#define MICX_COMPAT_KHAT_PLUS1    32

/* Opaque context: device, workspace, cached tables and launch graphs. */
typedef struct micx_ctx micx_ctx;

/* The dataset of one pair (the paper's dataset structure): n samples of two
 * variables, HOST arrays of n doubles owned by the caller. */
typedef struct {
    int n;
    const double *x;
    const double *y;
} micx_problem;

/* The parameters of the method (the paper's parameter structure, Sec. 2):
 * alpha sets the grid bound B = n^alpha (Sec. 2C), c the superclump bound
 * khat = c x (Algorithm 2).  Defaults 0.6 and 15 (the paper's usage
 * example). */
typedef struct {
    double alpha;
    double c;
} micx_param;
#define MICX_ALPHA_DEFAULT 0.6
#define MICX_C_DEFAULT 15.0

/* Score of one pair: the characteristic matrix (the paper's score structure). */
typedef struct {
    int n;            /* sample size */
    int B;            /* largest cell count xy: floor(n^alpha) (minus 1 with MICX_COMPAT_BOUND_STRICT) */
    int W;            /* matrix side, floor(B/2) - 1 */
    double *M;        /* W*W doubles, M[(y-2)*W + (x-2)] = M_{x,y}; NaN where x*y > B */
    double *Axy;      /* W*W: first variable into l columns (DP), second equipartitioned into r rows: Axy[(r-2)*W + (l-2)] */
    double *Ayx;      /* W*W: second variable into l columns (DP), first equipartitioned into r rows */
    double stats[4];  /* MIC, MAS, MEV, MCN (eps = 0), computed on the device */
} micx_score;

/* Create a context on HIP device `device`.  *ctx receives the handle. */
int micx_ctx_create(micx_ctx **ctx, int device);

/* Release a context and its workspace.  NULL is ignored. */
void micx_ctx_destroy(micx_ctx *ctx);

/* Parameter check (the paper's engine validates its parameter structure and
 * reports a message, Sec. 2 and the usage example).  Returns NULL when
 * param is non-null, 0 < alpha <= 1 and c > 0, else a static message. */
const char *micx_check_param(const micx_param *param);

/* Grid bound floor(pow(n, alpha)) in FP64 (Sec. 2C; Appendix A item 1). */
int micx_grid_bound(int n, double alpha);

/* Score of one pair: the paper's score function on its dataset and
 * parameter structures (Sec. 2; Appendix A items 1-10 for what it computes).
 * problem: the pair (host arrays).  mode: MICX_MODE_*.
 * *out receives a newly allocated score owned by the caller; release it
 * with micx_free_score().  Synchronous: returns once the score is on the
 * host, with MICX_ENONFINITE for NaN or infinite input. */
int micx_compute_score(micx_ctx *ctx, const micx_problem *problem, const micx_param *param, int mode,
                       micx_score **out);

/* The four statistics of a score (the paper's four statistic functions). */
double micx_mic(const micx_score *s);
double micx_mas(const micx_score *s);
double micx_mev(const micx_score *s);
double micx_mcn(const micx_score *s, double eps);

/* Free a score returned by micx_compute_score().  NULL is ignored. */
void micx_free_score(micx_score *s);

/* All pairs of rows of X: the all-pairs mode of the paper's engine (Sec. 2;
 * the mine application's default mode), each pair scored as by
 * micx_compute_score.
 * X_dev: DEVICE pointer to an m x n row-major matrix (one variable per row,
 *        n samples contiguous) of element type dtype (MICX_F32/F64/I32);
 *        owned by the caller, read only until the work completes.
 * out_dev: DEVICE pointer to m(m-1)/2 * 4 doubles owned by the caller; pair
 *        (i < j) is written at index p = i*m - i*(i+1)/2 + (j-i-1) as
 *        (MIC, MAS, MEV, MCN), with the first variable i and the second j.
 * stream: hipStream_t (as void*), or NULL for the null stream.
 * mode: MICX_MODE_*.
 * Asynchronous: the work is queued on stream and the call returns without
 * waiting for it.  Argument errors are returned at once; errors the device
 * finds (NaN or infinity in X) are returned by micx_status(), and out_dev
 * is then left untouched.  With launch graphs on (micx_set_graphs, the
 * default), the second call with the same arguments captures the work into
 * a HIP graph and later ones replay it. */
int micx_allpairs(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n, const micx_param *param,
                  int mode, double *out_dev, void *stream);

/* Waits for the work of the last pair call on ctx (micx_allpairs,
 * micx_pairs, micx_batch, micx_pearson) and returns its device-side result:
 * MICX_OK, MICX_ENONFINITE (NaN or infinity in the input; outputs untouched)
 * or MICX_EDEVICE.  A call's result holds until the next call. */
int micx_status(micx_ctx *ctx);

/* Launch graphs for micx_allpairs (1 = on, the default; 0 = every call
 * launches its kernels one by one).  Cached graphs are dropped when the
 * context's workspace grows. */
int micx_set_graphs(micx_ctx *ctx, int enable);

/* Listed pairs of rows of X: the paper's "master variable" (one variable
 * against all others) and single-pair modes of its mine application
 * (Sec. 2) are lists of this kind.
 * pairs_host: HOST array of npairs (i, j) int32 index pairs, 0 <= i, j < m,
 *        i != j (copied before the call returns); out_dev: DEVICE pointer to
 *        npairs * 4 doubles, pair k written at 4k as (MIC, MAS, MEV, MCN)
 *        with i the first variable.
 * Asynchronous, as micx_allpairs (results of the device: micx_status). */
int micx_pairs(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n,
               const int32_t *pairs_host, int64_t npairs, const micx_param *param, int mode,
               double *out_dev, void *stream);

/* Pearson's correlation coefficient rho and the non-linearity index
 * MIC - rho^2 of pairs of rows of X: the two statistics the paper's engine
 * reports beside the four MINE statistics (Sec. 2 and Fig. 1; the
 * Performance experiments of the supplement time all six together).
 * X_dev: DEVICE pointer, m x n row-major, dtype MICX_F32/F64/I32, as for
 *        micx_allpairs; m >= 2, n >= 2.
 * pairs_host: HOST array of npairs (i, j) int32 pairs (0 <= i, j < m), or
 *        NULL for all pairs i < j in micx_allpairs order, with npairs then
 *        equal to m(m-1)/2 (at most 2^31 - 1 pairs).
 * stats_dev: DEVICE pointer to the 4-double MINE records of the same pairs in
 *        the same order (micx_allpairs or micx_pairs output), or NULL.
 * out_dev: DEVICE pointer to npairs * 2 doubles, pair k at 2k as
 *        (rho, MIC - rho^2).  rho is NaN when either variable is constant; the
 *        index is NaN when rho is NaN or stats_dev is NULL.
 * FP64: per variable the mean, then the centred sum of squares; per pair one
 * centred dot product, rho clamped to [-1, 1].  Errors: MICX_EINVAL (null
 * pointer, bad sizes, dtype or pair index, npairs mismatch), MICX_EDEVICE.
 * Asynchronous, as micx_allpairs (pairs_host is copied before the call
 * returns). */
int micx_pearson(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n,
                 const int32_t *pairs_host, int64_t npairs, const double *stats_dev,
                 double *out_dev, void *stream);

/* One independent pair of a batch: both variables are n consecutive
 * elements of the packed data buffer, at element offsets off_x and off_y;
 * alpha and c are the pair's own parameters. */
typedef struct {
    int64_t off_x;
    int64_t off_y;
    int32_t n;
    int32_t reserved;     /* set to 0 */
    double alpha;
    double c;
} micx_pair_desc;

/* A stream of independent pairs of uneven n and uneven (alpha, c), each
 * scored as by micx_compute_score on its own two variables (the pair-level
 * parallelism of the paper's multi-core and MPI drivers, Sec. 2A-2B, on one
 * device).
 * data_dev: DEVICE pointer to the packed variables, element type dtype
 *        (MICX_F32/F64/I32), owned by the caller, read only.
 * pairs_host: HOST array of npairs descriptors.  Every descriptor is checked
 *        before any work starts: n in [2, MICX_MAX_N], floor(n^alpha) >= 4,
 *        alpha in (0, 1], c > 0, offsets >= 0 (the caller guarantees that
 *        off + n lies inside data_dev).
 * out_dev: DEVICE pointer to npairs * 4 doubles owned by the caller; pair k
 *        is written at 4k as (MIC, MAS, MEV, MCN), x the first variable.
 *        On any error out_dev is left untouched.
 * Pairs that share (n, alpha, c) run together.  Asynchronous, as
 * micx_allpairs (pairs_host is read before the call returns; device-side
 * results: micx_status). */
int micx_batch(micx_ctx *ctx, const void *data_dev, int dtype, const micx_pair_desc *pairs_host,
               int64_t npairs, int mode, double *out_dev, void *stream);

/* Integer stages of one item, read back for bit-exact tests:
 * EquipartitionYAxis (App. A items 3-4), GetClumpsPartition (Algorithm 1)
 * and GetSuperclumpsPartition (Algorithm 2).
 * problem: the pair (host arrays).  orient 0: columns from x, rows from y;
 * orient 1: swapped.  ry: requested row count, 2 <= ry <= floor(B/2).
 * Outputs (host): *yhat rows produced; row_starts[0..yhat] positions (in
 * the row variable's sorted order) where each row starts, then n (caller
 * provides ry+1 ints); *k clumps; *K (super)clumps; ends[0..K-1] number of
 * points, in the column variable's order, up to and including each
 * (super)clump (caller provides n ints).  Synchronous. */
int micx_debug_item(micx_ctx *ctx, const micx_problem *problem, const micx_param *param, int orient,
                    int ry, int *yhat, int *row_starts, int *k, int *K, int *ends);

/* The ranks and the DP's cumulative count table of one item, read back for
 * bit-exact tests (App. A item 10a).
 * group_start_x, group_start_y: HOST arrays of n ints: for every sample, the
 *        position in its variable's sorted order where its tie group starts
 *        (the number of smaller values), as the rank kernel stores it.
 * counts: HOST array of (n+1)*ry ints (or NULL): counts[t*yhat + r] = points
 *        of the first t (super)clumps, in the column variable's order, that
 *        lie in row r, for t = 0..K and r = 0..yhat-1 -- the table the DP
 *        kernel builds in LDS, written out by a debug instance of it.
 * Same item selection as micx_debug_item.  Synchronous. */
int micx_debug_tables(micx_ctx *ctx, const micx_problem *problem, const micx_param *param, int orient,
                      int ry, int *group_start_x, int *group_start_y, int *counts);

/* Instrumentation of the pair calls (micx_allpairs, micx_pairs, micx_batch).
 * With profiling enabled, each call records HIP events on its stream around
 * every launch of the dynamic-program kernel and counts the algorithmic work
 * of its items from their actual sizes (K (super)clumps, yhat rows, x
 * columns).  Layers 2..x-1 are needed at every target and layer x only at
 * the last one, so dp_cells = sum (x-2) K(K+1)/2 + K (one add and one min
 * each); h_evals = sum of the column costs needed (K(K+1)/2 when x >= 3,
 * else 2K-1); h_terms = sum (yhat+1) h_evals table terms.
 * micx_get_profile() returns the totals of the last call. */
typedef struct {
    int64_t items;        /* (pair, orientation, y) items */
    int64_t dp_cells;     /* DP cell updates */
    int64_t h_evals;      /* column cost evaluations h(s,t) */
    int64_t h_terms;      /* x ln x table terms read by those evaluations */
    double dp_ms;         /* summed duration of the DP kernel launches (HIP events) */
    int dp_launches;      /* number of DP kernel launches */
    int dp32_classes;     /* row counts run in 32-bit fixed point (MICX_MODE_DP32) */
    int fp64_classes;     /* row counts run in FP64 */
    double dp32_bound;    /* largest |dM| bound among the fixed-point row counts */
    int64_t recheck_pairs; /* MICX_MODE_DP32: pairs whose MCN the 32-bit entries left open */
    int64_t recheck_items; /* items of those pairs re-run in FP64 */
    double recheck_ms;    /* duration of the FP64 re-runs and the statistics after them */
    int coop_classes;     /* (pair, row count) classes whose DP ran cooperatively (one
                           * item per workgroup); per row count for pair calls */
    double host_ms;       /* micx_batch: host time inside the call (grouping, launch
                           * planning, uploads and launches; the device work may
                           * still run when the call returns); 0 for other calls */
} micx_profile;

int micx_set_profiling(micx_ctx *ctx, int enable);
int micx_get_profile(micx_ctx *ctx, micx_profile *out);

/* Tolerance on |dM| for MICX_MODE_DP32 (default 5e-7, half of the 1e-6
 * agreement required of the scores): a row count whose
 * fixed-point bound exceeds it runs in FP64.  Returns MICX_EINVAL unless
 * tol > 0. */
int micx_set_dp32_tolerance(micx_ctx *ctx, double tol);

/* The a-priori bound on |dM| that MICX_MODE_DP32 guarantees for the entries
 * M[l][y], 2 <= l <= x, of one row count at sample count n, at that row
 * count's own scale S = floor(2^32 / (1.02 n ln y)): the largest
 * l (yhat+1) / (2 S n ln min(l, yhat)) over 2 <= l <= x and 2 <= yhat <= y.
 * Host arithmetic only (no device); 0 for x < 2, y < 2 or n < 1. */
double micx_dp32_bound(int n, int x, int y);

/* Compatibility flags (MICX_COMPAT_*, OR-ed) for every later call on ctx.
 * Returns MICX_EINVAL for unknown bits. */
int micx_set_compat(micx_ctx *ctx, int flags);

/* Autotuner of the DP launch shapes (the OptimizeXAxis speed-ups the paper
 * tunes for its engine, App. A item 10, picked by measurement on this
 * device).  For every row count of the (n, alpha, c, mode) problem, it times
 * each distinct launch shape -- targets per lane (1-3), cap on the layers
 * per pass (12-36), workgroups per CU the LDS split aims for (1, 2, 4) -- on
 * all pairs of the first min(m, 192) rows of X_dev, checks that every shape
 * gives bit-identical entries (else MICX_EDEVICE and no choice is kept),
 * and keeps the fastest in a process-wide table that later calls on any
 * context use for classes with the same key (numeric form, n rounded up to a
 * power of two, y, x, khat rounded up to a power of two).
 * cache_path: file the whole table is written to (micx_tune_save), or NULL.
 * Synchronous; takes seconds. */
int micx_autotune(micx_ctx *ctx, const void *X_dev, int dtype, int m, int n, const micx_param *param,
                  int mode, const char *cache_path, void *stream);
/* Write the tuned table to a text file / merge a file written by
 * micx_tune_save into it (MICX_EINVAL if unreadable or for another device
 * architecture) / empty it (later calls use the default rules). */
int micx_tune_save(const char *path);
int micx_tune_load(const char *path);
int micx_tune_clear(void);

/* Size of the device array behind micx_score_noalloc (per device, held
 * until the process ends). */
#define MICX_NOALLOC_BYTES (32u << 20)

/* micx_compute_score for callers that cannot allocate (code under HIP graph
 * capture, serving loops or harnesses that forbid allocation): the same
 * score of one pair, with inputs and outputs in device memory, and no
 * allocation of any kind -- every intermediate buffer lives in one
 * file-scope device array of MICX_NOALLOC_BYTES (32 MiB) per device.
 * x_dev, y_dev: DEVICE pointers to n elements each of type dtype
 *        (MICX_F32/F64/I32), read only.
 * stats_dev: DEVICE pointer to 4 doubles: MIC, MAS, MEV, MCN.
 * mats_dev: DEVICE pointer to 3*W*W doubles (M, then Axy, then Ayx, each laid
 *        out as in micx_score, W = floor(B/2) - 1), or NULL.
 * status_dev: DEVICE pointer to one int that receives the call's device-side
 *        result once its work completes (MICX_OK, or MICX_ENONFINITE for a
 *        NaN or infinity in the input, in which case stats_dev and mats_dev
 *        are left untouched), or NULL.
 * stream: hipStream_t (as void*) or NULL.  The work is queued on it and the
 *        call returns without waiting.  All calls on one device share its
 *        array, which keeps the last call's contents (each call clears what
 *        it needs first): calls that overlap on one device race, so order
 *        them (one stream, or events).
 * Errors found before any work is queued: MICX_EINVAL (null pointer, bad
 * alpha/c/mode/dtype, n < 2), MICX_ESMALLN, MICX_ETOOBIG (n > MICX_MAX_N, or
 * a problem whose buffers exceed MICX_NOALLOC_BYTES -- alpha = 0.6 fits up
 * to n = MICX_MAX_N), MICX_EDEVICE. */
int micx_score_noalloc(micx_ctx *ctx, const void *x_dev, const void *y_dev, int dtype, int n,
                       const micx_param *param, int mode, double *stats_dev, double *mats_dev,
                       int *status_dev, void *stream);

/* Message for a return code (static string). */
const char *micx_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* MICX_H */
