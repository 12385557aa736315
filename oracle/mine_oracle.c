/*
 * mine_oracle.c -- reference CPU implementation of the approximate
 * characteristic matrix and of the four MINE statistics (MIC, MAS, MEV, MCN).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the GPU
 * library is checked.  Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or constant with the GPU library, and the GPU library never calls it.
 *
 * It is deliberately plain and slow: FP64 throughout, libm log() on counts,
 * the paper's real-valued comparisons, every step in the order the method
 * states it.  Citations name the passages of Albanese et al. 2012, "minerva
 * and minepy: a C engine for the MINE suite and its R, Python and MATLAB
 * wrappers" (arXiv:1208.4271): its Appendix A ("Implementation Details",
 * items 1-10), Algorithm 1 (GetClumpsPartition), Algorithm 2
 * (GetSuperclumpsPartition), Fig. 2 (worked example) and Sec. 2C (B = n^alpha).
 * Steps the paper takes from Reshef et al. 2011 (Science, supplementary
 * material) without reproducing them -- EquipartitionYAxis, OptimizeXAxis,
 * the characteristic-matrix loop and the statistics' definitions -- are
 * restated here from their mathematics.
 *
 * Readings taken where the paper is silent or garbled (each is selectable by
 * a flag so that alternatives can be measured):
 *   - EquipartitionYAxis closes a row when adding the next tie group does not
 *     bring the row closer to its target: |a+s-d| >= |a-d| (flag
 *     ORC_TIE_STRICT switches to '>').  A row is never closed while empty.
 *   - Algorithm 1 relabels each x-tie group that spans two or more rows with
 *     ONE fresh label (the output Fig. 2 prints), not one label per point.
 *   - The DP is exact: it minimises the point-weighted conditional entropy
 *     of Q given the column, over partitions with at most l columns whose
 *     cuts lie on superclump boundaries.
 *   - Each orientation is normalised by ln min(l, yhat) with its own yhat
 *     (Appendix A item 4); M[x][y] is the larger of the two orientations'
 *     values for the same grid shape (x bins of the first variable, y bins
 *     of the second).
 *   - MCN takes eps = 0 and log base 2 (Appendix A item 2); "M = MIC" is
 *     tested as M >= MIC - 1e-12.
 *   - Grid bound: floor(pow(n, alpha)) in FP64 on the host libm; cells obey
 *     xy <= B (Appendix A item 1).
 *   - Degenerate cases: an entry whose min(l, yhat) < 2 is 0; a single
 *     column gives I = 0.
 *
 * Parity status: every function here is pinned by the tests (Fig. 2, the
 * paper's C++ example, brute-force enumeration of column partitions,
 * closed forms, invariances); see tests/test_oracle_pins.py.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Reading flags (bit mask).  0 = the readings listed above. */
#define ORC_TIE_STRICT      1   /* close rows on '>' instead of '>=' */
#define ORC_DESIRED_INT     2   /* integer-cast desiredRowSize (App. A item 3 alternative) */
#define ORC_COMBINE_INDEX   4   /* combine orientations at equal (equip, opt) index, not equal shape */
#define ORC_NORM_BY_Y       8   /* normalise by ln min(x, y) instead of ln min(x, yhat) */
#define ORC_BOUND_STRICT   16   /* cells with xy < B instead of xy <= B */
#define ORC_KHAT_PLUS1     32   /* allow khat+1 superclumps (App. A item 7 behaviour) */

#define ORC_MCN_TOL 1e-12

/* ---------------------------------------------------------------------- */
/* Grid bound B(n) = n^alpha (Sec. 2C; App. A item 1).                      */
/* ---------------------------------------------------------------------- */
int oracle_grid_bound(int n, double alpha)
{
    return (int) floor(pow((double) n, alpha));
}

/* Largest cell count allowed: xy <= B, or xy < B with the strict flag. */
static int cell_limit(int B, int flags)
{
    return (flags & ORC_BOUND_STRICT) ? B - 1 : B;
}

/* ---------------------------------------------------------------------- */
/* EquipartitionYAxis (App. A items 3-4; Fig. 2).                          */
/* v: values sorted ascending.  Points with equal value form one tie group */
/* and always share a row.  The greedy walks the groups in order; a row is */
/* closed before a group when the row is not empty and adding the group    */
/* would leave the row no closer to the desired size.  The desired size    */
/* starts at n/y and is reset, each time a new row opens at 1-based        */
/* position i, to (n-i+1)/(y-currRow+1).  q[i] receives the 0-based row.   */
/* Returns the number of rows actually produced (yhat <= y).               */
/* ---------------------------------------------------------------------- */
int oracle_equipartition(const double *v, int n, int y, int flags, int *q)
{
    int i = 0, row = 0;
    double a = 0.0;
    double desired = (double) n / (double) y;
    if (flags & ORC_DESIRED_INT) desired = (double) (int) desired;
    while (i < n) {
        int s = 1;
        while (i + s < n && v[i + s] == v[i]) s++;
        if (a != 0.0) {
            double after = fabs(a + s - desired), before = fabs(a - desired);
            int close = (flags & ORC_TIE_STRICT) ? (after > before) : (after >= before);
            if (close) {
                row++;
                a = 0.0;
                /* the group's first point is at 1-based position i+1 and the
                   new row is the (row+1)-th: (n-(i+1)+1) / (y-(row+1)+1) */
                desired = (double) (n - i) / (double) (y - row);
                if (flags & ORC_DESIRED_INT) desired = (double) (int) desired;
            }
        }
        for (int j = 0; j < s; j++) q[i + j] = row;
        a += s;
        i += s;
    }
    return n > 0 ? row + 1 : 0;
}

/* ---------------------------------------------------------------------- */
/* GetClumpsPartition (Algorithm 1, as its Fig. 2 output fixes it).        */
/* a: first coordinates sorted ascending; q: row of each point (same       */
/* order).  Each tie group of a whose points carry two or more distinct    */
/* rows receives one fresh label of its own; clumps are then the maximal   */
/* runs of equal labels.  p[i] receives the 0-based clump.  Returns k.     */
/* ---------------------------------------------------------------------- */
int oracle_clumps(const double *a, const int *q, int n, int *p)
{
    if (n <= 0) return 0;
    int *lab = (int *) malloc(sizeof(int) * (size_t) n);
    for (int i = 0; i < n; i++) lab[i] = q[i];
    int fresh = -1;                        /* rows are >= 0, fresh labels < 0 */
    int i = 0;
    while (i < n) {
        int s = 1, mixed = 0;
        while (i + s < n && a[i + s] == a[i]) {
            if (q[i + s] != q[i]) mixed = 1;
            s++;
        }
        if (s > 1 && mixed) {
            for (int j = 0; j < s; j++) lab[i + j] = fresh;
            fresh--;
        }
        i += s;
    }
    p[0] = 0;
    for (int j = 1; j < n; j++) p[j] = p[j - 1] + (lab[j] != lab[j - 1]);
    int k = p[n - 1] + 1;
    free(lab);
    return k;
}

/* ---------------------------------------------------------------------- */
/* GetSuperclumpsPartition (Algorithm 2; App. A items 6-7).                */
/* If the clumps outnumber khat, EquipartitionYAxis is run over the        */
/* sequence of clump labels (each clump one tie group) with khat rows, and */
/* consecutive clumps are merged accordingly.  Returns the number K of     */
/* (super)clumps; p[i] receives the 0-based (super)clump of point i.       */
/* *k_out (if not NULL) receives the number of clumps before merging.      */
/* ---------------------------------------------------------------------- */
int oracle_superclumps(const double *a, const int *q, int n, int khat, int flags,
                       int *p, int *k_out)
{
    int k = oracle_clumps(a, q, n, p);
    if (k_out) *k_out = k;
    int limit = khat + ((flags & ORC_KHAT_PLUS1) ? 1 : 0);
    if (k > limit) {
        double *d = (double *) malloc(sizeof(double) * (size_t) n);
        for (int i = 0; i < n; i++) d[i] = (double) p[i];
        int K = oracle_equipartition(d, n, limit, flags & (ORC_TIE_STRICT | ORC_DESIRED_INT), p);
        free(d);
        return K;
    }
    return k;
}

/* Superclump bound for cx columns: khat = floor(c * cx) (Algorithm 2's     */
/* \hat{k} = cx, App. A items 6-7), at least 1 so that c < 1/2 stays valid. */
static int khat_of(double c, int cx)
{
    int k = (int) floor(c * (double) cx);
    return k < 1 ? 1 : k;
}

/* ---------------------------------------------------------------------- */
/* OptimizeXAxis (App. A item 10).                                         */
/* Inputs, in first-coordinate order: col[i] = (super)clump of point i     */
/* (0..K-1, nondecreasing), row[i] = row of point i (0..yhat-1).           */
/* Item 10a: the count matrix of points per (column span, row), kept as    */
/* cumulative counts N[t][r] over the first t (super)clumps.               */
/* Item 10b: the entropy matrix over all column spans (s, t]: here         */
/* h(s,t) = sum_r n_r ln(m / n_r), m = points in the span, n_r = those in  */
/* row r -- the span's entropy H(<c_s,c_t>, Q) times its point count.      */
/* DP: G_1(t) = h(0,t); G_l(t) = min(G_{l-1}(t), min_{0<s<t} G_{l-1}(s) +  */
/* h(s,t)).  G_l(K)/n is the least H(Q|P) over partitions P into at most l */
/* columns whose cuts lie on (super)clump boundaries, so                   */
/* max I(P;Q) = H(Q) - G_l(K)/n.  The optimal partition is rebuilt by      */
/* backtracking (ties: keep the coarser option, then the smallest s) and   */
/* its mutual information is recomputed from the grid's counts as          */
/* H(Q) + H(P) - H(P,Q).                                                   */
/* I[l-2] receives that value (nats) for l = 2..x.  If cuts != NULL,       */
/* cuts[(l-2)*x + j] receives the j-th column end (as a point count) of    */
/* the chosen partition, 0 after its last column.                          */
/* ---------------------------------------------------------------------- */
static double span_cost(int m, int c)   /* c * ln(m / c), 0 when c == 0 */
{
    if (c <= 0) return 0.0;
    return (double) c * log((double) m / (double) c);
}

static double plogp(int c, int n)       /* -(c/n) ln(c/n), 0 when c == 0 */
{
    if (c <= 0) return 0.0;
    double p = (double) c / (double) n;
    return -p * log(p);
}

int oracle_optimize_x_axis(const int *col, const int *row, int n, int K, int yhat,
                           int x, double *I, int *cuts)
{
    if (x < 2 || K < 1 || yhat < 1) return -1;
    size_t K1 = (size_t) K + 1;
    int *e = (int *) calloc(K1, sizeof(int));
    int *N = (int *) calloc(K1 * (size_t) yhat, sizeof(int));
    for (int i = 0; i < n; i++) {
        e[col[i] + 1]++;
        N[(size_t) (col[i] + 1) * yhat + row[i]]++;
    }
    for (size_t t = 1; t <= (size_t) K; t++) {
        e[t] += e[t - 1];
        for (int r = 0; r < yhat; r++) N[t * yhat + r] += N[(t - 1) * yhat + r];
    }
    /* entropy matrix over spans (s, t], 0 <= s < t <= K */
    double *h = (double *) malloc(sizeof(double) * K1 * K1);
    for (size_t s = 0; s < (size_t) K; s++)
        for (size_t t = s + 1; t <= (size_t) K; t++) {
            int m = e[t] - e[s];
            double acc = 0.0;
            for (int r = 0; r < yhat; r++)
                acc += span_cost(m, N[t * yhat + r] - N[s * yhat + r]);
            h[s * K1 + t] = acc;
        }
    /* DP tables G[l][t], arg[l][t] (arg = -1: keep the (l-1)-column optimum) */
    double *G = (double *) malloc(sizeof(double) * (size_t) (x + 1) * K1);
    int *arg = (int *) malloc(sizeof(int) * (size_t) (x + 1) * K1);
    for (size_t t = 1; t <= (size_t) K; t++) { G[K1 + t] = h[t]; arg[K1 + t] = 0; }
    for (size_t l = 2; l <= (size_t) x; l++)
        for (size_t t = 1; t <= (size_t) K; t++) {
            double best = G[(l - 1) * K1 + t];
            int bs = -1;
            for (size_t s = 1; s < t; s++) {
                double c = G[(l - 1) * K1 + s] + h[s * K1 + t];
                if (c < best) { best = c; bs = (int) s; }
            }
            G[l * K1 + t] = best;
            arg[l * K1 + t] = bs;
        }
    double HQ = 0.0;
    for (int r = 0; r < yhat; r++) HQ += plogp(N[(size_t) K * yhat + r], n);
    int *ends = (int *) malloc(sizeof(int) * ((size_t) x + 1));
    for (int l = 2; l <= x; l++) {
        /* backtrack the optimal partition into at most l columns */
        int nc = 0, layer = l;
        size_t t = (size_t) K;
        while (t > 0) {
            if (layer == 1) { ends[nc++] = (int) t; break; }
            int a = arg[(size_t) layer * K1 + t];
            if (a < 0) { layer--; continue; }
            ends[nc++] = (int) t;
            t = (size_t) a;
            layer--;
        }
        for (int j = 0; j < nc / 2; j++) {
            int tmp = ends[j]; ends[j] = ends[nc - 1 - j]; ends[nc - 1 - j] = tmp;
        }
        /* mutual information of the grid (P_l, Q) from its counts */
        double HP = 0.0, HPQ = 0.0;
        int prev = 0;
        for (int j = 0; j < nc; j++) {
            int tt = ends[j];
            HP += plogp(e[tt] - e[prev], n);
            for (int r = 0; r < yhat; r++)
                HPQ += plogp(N[(size_t) tt * yhat + r] - N[(size_t) prev * yhat + r], n);
            prev = tt;
        }
        I[l - 2] = HQ + HP - HPQ;
        if (cuts) {
            for (int j = 0; j < x; j++) cuts[(size_t) (l - 2) * x + j] = 0;
            for (int j = 0; j < nc && j < x; j++) cuts[(size_t) (l - 2) * x + j] = e[ends[j]];
        }
    }
    free(ends); free(arg); free(G); free(h); free(N); free(e);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Sorting: indices by value (ties by index), a plain merge sort.          */
/* ---------------------------------------------------------------------- */
static void argsort(const double *v, int n, int *idx)
{
    int *tmp = (int *) malloc(sizeof(int) * (size_t) (n > 0 ? n : 1));
    for (int i = 0; i < n; i++) idx[i] = i;
    for (int w = 1; w < n; w *= 2) {
        for (int lo = 0; lo < n; lo += 2 * w) {
            int mid = lo + w < n ? lo + w : n, hi = lo + 2 * w < n ? lo + 2 * w : n;
            int i = lo, j = mid, o = lo;
            while (i < mid && j < hi) {
                int a = idx[i], b = idx[j];
                if (v[b] < v[a] || (v[b] == v[a] && b < a)) tmp[o++] = idx[j++];
                else tmp[o++] = idx[i++];
            }
            while (i < mid) tmp[o++] = idx[i++];
            while (j < hi) tmp[o++] = idx[j++];
        }
        memcpy(idx, tmp, sizeof(int) * (size_t) n);
    }
    free(tmp);
}

/* ---------------------------------------------------------------------- */
/* One orientation of the characteristic-matrix loop (App. A items 1, 4).  */
/* u is partitioned by the DP (columns), v is equipartitioned (rows).      */
/* For every ry = 2..floor(B/2) with cx = floor(B/ry):                     */
/*   Q <- EquipartitionYAxis(v, ry); P <- GetSuperclumpsPartition(u, Q,    */
/*   floor(c*cx)); I_l <- OptimizeXAxis for l = 2..cx;                     */
/*   A[ry][l] = I_l / ln min(l, yhat)   (0 when min(l, yhat) < 2).         */
/* A is dense (Bh-1) x (Bh-1), Bh = floor(B/2), A[(ry-2)*(Bh-1) + l-2];    */
/* entries outside the grid bound are left untouched.                      */
/* ---------------------------------------------------------------------- */
static void orientation(const double *u, const double *v, int n, int B, double c,
                        int flags, double *A)
{
    int lim = cell_limit(B, flags);
    int Bh = lim / 2, W = Bh - 1;
    int *ou = (int *) malloc(sizeof(int) * (size_t) n);
    int *ov = (int *) malloc(sizeof(int) * (size_t) n);
    double *us = (double *) malloc(sizeof(double) * (size_t) n);
    double *vs = (double *) malloc(sizeof(double) * (size_t) n);
    int *qv = (int *) malloc(sizeof(int) * (size_t) n);
    int *rowpt = (int *) malloc(sizeof(int) * (size_t) n);
    int *qu = (int *) malloc(sizeof(int) * (size_t) n);
    int *col = (int *) malloc(sizeof(int) * (size_t) n);
    double *I = (double *) malloc(sizeof(double) * (size_t) (lim + 1));
    argsort(u, n, ou);
    argsort(v, n, ov);
    for (int i = 0; i < n; i++) { us[i] = u[ou[i]]; vs[i] = v[ov[i]]; }
    for (int ry = 2; ry <= Bh; ry++) {
        int cx = lim / ry;
        if (cx < 2) continue;
        int yhat = oracle_equipartition(vs, n, ry, flags, qv);
        for (int i = 0; i < n; i++) rowpt[ov[i]] = qv[i];
        for (int i = 0; i < n; i++) qu[i] = rowpt[ou[i]];
        int K = oracle_superclumps(us, qu, n, khat_of(c, cx), flags, col, NULL);
        oracle_optimize_x_axis(col, qu, n, K, yhat, cx, I, NULL);
        for (int l = 2; l <= cx; l++) {
            int norm = (flags & ORC_NORM_BY_Y) ? (l < ry ? l : ry) : (l < yhat ? l : yhat);
            A[(size_t) (ry - 2) * W + (l - 2)] = norm >= 2 ? I[l - 2] / log((double) norm) : 0.0;
        }
    }
    free(I); free(col); free(qu); free(rowpt); free(qv); free(vs); free(us); free(ov); free(ou);
}

/* ---------------------------------------------------------------------- */
/* Statistics (App. A item 2; SOM definitions restated).                   */
/* M dense W x W, M[(y-2)*W + (x-2)] = M_{x,y}, valid when xy <= lim.      */
/* MIC = max M; MAS = max |M_{x,y} - M_{y,x}|; MEV = max over x = 2 or     */
/* y = 2; MCN = min log2(xy) over cells with M >= MIC - 1e-12.             */
/* ---------------------------------------------------------------------- */
static void statistics(const double *M, int lim, double *st)
{
    int W = lim / 2 - 1;
    double mic = 0.0, mas = 0.0, mev = 0.0, mcn = INFINITY;
    for (int y = 2; y <= lim / 2; y++)
        for (int x = 2; x * y <= lim; x++) {
            double m = M[(size_t) (y - 2) * W + (x - 2)];
            if (m > mic) mic = m;
        }
    for (int y = 2; y <= lim / 2; y++)
        for (int x = 2; x * y <= lim; x++) {
            double m = M[(size_t) (y - 2) * W + (x - 2)];
            double mt = M[(size_t) (x - 2) * W + (y - 2)];
            double d = fabs(m - mt);
            if (d > mas) mas = d;
            if ((x == 2 || y == 2) && m > mev) mev = m;
            if (m >= mic - ORC_MCN_TOL) {
                double l2 = log((double) (x * y)) / log(2.0);
                if (l2 < mcn) mcn = l2;
            }
        }
    st[0] = mic; st[1] = mas; st[2] = mev; st[3] = mcn;
}

/* ---------------------------------------------------------------------- */
/* Whole score of one pair (x, y).  Returns 0, or -1 when B < 4 (no cell)  */
/* or n < 2.  Optional outputs (NULL to skip), each W x W doubles with     */
/* W = floor(lim/2) - 1 (see oracle_grid_width):                           */
/*   A_xy[(ry-2)*W + l-2]: y equipartitioned into ry rows, x into l cols;  */
/*   A_yx[(rx-2)*W + l-2]: x equipartitioned into rx rows, y into l cols;  */
/*   M[(yy-2)*W + xx-2] = M_{xx,yy} (xx bins of x, yy bins of y).          */
/* stats (4 doubles): MIC, MAS, MEV, MCN.                                  */
/* ---------------------------------------------------------------------- */
int oracle_grid_width(int n, double alpha, int flags)
{
    return cell_limit(oracle_grid_bound(n, alpha), flags) / 2 - 1;
}

int oracle_score(const double *x, const double *y, int n, double alpha, double c,
                 int flags, double *M_out, double *Axy_out, double *Ayx_out, double *stats)
{
    if (n < 2) return -1;
    int B = oracle_grid_bound(n, alpha);
    int lim = cell_limit(B, flags);
    if (lim < 4) return -1;
    int W = lim / 2 - 1;
    size_t WW = (size_t) W * W;
    double *Axy = (double *) calloc(WW, sizeof(double));
    double *Ayx = (double *) calloc(WW, sizeof(double));
    double *M = (double *) calloc(WW, sizeof(double));
    orientation(x, y, n, B, c, flags, Axy);
    orientation(y, x, n, B, c, flags, Ayx);
    for (int yy = 2; yy <= lim / 2; yy++)
        for (int xx = 2; xx * yy <= lim; xx++) {
            double a = Axy[(size_t) (yy - 2) * W + (xx - 2)];
            double b = (flags & ORC_COMBINE_INDEX) ? Ayx[(size_t) (yy - 2) * W + (xx - 2)]
                                                  : Ayx[(size_t) (xx - 2) * W + (yy - 2)];
            M[(size_t) (yy - 2) * W + (xx - 2)] = a > b ? a : b;
        }
    double st[4];
    statistics(M, lim, st);
    if (stats) memcpy(stats, st, sizeof(st));
    if (M_out) memcpy(M_out, M, WW * sizeof(double));
    if (Axy_out) memcpy(Axy_out, Axy, WW * sizeof(double));
    if (Ayx_out) memcpy(Ayx_out, Ayx, WW * sizeof(double));
    free(M); free(Ayx); free(Axy);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Integer stages of one item, for bit-exact comparisons.                  */
/* Orientation 0: columns from x, rows from y; orientation 1: swapped.     */
/* Outputs: *yhat; row_starts[0..yhat] = sorted positions (of the row      */
/* variable) where each row starts, then n; *k clumps; *K superclumps;     */
/* ends[0..K-1] = number of points (in column-variable order) up to and    */
/* including each superclump.  Returns 0, or -1 on bad arguments.          */
/* ---------------------------------------------------------------------- */
int oracle_item(const double *x, const double *y, int n, double alpha, double c, int flags,
                int orient, int ry, int *yhat, int *row_starts, int *k, int *K, int *ends)
{
    int B = oracle_grid_bound(n, alpha);
    int lim = cell_limit(B, flags);
    if (n < 2 || ry < 2 || ry > lim / 2) return -1;
    const double *u = orient ? y : x, *v = orient ? x : y;
    int cx = lim / ry;
    int *ou = (int *) malloc(sizeof(int) * (size_t) n);
    int *ov = (int *) malloc(sizeof(int) * (size_t) n);
    double *us = (double *) malloc(sizeof(double) * (size_t) n);
    double *vs = (double *) malloc(sizeof(double) * (size_t) n);
    int *qv = (int *) malloc(sizeof(int) * (size_t) n);
    int *rowpt = (int *) malloc(sizeof(int) * (size_t) n);
    int *qu = (int *) malloc(sizeof(int) * (size_t) n);
    int *col = (int *) malloc(sizeof(int) * (size_t) n);
    argsort(u, n, ou);
    argsort(v, n, ov);
    for (int i = 0; i < n; i++) { us[i] = u[ou[i]]; vs[i] = v[ov[i]]; }
    int yh = oracle_equipartition(vs, n, ry, flags, qv);
    *yhat = yh;
    int r = 0;
    row_starts[0] = 0;
    for (int i = 1; i < n; i++)
        if (qv[i] != qv[i - 1] && r + 1 <= ry) row_starts[++r] = i;
    row_starts[yh <= ry ? yh : ry] = n;
    for (int i = 0; i < n; i++) rowpt[ov[i]] = qv[i];
    for (int i = 0; i < n; i++) qu[i] = rowpt[ou[i]];
    int kk = 0;
    int KK = oracle_superclumps(us, qu, n, khat_of(c, cx), flags, col, &kk);
    *k = kk;
    *K = KK;
    for (int i = 0; i < n; i++) if (i == n - 1 || col[i + 1] != col[i]) ends[col[i]] = i + 1;
    free(col); free(qu); free(rowpt); free(qv); free(vs); free(us); free(ov); free(ou);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Cumulative count table of one item (App. A item 10a):                   */
/* N[t*yhat + r] = number of points among the first e_t in column-variable */
/* order (the first t superclumps) that lie in row r, t = 0..K,            */
/* r = 0..yhat-1.  Same item as oracle_item; N holds (n+1)*ry ints at      */
/* most.  Returns K, or -1 on bad arguments.                               */
/* ---------------------------------------------------------------------- */
int oracle_counts(const double *x, const double *y, int n, double alpha, double c, int flags,
                  int orient, int ry, int *N)
{
    int B = oracle_grid_bound(n, alpha);
    int lim = cell_limit(B, flags);
    if (n < 2 || ry < 2 || ry > lim / 2) return -1;
    const double *u = orient ? y : x, *v = orient ? x : y;
    int cx = lim / ry;
    int *ou = (int *) malloc(sizeof(int) * (size_t) n);
    int *ov = (int *) malloc(sizeof(int) * (size_t) n);
    double *us = (double *) malloc(sizeof(double) * (size_t) n);
    double *vs = (double *) malloc(sizeof(double) * (size_t) n);
    int *qv = (int *) malloc(sizeof(int) * (size_t) n);
    int *rowpt = (int *) malloc(sizeof(int) * (size_t) n);
    int *qu = (int *) malloc(sizeof(int) * (size_t) n);
    int *col = (int *) malloc(sizeof(int) * (size_t) n);
    argsort(u, n, ou);
    argsort(v, n, ov);
    for (int i = 0; i < n; i++) { us[i] = u[ou[i]]; vs[i] = v[ov[i]]; }
    int yh = oracle_equipartition(vs, n, ry, flags, qv);
    for (int i = 0; i < n; i++) rowpt[ov[i]] = qv[i];
    for (int i = 0; i < n; i++) qu[i] = rowpt[ou[i]];
    int K = oracle_superclumps(us, qu, n, khat_of(c, cx), flags, col, NULL);
    /* row t+1 of the table adds superclump t's points to row t */
    for (int r = 0; r < yh; r++) N[r] = 0;
    for (int t = 0; t < K; t++) {
        for (int r = 0; r < yh; r++) N[(size_t) (t + 1) * yh + r] = N[(size_t) t * yh + r];
        for (int i = 0; i < n; i++)
            if (col[i] == t) N[(size_t) (t + 1) * yh + qu[i]]++;
    }
    free(col); free(qu); free(rowpt); free(qv); free(vs); free(us); free(ov); free(ou);
    return K;
}

/* Tie-group start of every sample: out[j] = number of samples whose value */
/* is smaller than v[j], i.e. the sorted position where v[j]'s tie group   */
/* begins (the rank information the method uses: order and ties).         */
void oracle_group_starts(const double *v, int n, int *out)
{
    int *o = (int *) malloc(sizeof(int) * (size_t) (n > 0 ? n : 1));
    argsort(v, n, o);
    int start = 0;
    for (int i = 0; i < n; i++) {
        if (i > 0 && v[o[i]] != v[o[i - 1]]) start = i;
        out[o[i]] = start;
    }
    free(o);
}

/* ---------------------------------------------------------------------- */
/* Many pairs on CPU threads (one pair per task).  X is m x n row-major    */
/* (variable-contiguous).  pairs: npairs (i, j) index pairs as 2*npairs    */
/* int64, or NULL for all i < j in the order (0,1), (0,2), ..., (m-2,m-1). */
/* out: 4 doubles per pair.  Returns 0, or -1 on bad arguments.            */
/* ---------------------------------------------------------------------- */
typedef struct {
    const double *X; int m, n; double alpha, c; int flags;
    const long long *pairs; long long npairs; double *out;
    long long next; pthread_mutex_t lock; int err;
} job_t;

static void pair_of(const job_t *J, long long p, int *i, int *j)
{
    if (J->pairs) { *i = (int) J->pairs[2 * p]; *j = (int) J->pairs[2 * p + 1]; return; }
    /* row-major upper triangle */
    long long m = J->m, rem = p;
    int a = 0;
    while (rem >= m - 1 - a) { rem -= m - 1 - a; a++; }
    *i = a; *j = a + 1 + (int) rem;
}

static void *worker(void *arg)
{
    job_t *J = (job_t *) arg;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        long long p = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (p >= J->npairs) break;
        int i, j;
        pair_of(J, p, &i, &j);
        if (oracle_score(J->X + (size_t) i * J->n, J->X + (size_t) j * J->n, J->n, J->alpha, J->c,
                         J->flags, NULL, NULL, NULL, J->out + 4 * p) != 0)
            J->err = 1;
    }
    return NULL;
}

int oracle_allpairs(const double *X, int m, int n, double alpha, double c, int flags,
                    const long long *pairs, long long npairs, int nthreads, double *out)
{
    if (m < 2 || n < 2 || nthreads < 1) return -1;
    job_t J;
    J.X = X; J.m = m; J.n = n; J.alpha = alpha; J.c = c; J.flags = flags;
    J.pairs = pairs;
    J.npairs = pairs ? npairs : (long long) m * (m - 1) / 2;
    J.out = out; J.next = 0; J.err = 0;
    pthread_mutex_init(&J.lock, NULL);
    pthread_t *th = (pthread_t *) malloc(sizeof(pthread_t) * (size_t) nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, worker, &J);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&J.lock);
    return J.err ? -1 : 0;
}
