// micx_kernels.hip -- gfx950 kernels for the approximate characteristic matrix
// of the MINE statistics (Albanese et al. 2012, arXiv:1208.4271).
//
// Pipeline (one launch each; host orchestration in micx_api.hip):
//   k_xlogx  table L[j] = j ln j, j = 0..n (FP64) used by every entropy term
//   k_rank   per variable: sort in LDS, tie groups, dense group ranks
//   k_equip  per (variable, row count y): EquipartitionYAxis (App. A items 3-4)
//   k_part   per item (pair, orientation, y), one item per lane:
//            GetClumpsPartition (Algorithm 1) and GetSuperclumpsPartition
//            (Algorithm 2) streamed over the points in column order
//   k_dp     (micx_dp.hip) per item, one wavefront: cumulative count table
//            (App. A item 10a), column costs (item 10b) and the OptimizeXAxis
//            dynamic program over the superclump boundaries
//   k_stats  per pair: characteristic matrix from both orientations and
//            MIC, MAS, MEV, MCN (App. A items 1, 2, 4)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "micx_device.h"

namespace micx {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double load_value(const void *X, int dtype, size_t idx) {
    if (dtype == 0) return (double)((const float *)X)[idx];
    if (dtype == 1) return ((const double *)X)[idx];
    return (double)((const int32_t *)X)[idx];
}

// Order-preserving 64-bit key of a finite double; -0.0 and +0.0 map to the
// same key because the method compares values with ==.
__device__ __forceinline__ uint64_t order_key(double d) {
    if (d == 0.0) d = 0.0;
    uint64_t b = __double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// EquipartitionYAxis row-closing test on integers (App. A item 3): a points
// in the open row, s in the next tie group, R points left when the row
// opened, L rows left including it.  |a + s - d| >= |a - d| with d = R/L
// is (2a + s) L >= 2R.  Compatibility flags: MICX_COMPAT_TIE_STRICT closes
// on '>' only; MICX_COMPAT_DESIRED_INT takes d = floor(R/L), giving
// 2a + s >= 2 floor(R/L).  (2a + s) <= 3n and L <= n, so 32 bits hold
// the products for n <= MICX_MAX_N; L >= 1 always (the last row never
// closes).
// DINT: the integer-cast target row size (MICX_COMPAT_DESIRED_INT) as a
// compile-time choice, so the default test carries no division.
template <bool DINT>
__device__ __forceinline__ bool closes_row_t(int a, int s, int R, int L, bool strict) {
    const int lhs = DINT ? 2 * a + s : (2 * a + s) * L;
    const int rhs = DINT ? 2 * (R / L) : 2 * R;
    return strict ? lhs > rhs : lhs >= rhs;
}

__device__ __forceinline__ bool closes_row(int a, int s, int R, int L, int compat) {
    const bool strict = (compat & MICX_COMPAT_TIE_STRICT) != 0;
    return (compat & MICX_COMPAT_DESIRED_INT) ? closes_row_t<true>(a, s, R, L, strict)
                                               : closes_row_t<false>(a, s, R, L, strict);
}

// ------------------------------------------------------------------ k_xlogx

__global__ void k_xlogx(int n, double *L) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j <= n) L[j] = j > 1 ? (double)j * log((double)j) : 0.0;
}

// --------------------------------------------------------------- k_geometry
// Grid geometry on the device (asynchronous calls need no host staging for it): x(y) = floor(B/y),
// khat(y) = max(1, min(floor(c x(y)) (+1 with MICX_COMPAT_KHAT_PLUS1), n)),
// and the prefix offsets of the per-item end buffers and score rows; the
// same arithmetic as the host's geometry of the other entry points.
__global__ void k_geometry(int n, int B, double c, int compat, int NY, int *geo) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int ks = 0, as = 0;
    for (int yi = 0; yi < NY; yi++) {
        const int y = yi + 2, x = B / y;
        double kd = floor(c * (double)x);
        if (compat & MICX_COMPAT_KHAT_PLUS1) kd += 1.0;
        int kh = kd >= (double)n ? n : (int)kd;
        if (kh < 1) kh = 1;
        geo[yi] = x;
        geo[NY + yi] = kh;
        geo[2 * NY + yi] = ks;
        geo[3 * NY + yi] = as;
        ks += end_slots(kh);
        as += x - 1;
    }
}


// ------------------------------------------------------------------- k_rank
// One workgroup per variable.  Bitonic sort of (key, sample index) pairs in
// LDS (N2 = next power of two >= n), then tie-group starts by a max-scan.

__device__ __forceinline__ void rank_body(const void *X, int dtype, int v, int n, int N2, int *perm,
                                          int *gsize, int *grank, int *status, unsigned char *smem) {
    uint64_t *key = (uint64_t *)smem;
    int *idx = (int *)(key + N2);
    int *gst = idx + N2;
    const int tid = threadIdx.x, nt = blockDim.x;
    const size_t base = (size_t)v * n;
    for (int i = tid; i < N2; i += nt) {
        if (i < n) {
            const double d = load_value(X, dtype, base + i);
            if (!isfinite(d)) atomicOr(status, 1);
            key[i] = order_key(d);
            idx[i] = i;
        } else {
            key[i] = ~0ull;
            idx[i] = 0x7fffffff;
        }
    }
    __syncthreads();
    for (int k = 2; k <= N2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < N2; i += nt) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t ka = key[i], kb = key[ixj];
                    const int ia = idx[i], ib = idx[ixj];
                    const bool a_gt_b = (ka > kb) || (ka == kb && ia > ib);
                    const bool up = (i & k) == 0;
                    if (a_gt_b == up) {
                        key[i] = kb; key[ixj] = ka;
                        idx[i] = ib; idx[ixj] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
    // group start of every position: inclusive max-scan of (start ? i : 0)
    for (int i = tid; i < N2; i += nt)
        gst[i] = (i < n && (i == 0 || key[i] != key[i - 1])) ? i : 0;
    __syncthreads();
    for (int d = 1; d < N2; d <<= 1) {
        int vals[8];
        int c = 0;
        for (int i = tid; i < N2; i += nt, c++) vals[c] = (i >= d) ? max(gst[i], gst[i - d]) : gst[i];
        __syncthreads();
        c = 0;
        for (int i = tid; i < N2; i += nt, c++) gst[i] = vals[c];
        __syncthreads();
    }
    for (int i = tid; i < n; i += nt) {
        const int s = gst[i];
        perm[base + i] = idx[i];
        grank[base + idx[i]] = s;
        const bool end = (i == n - 1) || key[i + 1] != key[i];
        if (end) gsize[base + s] = i - s + 1;
        if (s != i) gsize[base + i] = 0;
    }
}

__global__ __launch_bounds__(1024) void k_rank(const void *X, int dtype, int m, int n, int N2,
                                               int *perm, int *gsize, int *grank, int *status) {
    extern __shared__ __align__(16) unsigned char smem[];
    rank_body(X, dtype, blockIdx.x, n, N2, perm, gsize, grank, status, smem);
}

// ------------------------------------------------------------------ k_equip
// EquipartitionYAxis (App. A items 3-4), one (variable, y) per lane.  The
// greedy walks the tie groups in order; with a the current row's size, s the
// next group's size, R the points left when the row opened and L the rows
// left (including the current one), the paper's real-valued rule
// |a + s - R/L| >= |a - R/L| (row not empty) is equivalent to the integer
// test (2a + s) * L >= 2R, used here so that the partition is bit-exact.

__device__ __forceinline__ void equip_body(int v, int yb, int n, int NY, int NYP, const int *gsize,
                                           uint16_t *rowof, int *yhat, int *rowstart, int RS, int *gs,
                                           int compat) {
    // gs: the variable's tie-group sizes in LDS, copied once (coalesced)
    const int yi = yb * 64 + threadIdx.x;
    const bool act = yi < NY;
    const int y = yi + 2;
    for (int p = threadIdx.x; p < n; p += 64) gs[p] = gsize[(size_t)v * n + p];
    __syncthreads();
    uint16_t *ro = rowof + (size_t)v * n * NYP + yi;
    int *rs = rowstart ? rowstart + ((size_t)v * NY + yi) * RS : nullptr;
    int r = 0, a = 0, R = n, L = y;
    if (act && rs) rs[0] = 0;
    for (int p = 0; p < n;) {
        const int s = gs[p];
        if (a != 0 && closes_row(a, s, R, L, compat)) {
            r++;
            a = 0;
            R = n - p;
            L = y - r;
            if (act && rs) rs[r] = p;
        }
        if (act) ro[(size_t)p * NYP] = (uint16_t)r;
        a += s;
        p += s;
    }
    if (act) {
        yhat[(size_t)v * NY + yi] = r + 1;
        if (rs) rs[r + 1] = n;
    }
}

__global__ __launch_bounds__(64) void k_equip(int m, int n, int NY, int NYP, const int *gsize,
                                              uint16_t *rowof, int *yhat, int *rowstart, int RS, int compat) {
    extern __shared__ int gsl[];
    const int nyb = (NY + 63) / 64;
    equip_body(blockIdx.x / nyb, blockIdx.x % nyb, n, NY, NYP, gsize, rowof, yhat, rowstart, RS, gsl, compat);
}

// ------------------------------------------------------------------- k_part
// Clumps and superclumps of one item per lane.  A wavefront serves one
// (pair, orientation) and up to 64 row counts y; the points are visited in
// the column variable's order, so the per-point reads (tie-group size of the
// column variable, group rank of the row variable) are the same for every
// lane and only the row lookup differs.
//
// GetClumpsPartition (Algorithm 1, with one fresh label per mixed tie group
// as Fig. 2 prints it): a column-variable tie group whose points lie in two
// or more rows is a clump boundary on both sides; otherwise a boundary sits
// between consecutive groups whose rows differ.
// GetSuperclumpsPartition (Algorithm 2): when the clumps outnumber
// khat = floor(c x), EquipartitionYAxis runs over the clump sequence (each
// clump one tie group) with khat rows.  Both are computed in one pass; the
// clump list is kept only while it fits in khat entries.

struct PartArgs {
    int n, NY, NYP, KSUM;
    PairSource ps;
    const int *perm, *gsize, *grank;
    const uint16_t *rowof;       // [v][p][NYP]
    const int *khat, *koff;
    const int *yhat;             // [v][y-2]: rows of each variable's equipartitions
    int *cbuf, *sbuf, *K, *k, *src, *Yh;
    unsigned char *lab;          // row labels in column order, [item][y-2][p]
    size_t lab_row;
    int compat;                  // MICX_COMPAT_* flags
    int64_t nitems;              // (pair, orientation) items
    int flat;                    // waves over consecutive (item, row count) slots
};

// LDS tile of one 64-point block: each point's labels for the wave's row
// counts (up to 64 x 2 bytes), rows 144 bytes apart so that the 16-byte row
// writes of neighbouring lanes fall in different banks.
constexpr int PART_TILE = 144;

template <bool L16, bool DINT, bool STRICT>
__device__ __forceinline__ void part_body(const PartArgs &a, int w, unsigned char *tile) {
    const int nyb = (a.NY + 63) / 64;
    const int yb = w % nyb, po = w / nyb;
    const int o = po & 1, pl = po >> 1;
    int pi, pj;
    pair_of(a.ps, pl, pi, pj);
    const int U = o ? pj : pi, V = o ? pi : pj;
    const int lane = threadIdx.x;
    const int y0 = yb * 64, yi = y0 + lane;
    const int nlab = min(64, a.NYP - y0);    // labels per point held in the tile (multiple of 8)
    const bool act = yi < a.NY;
    const int yic = act ? yi : a.NY - 1;
    const int n = a.n;
    const int kh = a.khat[yic];
    const size_t base = (size_t)po * a.KSUM + a.koff[yic];
    int *cb = a.cbuf + base;
    int *sb = a.sbuf + base;
    const int *permU = a.perm + (size_t)U * n;
    const int *gsU = a.gsize + (size_t)U * n;
    const int *grV = a.grank + (size_t)V * n;
    const uint16_t *rowV = a.rowof + (size_t)V * n * a.NYP + y0;
    uint4 *labo = (uint4 *)(a.lab + ((size_t)po * a.NY + yic) * a.lab_row);

    int first = 0, mixed = 0, gstart = 0;   // current tie group of the column variable
    int last = -2;                           // label of the previous group: -2 none, -1 mixed
    int cstart = 0, k = 0;                   // current clump start, clumps emitted
    int sa = 0, sP0 = 0, sR = n, sL = kh, sr = 0;   // superclump greedy state

    // A clump boundary at ce when e (per lane): the clump list and the
    // superclump greedy (EquipartitionYAxis over the clump sizes, same
    // integer test as k_equip) advance through selects; only the two stores
    // are conditional.  (2a + s) <= 3n and L <= n with n <= MICX_MAX_N, so
    // the product fits 32 bits.
    auto emit_clump = [&](bool e, int ce) {
        const int size = ce - cstart;
        k += e ? 1 : 0;
        if (e & act & (k <= kh)) cb[k - 1] = ce;
        const bool sup = e & (sa != 0) & closes_row_t<DINT>(sa, size, sR, sL, STRICT);   // no short-circuit
        if (sup & act) sb[sr] = sP0 + sa;
        sr += sup ? 1 : 0;
        sP0 += sup ? sa : 0;
        sa = sup ? 0 : sa;
        sR = n - sP0;
        sL = kh - sr;
        sa += e ? size : 0;
        cstart = e ? ce : cstart;
    };
    auto close_group = [&]() {
        const int lg = mixed ? -1 : first;
        emit_clump((last != -2) & ((lg == -1) | (last == -1) | (lg != last)), gstart);
        last = lg;
    };

    // per-point reads of the next 64-point block, issued one block ahead:
    // column-group size and the row variable's group rank
    int gsz_n = 0, grk_n = 0;
    if (lane < n) {
        gsz_n = gsU[lane];
        grk_n = grV[permU[lane]];
    }
    for (int p0 = 0; p0 < n; p0 += 64) {
        const int q = p0 + lane;
        const int gsz = gsz_n, grk = grk_n;
        const int cnt = min(64, n - p0);
        // this lane's point: its labels for the wave's row counts into the tile
        if (q < n) {
            const uint4 *src = (const uint4 *)(rowV + (size_t)grk * a.NYP);
            uint4 *dst = (uint4 *)(tile + lane * PART_TILE);
#pragma unroll
            for (int v = 0; v < 8; v++)
                if (8 * v < nlab) dst[v] = src[v];
        }
        if (q + 64 < n) {
            gsz_n = gsU[q + 64];
            grk_n = grV[permU[q + 64]];
        }
        const uint64_t starts = __ballot(q < n && gsz > 0);   // tie-group starts of the block
        wave_sync();
        // the points in order; this lane's labels are packed for the DP's
        // count table as they are read (padding beyond n holds 0)
        constexpr int NW = L16 ? 32 : 16;
        uint32_t pk[NW];
#pragma unroll
        for (int v = 0; v < NW; v++) pk[v] = 0;
#pragma unroll
        for (int s = 0; s < 64; s++) {
            if (s < cnt) {
                const int lab = *(const uint16_t *)(tile + s * PART_TILE + 2 * lane);
                if (L16) pk[s >> 1] |= (uint32_t)lab << (16 * (s & 1));
                else pk[s >> 2] |= (uint32_t)lab << (8 * (s & 3));
                if ((starts >> s) & 1) {
                    if (p0 + s > 0) close_group();
                    first = lab;
                    mixed = 0;
                    gstart = p0 + s;
                } else {
                    mixed |= (lab != first);
                }
            }
        }
        if (act) {
            uint4 *d = labo + (p0 >> (L16 ? 3 : 4));
#pragma unroll
            for (int v = 0; v < NW / 4; v++) d[v] = make_uint4(pk[4 * v], pk[4 * v + 1], pk[4 * v + 2], pk[4 * v + 3]);
        }
        wave_sync();   // the tile is rewritten by the next block
    }
    close_group();
    emit_clump(true, n);
    if (act) sb[sr] = n;
    if (act) {
        const size_t it = (size_t)po * a.NY + yi;
        a.k[it] = k;
        a.Yh[it] = a.yhat[(size_t)V * a.NY + yi];
        if (k <= kh) {
            a.K[it] = k;
            a.src[it] = 0;
        } else {
            a.K[it] = sr + 1;
            a.src[it] = 1;
        }
    }
}

// The same scan with a wavefront over 64 consecutive (item, row count)
// slots, so that the lanes beyond an item's row counts serve the next items
// (22 <= NY <= 64: at most four items per wave).  Each lane follows its own
// item's tie groups.  A tile row holds, per item of the wave, the 16-byte
// chunks of that item's row of labels that cover its row counts in the wave
// (at most 12 chunks, 192 bytes: a chunk per 8 row counts, plus one per item
// for a slice that starts or ends inside a chunk); a lane reads its label at
// its own column.  Rows are 13 x 16 bytes apart (the 16-byte writes of
// neighbouring lanes fall in different banks).
constexpr int PART_FSTRIDE = 208;
constexpr int PART_FSLOTS = 4;

template <bool L16, bool DINT, bool STRICT>
__device__ __forceinline__ void part_body_flat(const PartArgs &a, int w, unsigned char *tile) {
    const int NY = a.NY, n = a.n, NYP = a.NYP;
    const int lane = threadIdx.x;
    const int64_t total = a.nitems * NY;
    const int64_t f0 = (int64_t)w * 64, f = f0 + lane;
    const bool act = f < total;
    const int64_t fc = act ? f : total - 1;
    const int po = (int)(fc / NY), yi = (int)(fc - (int64_t)po * NY);
    const int po0 = (int)(f0 / NY);
    const int jl = po - po0;                                   // this lane's item among the wave's
    const int nit = (int)((f0 + 63 < total ? f0 + 63 : total - 1) / NY) - po0 + 1;
    // the wave's items: column variable U, row variable V, the first 16-byte
    // chunk of its row counts in the wave, the chunk count, and its first
    // chunk's place in the tile row
    // (only indexes are kept per item; the addresses are formed where used)
    int uS[PART_FSLOTS], vS[PART_FSLOTS], chS[PART_FSLOTS], tS[PART_FSLOTS];
    int tcol = 0;
#pragma unroll
    for (int j = 0; j < PART_FSLOTS; j++) {
        const int poj = po0 + (j < nit ? j : nit - 1);
        int pi, pj;
        pair_of(a.ps, poj >> 1, pi, pj);
        uS[j] = (poj & 1) ? pj : pi;
        vS[j] = (poj & 1) ? pi : pj;
        const int lb = j == 0 ? 0 : (int)((int64_t)poj * NY - f0);   // first lane
        const int c0 = j == 0 ? (int)(f0 - (int64_t)po0 * NY) : 0;   // first row count
        const int len = min(NY - c0, 64 - lb);
        chS[j] = j < nit ? ((c0 & 7) + len + 7) >> 3 : 0;
        tS[j] = tcol;
        tcol += chS[j];
    }
    const int c0q = (int)(f0 - (int64_t)po0 * NY) >> 3;   // first item's first chunk
    const int myV = jl == 0 ? vS[0] : jl == 1 ? vS[1] : jl == 2 ? vS[2] : vS[3];
    const int myT = jl == 0 ? tS[0] : jl == 1 ? tS[1] : jl == 2 ? tS[2] : tS[3];
    // this lane's label: byte offset in a tile row
    const int col = 16 * myT + 2 * (yi & 7) + 16 * ((yi >> 3) - (jl == 0 ? c0q : 0));
    const int kh = a.khat[yi];
    const size_t base = (size_t)po * a.KSUM + a.koff[yi];
    int *cb = a.cbuf + base;
    int *sb = a.sbuf + base;
    uint4 *labo = (uint4 *)(a.lab + ((size_t)po * NY + yi) * a.lab_row);

    int first = 0, mixed = 0, gstart = 0;
    int last = -2;
    int cstart = 0, k = 0;
    int sa = 0, sP0 = 0, sR = n, sL = kh, sr = 0;
    // the last four clump and superclump ends, stored four at a time (16-byte
    // aligned: the buffers hold end_slots(khat) ints per row count); the rest
    // is stored at the end
    int cq0 = 0, cq1 = 0, cq2 = 0, cq3 = 0, sq0 = 0, sq1 = 0, sq2 = 0, sq3 = 0;

    auto emit_clump = [&](bool e, int ce) {
        const int size = ce - cstart;
        k += e ? 1 : 0;
        const bool cpush = e & (k <= kh);
        cq0 = cpush ? cq1 : cq0;
        cq1 = cpush ? cq2 : cq1;
        cq2 = cpush ? cq3 : cq2;
        cq3 = cpush ? ce : cq3;
        if (cpush & act & ((k & 3) == 0)) *(int4 *)(cb + k - 4) = make_int4(cq0, cq1, cq2, cq3);
        const bool sup = e & (sa != 0) & closes_row_t<DINT>(sa, size, sR, sL, STRICT);
        const int se = sP0 + sa;
        sq0 = sup ? sq1 : sq0;
        sq1 = sup ? sq2 : sq1;
        sq2 = sup ? sq3 : sq2;
        sq3 = sup ? se : sq3;
        if (sup & act & (((sr + 1) & 3) == 0)) *(int4 *)(sb + sr - 3) = make_int4(sq0, sq1, sq2, sq3);
        sr += sup ? 1 : 0;
        sP0 += sup ? sa : 0;
        sa = sup ? 0 : sa;
        sR = n - sP0;
        sL = kh - sr;
        sa += e ? size : 0;
        cstart = e ? ce : cstart;
    };
    // closes the current group where g (per lane)
    auto close_group_if = [&](bool g) {
        const int lg = mixed ? -1 : first;
        emit_clump(g & (last != -2) & ((lg == -1) | (last == -1) | (lg != last)), gstart);
        last = g ? lg : last;
    };

    int gsz_n[PART_FSLOTS], grk_n[PART_FSLOTS];
#pragma unroll
    for (int j = 0; j < PART_FSLOTS; j++) {
        gsz_n[j] = 0;
        grk_n[j] = 0;
        if (j < nit && lane < n) {
            gsz_n[j] = a.gsize[(size_t)uS[j] * n + lane];
            grk_n[j] = a.grank[(size_t)vS[j] * n + a.perm[(size_t)uS[j] * n + lane]];
        }
    }
    for (int p0 = 0; p0 < n; p0 += 64) {
        const int q = p0 + lane;
        const int cnt = min(64, n - p0);
        uint64_t st[PART_FSLOTS];
        uint64_t sall = 0;
#pragma unroll
        for (int j = 0; j < PART_FSLOTS; j++) {
            st[j] = 0;
            if (j < nit) {
                if (q < n) {
                    // up to five chunks loaded together (indexes clamped to the
                    // slice), the rest (row counts above 33) after them
                    const uint4 *src = (const uint4 *)(a.rowof + ((size_t)vS[j] * n + grk_n[j]) * NYP) +
                                       (j == 0 ? c0q : 0);
                    uint4 *dst = (uint4 *)(tile + lane * PART_FSTRIDE) + tS[j];
                    const int ch = chS[j];
                    uint4 v[5];
#pragma unroll
                    for (int e = 0; e < 5; e++) v[e] = src[min(e, ch - 1)];
                    if (ch > 5) {
                        uint4 u[4];
#pragma unroll
                        for (int e = 0; e < 4; e++) u[e] = src[min(5 + e, ch - 1)];
#pragma unroll
                        for (int e = 0; e < 4; e++)
                            if (5 + e < ch) dst[5 + e] = u[e];
                    }
#pragma unroll
                    for (int e = 0; e < 5; e++)
                        if (e < ch) dst[e] = v[e];
                }
                st[j] = __ballot(q < n && gsz_n[j] > 0);
                sall |= st[j];
                if (q + 64 < n) {
                    gsz_n[j] = a.gsize[(size_t)uS[j] * n + q + 64];
                    grk_n[j] = a.grank[(size_t)vS[j] * n + a.perm[(size_t)uS[j] * n + q + 64]];
                }
            }
        }
        const uint64_t mine = jl == 0 ? st[0] : jl == 1 ? st[1] : jl == 2 ? st[2] : st[3];
        const uint32_t mlo = (uint32_t)mine, mhi = (uint32_t)(mine >> 32);
        wave_sync();
        constexpr int NW = L16 ? 32 : 16;
        uint32_t pk[NW];
#pragma unroll
        for (int v = 0; v < NW; v++) pk[v] = 0;
#pragma unroll
        for (int s = 0; s < 64; s++) {
            if (s < cnt) {
                const int lab = *(const uint16_t *)(tile + s * PART_FSTRIDE + col);
                if (L16) pk[s >> 1] |= (uint32_t)lab << (16 * (s & 1));
                else pk[s >> 2] |= (uint32_t)lab << (8 * (s & 3));
                if ((sall >> s) & 1) {
                    // some item's tie group starts at this point: the lanes of
                    // those items close their previous group
                    const bool g = (((s < 32 ? mlo : mhi) >> (s & 31)) & 1) != 0;
                    if (p0 + s > 0) close_group_if(g);
                    mixed = g ? 0 : (mixed | (lab != first));
                    first = g ? lab : first;
                    gstart = g ? p0 + s : gstart;
                } else {
                    mixed |= (lab != first);
                }
            }
        }
        if (act) {
            uint4 *d = labo + (p0 >> (L16 ? 3 : 4));
#pragma unroll
            for (int v = 0; v < NW / 4; v++) d[v] = make_uint4(pk[4 * v], pk[4 * v + 1], pk[4 * v + 2], pk[4 * v + 3]);
        }
        wave_sync();   // the tile is rewritten by the next block
    }
    close_group_if(true);
    emit_clump(true, n);
    if (act) {
        // the ends still queued: the last (count mod 4) of each buffer
        const int kc = min(k, kh), rc = kc & 3, rs = sr & 3;
        if (rc >= 1) cb[kc - 1] = cq3;
        if (rc >= 2) cb[kc - 2] = cq2;
        if (rc >= 3) cb[kc - 3] = cq1;
        if (rs >= 1) sb[sr - 1] = sq3;
        if (rs >= 2) sb[sr - 2] = sq2;
        if (rs >= 3) sb[sr - 3] = sq1;
        sb[sr] = n;
        const size_t it = (size_t)po * NY + yi;
        a.k[it] = k;
        a.Yh[it] = a.yhat[(size_t)myV * NY + yi];
        if (k <= kh) {
            a.K[it] = k;
            a.src[it] = 0;
        } else {
            a.K[it] = sr + 1;
            a.src[it] = 1;
        }
    }
}

// the compatibility variants of the row-closing test as compile-time choices
// (a uniform branch per launch; the default test has no select or division)
template <bool L16>
__device__ __forceinline__ void part_dispatch(const PartArgs &a, int w, unsigned char *tile) {
    const bool dint = (a.compat & MICX_COMPAT_DESIRED_INT) != 0;
    const bool strict = (a.compat & MICX_COMPAT_TIE_STRICT) != 0;
    if (dint) {
        if (strict) part_body<L16, true, true>(a, w, tile);
        else part_body<L16, true, false>(a, w, tile);
    } else {
        if (strict) part_body<L16, false, true>(a, w, tile);
        else part_body<L16, false, false>(a, w, tile);
    }
}

template <bool L16>
__global__ __launch_bounds__(64) void k_part(PartArgs a) {
    __shared__ __align__(16) unsigned char tile[64 * PART_TILE];
    part_dispatch<L16>(a, blockIdx.x, tile);
}

// several items per wave (a kernel of its own: its registers do not weigh on
// the one-item scan)
template <bool L16>
__global__ __launch_bounds__(64) void k_part_flat(PartArgs a) {
    __shared__ __align__(16) unsigned char tile[64 * PART_FSTRIDE];
    const bool dint = (a.compat & MICX_COMPAT_DESIRED_INT) != 0;
    const bool strict = (a.compat & MICX_COMPAT_TIE_STRICT) != 0;
    if (dint) {
        if (strict) part_body_flat<L16, true, true>(a, blockIdx.x, tile);
        else part_body_flat<L16, true, false>(a, blockIdx.x, tile);
    } else {
        if (strict) part_body_flat<L16, false, true>(a, blockIdx.x, tile);
        else part_body_flat<L16, false, false>(a, blockIdx.x, tile);
    }
}

// ---------------------------------------------------------- k_moments/k_pearson
// Pearson's correlation coefficient beside the MINE statistics, and the
// non-linearity index MIC - rho^2 (the companion outputs of the paper's
// engine; Sec. 2, Fig. 1).  FP64 throughout: per variable a mean, then the
// centred sum of squares (two passes); per pair one centred dot product.

__device__ __forceinline__ double block_sum_256(double v, double *red) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

// one workgroup of 256 per variable: mean, and 1/sqrt(centred sum of squares)
// (NaN for a constant variable)
__global__ __launch_bounds__(256) void k_moments(const void *X, int dtype, int n, double *mean,
                                                 double *inorm) {
    __shared__ double red[4];
    const int v = blockIdx.x;
    const size_t base = (size_t)v * n;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += load_value(X, dtype, base + i);
    const double mu = block_sum_256(s, red) / (double)n;
    double q = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double d = load_value(X, dtype, base + i) - mu;
        q += d * d;
    }
    const double ss = block_sum_256(q, red);
    if (threadIdx.x == 0) {
        mean[v] = mu;
        inorm[v] = ss > 0.0 ? 1.0 / sqrt(ss) : NAN;
    }
}

// one wavefront per pair: rho (clamped to [-1, 1]) and, with the pair's MINE
// record, MIC - rho^2
__global__ __launch_bounds__(256) void k_pearson(const void *X, int dtype, int n, PairSource ps,
                                                 int npairs, const double *mean, const double *inorm,
                                                 const double *stats, double *out) {
    const int lane = threadIdx.x & 63;
    const int pl = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pl >= npairs) return;
    int i, j;
    pair_of(ps, pl, i, j);
    const double mi = mean[i], mj = mean[j];
    const size_t bi = (size_t)i * n, bj = (size_t)j * n;
    double d = 0.0;
    for (int k = lane; k < n; k += 64) d += (load_value(X, dtype, bi + k) - mi) * (load_value(X, dtype, bj + k) - mj);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if (lane == 0) {
        double r = d * inorm[i] * inorm[j];
        if (!isnan(r)) r = fmin(1.0, fmax(-1.0, r));
        out[2 * (size_t)pl] = r;
        out[2 * (size_t)pl + 1] = stats ? stats[4 * (size_t)pl] - r * r : NAN;
    }
}

hipError_t launch_pearson(const void *X, int dtype, int m, int n, PairSource ps, int npairs,
                          double *mean, double *inorm, const double *stats, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_moments, dim3(m), dim3(256), 0, s, X, dtype, n, mean, inorm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pearson, dim3((npairs + 3) / 4), dim3(256), 0, s, X, dtype, n, ps, npairs,
                       (const double *)mean, (const double *)inorm, stats, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_stats
// Characteristic matrix and statistics of a pair (one pair per thread in the
// batch-stream kernels, one per wavefront in k_stats).
// M_{x,y} (x bins of the first variable, y of the second) is the larger of
// the orientation scores for that grid shape: first variable optimised into
// x columns with the second equipartitioned into y rows, or the second
// optimised into y columns with the first equipartitioned into x rows.

struct StatsArgs {
    int npairs, B, NY, W, ASUM, compat;
    const int *aoff;
    const double *A;
    double *out, *M, *Axy, *Ayx;
    Recheck rc;                  // near-tie flags (rc.band > 0) of the 32-bit form
    const int *plist, *pcount;   // only these batch-local pairs (the recheck pass), or null
    const int *status;           // nothing is written while *status != 0, or null
    // batch streams: flags go to the pass's FP64 launch keys instead (then
    // srq->band > 0 and rc.band = 0)
    const StreamRecheck *srq;
    const GroupDev *grp;
    int gi;
};

// Queues item (po, yi) for the FP64 recheck, once.
__device__ __forceinline__ void queue_item(const Recheck &rc, int po, int yi) {
    const unsigned bit = 1u << (yi & 31);
    const unsigned old = atomicOr(rc.iflag + (size_t)po * rc.nyw + (yi >> 5), bit);
    if (!(old & bit)) {
        int *d = rc.ilist + 3 * (size_t)atomicAdd(rc.icount, 1);
        d[0] = 0;
        d[1] = yi;
        d[2] = po;
    }
}

// The same for an item of group gi of a batch stream pass: its descriptor
// goes to the FP64 launch key of its row count.
__device__ __forceinline__ void queue_item_g(const StreamRecheck &q, const GroupDev &g, int gi, int po,
                                             int yi) {
    const unsigned bit = 1u << (yi & 31);
    const unsigned old = atomicOr(g.iflag + (size_t)po * g.nyw + (yi >> 5), bit);
    if (!(old & bit)) {
        const int k = g.keyof[yi];
        int *d = q.klist + 3 * ((size_t)q.koff[k] + atomicAdd(q.kcount + k, 1));
        d[0] = gi;
        d[1] = yi;
        d[2] = po;
    }
}

__device__ __forceinline__ void stats_body(const StatsArgs &a, int pl) {
    const double *A0 = a.A + (size_t)(2 * pl) * a.ASUM;
    const double *A1 = a.A + (size_t)(2 * pl + 1) * a.ASUM;
    const int Bh = a.B / 2;
    auto Mxy = [&](int xx, int yy) -> double {
        // the other orientation at the same grid shape (x bins of the first
        // variable, y of the second); MICX_COMPAT_COMBINE_INDEX pairs equal
        // (equipartitioned, optimised) indices instead
        return fmax(A0[a.aoff[yy - 2] + xx - 2], (a.compat & MICX_COMPAT_COMBINE_INDEX)
                                                     ? A1[a.aoff[yy - 2] + xx - 2]
                                                     : A1[a.aoff[xx - 2] + yy - 2]);
    };
    double mic = 0.0;
    for (int yy = 2; yy <= Bh; yy++)
        for (int xx = 2; xx * yy <= a.B; xx++) mic = fmax(mic, Mxy(xx, yy));
    double mas = 0.0, mev = 0.0, mcn = INFINITY;
    for (int yy = 2; yy <= Bh; yy++)
        for (int xx = 2; xx * yy <= a.B; xx++) {
            const double v = Mxy(xx, yy);
            mas = fmax(mas, fabs(v - Mxy(yy, xx)));
            if (xx == 2 || yy == 2) mev = fmax(mev, v);
            if (v >= mic - 1e-12) mcn = fmin(mcn, log2((double)(xx * yy)));
        }
    // Near-tie flag (32-bit form).  Every entry is within bound d of its FP64
    // value, so a cell whose FP64 value reaches MIC - 1e-12 has a 32-bit
    // value of at least MIC - band (band = 2d + 1e-12).  When those cells do
    // not all share one product xy, MCN is not settled by the 32-bit values:
    // the pair is flagged and the items behind each such cell (both
    // orientations) are queued for an FP64 re-run.  Cells below the band stay
    // below MIC - 1e-12 in FP64 as well.
    const double band = a.srq ? a.srq->band : a.rc.band;
    if (band > 0.0) {
        const double lo = mic - band;
        int pmin = 0x7fffffff, pmax = 0;
        for (int yy = 2; yy <= Bh; yy++)
            for (int xx = 2; xx * yy <= a.B; xx++)
                if (Mxy(xx, yy) >= lo) {
                    pmin = min(pmin, xx * yy);
                    pmax = max(pmax, xx * yy);
                }
        if (pmin != pmax) {
            if (a.srq) {
                const int slot = atomicAdd(a.srq->pcount, 1);
                a.srq->plist[2 * slot] = a.gi;
                a.srq->plist[2 * slot + 1] = pl;
            } else {
                a.rc.plist[atomicAdd(a.rc.pcount, 1)] = pl;
            }
            const bool ci = (a.compat & MICX_COMPAT_COMBINE_INDEX) != 0;
            for (int yy = 2; yy <= Bh; yy++)
                for (int xx = 2; xx * yy <= a.B; xx++)
                    if (Mxy(xx, yy) >= lo) {
                        const int y1 = (ci ? yy : xx) - 2;
                        if (a.srq) {
                            queue_item_g(*a.srq, *a.grp, a.gi, 2 * pl, yy - 2);
                            queue_item_g(*a.srq, *a.grp, a.gi, 2 * pl + 1, y1);
                        } else {
                            queue_item(a.rc, 2 * pl, yy - 2);
                            queue_item(a.rc, 2 * pl + 1, y1);
                        }
                    }
        }
    }
    double *o = a.out + (size_t)4 * pl;
    o[0] = mic; o[1] = mas; o[2] = mev; o[3] = mcn;
    if (a.M) {
        const int W = a.W;
        for (int r = 2; r <= W + 1; r++)
            for (int cc = 2; cc <= W + 1; cc++) {
                const size_t q = (size_t)(r - 2) * W + (cc - 2);
                const bool ok = r * cc <= a.B;
                a.M[q] = ok ? Mxy(cc, r) : NAN;
                a.Axy[q] = ok ? A0[a.aoff[r - 2] + cc - 2] : NAN;
                a.Ayx[q] = ok ? A1[a.aoff[r - 2] + cc - 2] : NAN;
            }
    }
}

// The same statistics with one pair per wavefront (the pair calls): the lanes
// take a row's cells, so that the pair's entries are read in runs rather than
// 64 pairs' rows at once, and the four statistics and the near-tie products
// are wave reductions (maxima and minima: exact in any order).
__device__ __forceinline__ double wave_fmax(double v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ double wave_fmin(double v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ int wave_imin(int v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ int wave_imax(int v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ void stats_wave(const StatsArgs &a, int pl, int lane) {
    const double *A0 = a.A + (size_t)(2 * pl) * a.ASUM;
    const double *A1 = a.A + (size_t)(2 * pl + 1) * a.ASUM;
    const int Bh = a.B / 2;
    const bool ci = (a.compat & MICX_COMPAT_COMBINE_INDEX) != 0;
    auto Mxy = [&](int xx, int yy) -> double {
        return fmax(A0[a.aoff[yy - 2] + xx - 2], ci ? A1[a.aoff[yy - 2] + xx - 2] : A1[a.aoff[xx - 2] + yy - 2]);
    };
    // cells (xx, yy), xx * yy <= B: row yy holds xx = 2..B/yy
    double mic = 0.0, mas = 0.0, mev = 0.0;
    for (int yy = 2; yy <= Bh; yy++)
        for (int xx = 2 + lane; xx <= a.B / yy; xx += 64) {
            const double v = Mxy(xx, yy);
            mic = fmax(mic, v);
            mas = fmax(mas, fabs(v - Mxy(yy, xx)));
            if (xx == 2 || yy == 2) mev = fmax(mev, v);
        }
    mic = wave_fmax(mic);
    mas = wave_fmax(mas);
    mev = wave_fmax(mev);
    // MCN over the cells that reach MIC; the near-tie band of the 32-bit form
    // (the rule of stats_body)
    const double band = a.rc.band, lo = mic - band;
    double mcn = INFINITY;
    int pmin = 0x7fffffff, pmax = 0;
    for (int yy = 2; yy <= Bh; yy++)
        for (int xx = 2 + lane; xx <= a.B / yy; xx += 64) {
            const double v = Mxy(xx, yy);
            if (v >= mic - 1e-12) mcn = fmin(mcn, log2((double)(xx * yy)));
            if (band > 0.0 && v >= lo) {
                pmin = min(pmin, xx * yy);
                pmax = max(pmax, xx * yy);
            }
        }
    mcn = wave_fmin(mcn);
    if (band > 0.0) {
        pmin = wave_imin(pmin);
        pmax = wave_imax(pmax);
        if (pmin != pmax) {
            if (lane == 0) a.rc.plist[atomicAdd(a.rc.pcount, 1)] = pl;
            for (int yy = 2; yy <= Bh; yy++)
                for (int xx = 2 + lane; xx <= a.B / yy; xx += 64)
                    if (Mxy(xx, yy) >= lo) {
                        queue_item(a.rc, 2 * pl, yy - 2);
                        queue_item(a.rc, 2 * pl + 1, (ci ? yy : xx) - 2);
                    }
        }
    }
    if (lane == 0) {
        double *o = a.out + (size_t)4 * pl;
        o[0] = mic; o[1] = mas; o[2] = mev; o[3] = mcn;
    }
    if (a.M) {
        const int W = a.W;
        for (int q = lane; q < W * W; q += 64) {
            const int r = q / W + 2, cc = q % W + 2;
            const bool ok = r * cc <= a.B;
            a.M[q] = ok ? Mxy(cc, r) : NAN;
            a.Axy[q] = ok ? A0[a.aoff[r - 2] + cc - 2] : NAN;
            a.Ayx[q] = ok ? A1[a.aoff[r - 2] + cc - 2] : NAN;
        }
    }
}

__global__ __launch_bounds__(256) void k_stats(StatsArgs a) {
    if (a.status && *a.status) return;
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (a.plist) {
        if (k < min(*a.pcount, a.npairs)) stats_wave(a, a.plist[k], lane);
    } else if (k < a.npairs) {
        stats_wave(a, k, lane);
    }
}

__global__ void k_zero(unsigned *p, size_t nwords) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ------------------------------------------------------------------- k_work
// Algorithmic work of a batch (instrumentation).  Per item with K columns, x
// layers and yhat rows: layers 2..x-1 are needed at every target t (t
// candidate sources each) and layer x only at t = K, so the DP has
// (x-2) K(K+1)/2 + K cell updates; the column costs needed are all
// K(K+1)/2 spans when x >= 3, else the 2K-1 spans starting at 0 or ending
// at K; each cost reads yhat+1 table terms.

__global__ void k_work(int npairs, int NY, PairSource ps, const int *xcnt, const int *yhat,
                       const int *K, unsigned long long *counters) {
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c1 = 0, c2 = 0, c3 = 0, c0 = 0;
    if (it < (int64_t)npairs * 2 * NY) {
        const int yi = (int)(it % NY);
        const int po = (int)(it / NY);
        int pi, pj;
        pair_of(ps, po >> 1, pi, pj);
        const int V = (po & 1) ? pi : pj;
        const unsigned long long k = (unsigned long long)K[it];
        const unsigned long long x = (unsigned long long)xcnt[yi];
        const unsigned long long spans = k * (k + 1) / 2;
        c0 = 1;
        c1 = (x - 2) * spans + k;
        c2 = x >= 3 ? spans : 2 * k - 1;
        c3 = (unsigned long long)(yhat[(size_t)V * NY + yi] + 1) * c2;
    }
    for (int off = 32; off > 0; off >>= 1) {
        c0 += __shfl_down(c0, off);
        c1 += __shfl_down(c1, off);
        c2 += __shfl_down(c2, off);
        c3 += __shfl_down(c3, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&counters[0], c0);
        atomicAdd(&counters[1], c1);
        atomicAdd(&counters[2], c2);
        atomicAdd(&counters[3], c3);
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_work(const EquipTables &et, const Geometry &g, PairSource ps, int npairs,
                       const ItemBuffers &ib, unsigned long long *counters, hipStream_t s) {
    const int64_t items = (int64_t)npairs * 2 * g.NY;
    hipLaunchKernelGGL(k_work, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, npairs, g.NY,
                       ps, g.xcnt, et.yhat, ib.K, counters);
    return hipGetLastError();
}

hipError_t launch_geometry(int n, int B, double c, int compat, int NY, int *geo, hipStream_t s) {
    hipLaunchKernelGGL(k_geometry, dim3(1), dim3(64), 0, s, n, B, c, compat, NY, geo);
    return hipGetLastError();
}

hipError_t launch_xlogx(int n, double *xlogx, hipStream_t s) {
    hipLaunchKernelGGL(k_xlogx, dim3((n + 256) / 256), dim3(256), 0, s, n, xlogx);
    return hipGetLastError();
}

hipError_t launch_rank(const void *X, int dtype, int m, int n, RankTables &rt, int *status,
                       hipStream_t s) {
    int N2 = 1;
    while (N2 < n) N2 <<= 1;
    const size_t lds = (size_t)N2 * (8 + 4 + 4);
    const int threads = N2 >= 1024 ? 1024 : (N2 < 64 ? 64 : N2);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = ensure_lds_attr((const void *)k_rank);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank, dim3(m), dim3(threads), lds, s, X, dtype, m, n, N2, rt.perm,
                       rt.gsize, rt.grank, status);
    return hipGetLastError();
}

hipError_t launch_equip(const RankTables &rt, EquipTables &et, hipStream_t s) {
    const int nyb = (et.NY + 63) / 64;
    hipLaunchKernelGGL(k_equip, dim3(rt.m * nyb), dim3(64), (size_t)rt.n * sizeof(int), s, rt.m, rt.n,
                       et.NY, et.NYP, rt.gsize,
                       et.rowof, et.yhat, et.rowstart, et.RS, et.compat);
    return hipGetLastError();
}

hipError_t launch_part(const RankTables &rt, const EquipTables &et, const Geometry &g,
                       PairSource ps, int npairs, ItemBuffers &ib, hipStream_t s) {
    PartArgs a;
    a.n = rt.n; a.NY = g.NY; a.KSUM = g.KSUM; a.ps = ps;
    a.perm = rt.perm; a.gsize = rt.gsize; a.grank = rt.grank; a.rowof = et.rowof; a.NYP = et.NYP;
    a.khat = g.khat; a.koff = g.koff; a.yhat = et.yhat;
    a.cbuf = ib.cbuf; a.sbuf = ib.sbuf; a.K = ib.K; a.k = ib.k; a.src = ib.src; a.Yh = ib.Yh;
    a.lab = ib.lab; a.lab_row = ib.lab_row; a.compat = et.compat;
    a.nitems = 2 * (int64_t)npairs;
    // row counts of several items per wave where one item leaves lanes idle
    // and at most four items share a wave
    a.flat = g.NY >= 22 && g.NY <= 64;
    const int nyb = (g.NY + 63) / 64;
    const int64_t waves = a.flat ? (a.nitems * g.NY + 63) / 64 : 2 * (int64_t)npairs * nyb;
    if (a.flat) {
        if (ib.lab16) hipLaunchKernelGGL(k_part_flat<true>, dim3((unsigned)waves), dim3(64), 0, s, a);
        else hipLaunchKernelGGL(k_part_flat<false>, dim3((unsigned)waves), dim3(64), 0, s, a);
    } else if (ib.lab16) {
        hipLaunchKernelGGL(k_part<true>, dim3((unsigned)waves), dim3(64), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_part<false>, dim3((unsigned)waves), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_stats(const Geometry &g, int npairs, const ItemBuffers &ib, double *out,
                        double *M, double *Axy, double *Ayx, hipStream_t s, const Recheck *flag,
                        const int *plist, const int *pcount, const int *status) {
    StatsArgs a;
    a.npairs = npairs; a.B = g.B; a.NY = g.NY; a.W = g.W; a.ASUM = g.ASUM;
    a.aoff = g.aoff; a.A = ib.A; a.out = out; a.M = M; a.Axy = Axy; a.Ayx = Ayx; a.compat = g.compat;
    a.rc = flag ? *flag : Recheck();
    a.plist = plist; a.pcount = pcount; a.status = status;
    a.srq = nullptr; a.grp = nullptr; a.gi = 0;
    hipLaunchKernelGGL(k_stats, dim3((npairs + 3) / 4), dim3(256), 0, s, a);   // one pair per wavefront
    return hipGetLastError();
}

// Sum (mod 2^64) of the bit patterns of the entries A[po * ASUM + off + l],
// l < cnt, over all npo items: an order-free fingerprint of one row count's
// results (the autotuner checks that every launch shape gives the same bits).
__global__ void k_checksum(const double *A, int npo, int ASUM, int off, int cnt, unsigned long long *sum) {
    unsigned long long acc = 0;
    const int64_t total = (int64_t)npo * cnt;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t po = i / cnt;
        acc += (unsigned long long)__double_as_longlong(A[po * ASUM + off + (i - po * cnt)]);
    }
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(sum, acc);
}

hipError_t launch_checksum(const double *A, int npo, int ASUM, int off, int cnt, unsigned long long *sum,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_checksum, dim3(256), dim3(256), 0, s, A, npo, ASUM, off, cnt, sum);
    return hipGetLastError();
}

__global__ void k_put_group(DpGroup g, DpGroup *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = g;
}

__global__ void k_range_items(int yi_lo, int npo, int64_t total, int *items) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / npo;
        items[3 * i] = 0;
        items[3 * i + 1] = yi_lo + (int)c;
        items[3 * i + 2] = (int)(i - c * npo);
    }
}

hipError_t launch_range_items(int yi_lo, int ncls, int npo, int *items, hipStream_t s) {
    const int64_t total = (int64_t)ncls * npo;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_range_items, dim3((unsigned)blocks), dim3(256), 0, s, yi_lo, npo, total, items);
    return hipGetLastError();
}

hipError_t launch_put_group(const DpGroup &g, DpGroup *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_put_group, dim3(1), dim3(64), 0, s, g, dst);
    return hipGetLastError();
}

// T[j] = round(S * j ln j) mod 2^32 for several row-count classes at once
// (blockIdx.y = class).
__global__ void k_fxtables(int n, FxScales sc, const double *xlogx, uint32_t *tab, size_t stride) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j <= n) tab[(size_t)sc.cls[c] * stride + j] = (uint32_t)(unsigned long long)__double2ll_rn(sc.scale[c] * xlogx[j]);
}

hipError_t launch_fxtables(int n, const FxScales &sc, int count, const double *xlogx, uint32_t *tab,
                           size_t stride, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fxtables, dim3((n + 256) / 256, count), dim3(256), 0, s, n, sc, xlogx, tab, stride);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t nwords, hipStream_t s) {
    if (nwords == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((nwords + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned *)p, nwords);
    return hipGetLastError();
}

int device_cus(int device) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return 256;
    return p.multiProcessorCount;
}

// ------------------------------------------------------ batch gather/scatter
// Variables of a batch, scattered over a packed buffer, are copied into the
// rows of an nv x n matrix (one workgroup per variable); results computed in
// group order go back to the caller's pair order.

template <class E>
__global__ void k_gather(const E *src, const int64_t *offs, int n, E *dst) {
    const int v = blockIdx.x;
    const E *s = src + offs[v];
    E *d = dst + (size_t)v * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
}

__global__ void k_scatter_rows(const double *src, const int64_t *idx, int64_t rows, double *dst,
                               const int *status) {
    if (status && *status) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * rows) return;
    dst[4 * idx[k >> 2] + (k & 3)] = src[k];
}

hipError_t launch_gather(const void *src, int esize, const int64_t *offs, int nv, int n, void *dst,
                         hipStream_t s) {
    if (esize == 8)
        hipLaunchKernelGGL(k_gather<uint64_t>, dim3(nv), dim3(256), 0, s, (const uint64_t *)src, offs,
                           n, (uint64_t *)dst);
    else
        hipLaunchKernelGGL(k_gather<uint32_t>, dim3(nv), dim3(256), 0, s, (const uint32_t *)src, offs,
                           n, (uint32_t *)dst);
    return hipGetLastError();
}

hipError_t launch_scatter_rows(const double *src, const int64_t *idx, int64_t rows, double *dst,
                               hipStream_t s, const int *status) {
    const int64_t th = 4 * rows;
    hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((th + 255) / 256)), dim3(256), 0, s, src, idx,
                       rows, dst, status);
    return hipGetLastError();
}

// ------------------------------------------------ fused per-group stages
// A batch pass runs each per-group stage as one launch over all its groups:
// block b serves group map[b].x with the block index map[b].y that the
// group's own launch would give it.

__global__ void k_gather_g(const unsigned char *data, int esize, const GroupDev *G, const int2 *map) {
    const int2 m = map[blockIdx.x];
    const GroupDev &g = G[m.x];
    const unsigned char *src = data + (size_t)g.offs[m.y] * esize;
    unsigned char *dst = (unsigned char *)g.X + (size_t)m.y * g.n * esize;
    if (esize == 8) {
        for (int i = threadIdx.x; i < g.n; i += blockDim.x) ((uint64_t *)dst)[i] = ((const uint64_t *)src)[i];
    } else {
        for (int i = threadIdx.x; i < g.n; i += blockDim.x) ((uint32_t *)dst)[i] = ((const uint32_t *)src)[i];
    }
}

__global__ __launch_bounds__(1024) void k_rank_g(const GroupDev *G, const int2 *map, int dtype, int *status) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 m = map[blockIdx.x];
    const GroupDev &g = G[m.x];
    int N2 = 1;
    while (N2 < g.n) N2 <<= 1;
    rank_body(g.X, dtype, m.y, g.n, N2, g.perm, g.gsize, g.grank, status, smem);
}

__global__ __launch_bounds__(64) void k_equip_g(const GroupDev *G, const int2 *map) {
    extern __shared__ int gsl[];
    const int2 m = map[blockIdx.x];
    const GroupDev &g = G[m.x];
    const int nyb = (g.NY + 63) / 64;
    equip_body(m.y / nyb, m.y % nyb, g.n, g.NY, g.NYP, g.gsize, g.rowof, g.yhat, nullptr, g.NY + 2, gsl,
               g.compat);
}

__global__ __launch_bounds__(64) void k_part_g(const GroupDev *G, const int2 *map) {
    __shared__ __align__(16) unsigned char tile[64 * PART_TILE];
    const int2 m = map[blockIdx.x];
    const GroupDev &g = G[m.x];
    PartArgs a;
    a.n = g.n; a.NY = g.NY; a.NYP = g.NYP; a.KSUM = g.KSUM;
    a.ps.pairs = g.pairs; a.ps.p0 = 0; a.ps.m = g.nv;
    a.perm = g.perm; a.gsize = g.gsize; a.grank = g.grank; a.rowof = g.rowof;
    a.khat = g.khat; a.koff = g.koff; a.yhat = g.yhat;
    a.cbuf = g.cbuf; a.sbuf = g.sbuf; a.K = g.K; a.k = g.k; a.src = g.src; a.Yh = g.Yh;
    a.lab = g.lab; a.lab_row = g.lab_row; a.compat = g.compat;
    a.nitems = 2 * (int64_t)g.npairs;
    a.flat = 0;   // one item per wave (the map names it)
    if (g.lab16) part_dispatch<true>(a, m.y, tile);
    else part_dispatch<false>(a, m.y, tile);
}

__device__ __forceinline__ void stats_g_pair(const GroupDev *G, int gi, int pl, const StreamRecheck *q) {
    const GroupDev &g = G[gi];
    StatsArgs a;
    a.npairs = g.npairs; a.B = g.B; a.NY = g.NY; a.W = g.W; a.ASUM = g.ASUM;
    a.aoff = g.aoff; a.A = g.A; a.out = g.out; a.M = nullptr; a.Axy = nullptr; a.Ayx = nullptr;
    a.compat = g.compat;
    a.rc = Recheck();
    a.plist = nullptr; a.pcount = nullptr; a.status = nullptr;
    a.srq = q && q->band > 0.0 ? q : nullptr;
    a.grp = &g;
    a.gi = gi;
    stats_body(a, pl);
}

// 64 pairs per block: map[b].y is the group's first pair of the block
__global__ void k_stats_g(const GroupDev *G, const int2 *map, StreamRecheck q, const int *status) {
    if (status && *status) return;
    const int2 m = map[blockIdx.x];
    const int pl = m.y + threadIdx.x;
    if (pl >= G[m.x].npairs) return;
    stats_g_pair(G, m.x, pl, &q);
}

// the flagged pairs of a pass, (group, pair) each
__global__ void k_stats_g_list(const GroupDev *G, const int *plist, const int *pcount, int cap,
                               const int *status) {
    if (status && *status) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= min(*pcount, cap)) return;
    stats_g_pair(G, plist[2 * k], plist[2 * k + 1], nullptr);
}

hipError_t launch_gather_g(const void *data, int esize, const GroupDev *G, const int2 *map, int blocks,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_gather_g, dim3(blocks), dim3(256), 0, s, (const unsigned char *)data, esize, G, map);
    return hipGetLastError();
}

hipError_t launch_rank_g(const GroupDev *G, const int2 *map, int blocks, int nmax, int dtype,
                         int *status, hipStream_t s) {
    int N2 = 1;
    while (N2 < nmax) N2 <<= 1;
    const size_t lds = (size_t)N2 * (8 + 4 + 4);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = ensure_lds_attr((const void *)k_rank_g);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_g, dim3(blocks), dim3(1024), lds, s, G, map, dtype, status);
    return hipGetLastError();
}

hipError_t launch_equip_g(const GroupDev *G, const int2 *map, int blocks, int nmax, hipStream_t s) {
    hipLaunchKernelGGL(k_equip_g, dim3(blocks), dim3(64), (size_t)nmax * sizeof(int), s, G, map);
    return hipGetLastError();
}

hipError_t launch_part_g(const GroupDev *G, const int2 *map, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_part_g, dim3(blocks), dim3(64), 0, s, G, map);
    return hipGetLastError();
}

hipError_t launch_stats_g(const GroupDev *G, const int2 *map, int blocks, hipStream_t s,
                          const StreamRecheck *flag, const int *status) {
    const StreamRecheck q = flag ? *flag : StreamRecheck();
    hipLaunchKernelGGL(k_stats_g, dim3(blocks), dim3(64), 0, s, G, map, q, status);
    return hipGetLastError();
}

hipError_t launch_stats_g_list(const GroupDev *G, const int *plist, const int *pcount, int cap,
                               hipStream_t s, const int *status) {
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stats_g_list, dim3((cap + 127) / 128), dim3(128), 0, s, G, plist, pcount, cap,
                       status);
    return hipGetLastError();
}

}  // namespace micx
