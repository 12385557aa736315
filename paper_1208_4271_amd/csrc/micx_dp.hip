// micx_dp.hip -- the OptimizeXAxis dynamic program (Albanese et al. 2012,
// Appendix A item 10) for every (pair, orientation) item of one row count y.
//
// Per item (one wavefront):
//  * item 10a: cumulative counts N[t][r] -- points among the first t
//    (super)clumps that lie in row r -- built in LDS from the superclump ends
//    and the row labels (a flag scan gives each point's superclump, LDS
//    atomics count, a wavefront scan accumulates over t);
//  * item 10b: the column cost h(s,t) = L[m] - sum_r L[n_r], m = e_t - e_s,
//    n_r = N[t][r] - N[s][r], L[j] = j ln j: the span's point count times its
//    row entropy, computed once per (s,t) and used for every layer;
//  * the DP: G_1(t) = h(0,t), G_l(t) = min_{0 <= s < t} G_{l-1}(s) + h(s,t)
//    with G_{l-1}(0) = 0.  G_l(K) is the least sum of column costs over
//    partitions into at most l columns, and I_l = H(Q) - G_l(K)/n.
//
// Layout.  Lanes own targets t, T per lane (a chunk of 64T targets).  The
// layers of a pass (up to NL) live in registers, as do the target's
// cumulative counts (up to YR rows).  Sources from earlier chunks are final:
// their layer values are staged from the item's G table (global, layer-major)
// into LDS, SB sources at a time, and read back as wavefront-uniform
// broadcasts.  Sources inside the chunk are taken in order; the lane that
// owns a source publishes its layer values through LDS.
#include <algorithm>

#include "micx_device.h"

namespace micx {

struct DpArgs {
    int n, NY, KSUM, ASUM;
    int yi, x, RS, KS;           // class: row count y = yi+2, x(y), rec stride y+1, G row stride
    int nitems, npairs, SB;      // items of the class = 2 * npairs
    PairSource ps;
    const int *perm, *grank;
    const uint16_t *rowof;
    const int *yhat, *koff, *aoff;
    const int *cbuf, *sbuf, *K, *src;
    double *A;
    const double *xlogx;
    double *scratch;
    size_t slot;                 // doubles of G table per wavefront
    int lds_L, lds_stage, lds_pub, lds_wave;
};

template <int NL, int YR, int T>
__global__ __launch_bounds__(256) void k_dp64(DpArgs a) {
    constexpr int NLP = (NL + 1) & ~1;
    constexpr int YA = YR > 0 ? YR : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = a.n, NY = a.NY, RS = a.RS, KS = a.KS, x = a.x, yi = a.yi, SB = a.SB;
    const int sbs = __builtin_ctz(SB);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double *L = (double *)smem;
    for (int j = threadIdx.x; j <= n; j += blockDim.x) L[j] = a.xlogx[j];
    __syncthreads();
    unsigned char *wb = smem + a.lds_L + (size_t)wv * a.lds_wave;
    double *stage = (double *)wb;                              // SB x NLP, or n flag bytes
    double *pub = (double *)(wb + a.lds_stage);                // NLP
    int *rec = (int *)(wb + a.lds_stage + a.lds_pub);          // (K+1) x RS: e_t, N_t[0..yhat-1]
    const int wpb = blockDim.x >> 6;
    const int gw = blockIdx.x * wpb + wv, nw = gridDim.x * wpb;
    double *G = a.scratch + (size_t)gw * a.slot;

    for (int po = gw; po < a.nitems; po += nw) {
        const int o = po & 1, pl = po >> 1;
        int pi, pj;
        pair_of(a.ps, pl, pi, pj);
        const int U = o ? pj : pi, V = o ? pi : pj;
        const size_t it = (size_t)po * NY + yi;
        const int K = a.K[it];
        const int yh = a.yhat[(size_t)V * NY + yi];
        const int *ends = (a.src[it] ? a.sbuf : a.cbuf) + (size_t)po * a.KSUM + a.koff[yi];

        // ---- cumulative counts (item 10a) ----
        unsigned char *F = (unsigned char *)stage;
        for (int k = lane; k < (K + 1) * RS; k += 64) rec[k] = 0;
        for (int p = lane; p < n; p += 64) F[p] = 0;
        wave_sync();
        for (int t = lane; t < K; t += 64) {
            const int et = ends[t];
            rec[(t + 1) * RS] = et;
            if (t + 1 < K) F[et] = 1;
        }
        wave_sync();
        {
            const int *permU = a.perm + (size_t)U * n;
            const int *grV = a.grank + (size_t)V * n;
            const uint16_t *rowV = a.rowof + (size_t)V * n * NY + yi;
            int carry = 0;
            for (int p0 = 0; p0 < n; p0 += 64) {
                const int p = p0 + lane;
                const int f = p < n ? (int)F[p] : 0;
                const int incl = wave_incl_scan(f, lane);
                if (p < n) {
                    const int g = grV[permU[p]];
                    const int r = rowV[(size_t)g * NY];
                    atomicAdd(&rec[(carry + incl + 1) * RS + 1 + r], 1);
                }
                carry += __shfl(incl, 63, 64);
            }
        }
        wave_sync();
        for (int r = 0; r < yh; r++) {
            int c2 = 0;
            for (int t0 = 1; t0 <= K; t0 += 64) {
                const int t = t0 + lane;
                const int v = t <= K ? rec[t * RS + 1 + r] : 0;
                const int incl = wave_incl_scan(v, lane) + c2;
                if (t <= K) rec[t * RS + 1 + r] = incl;
                c2 = __shfl(incl, 63, 64);
            }
        }
        wave_sync();

        // ---- DP (item 10b costs, OptimizeXAxis recurrence) ----
        for (int l0 = 2; l0 <= x; l0 += NL) {
            const int nl = min(NL, x - l0 + 1);
            const int nlp = (nl + 1) & ~1;
            for (int c0 = 0; c0 < K; c0 += 64 * T) {
                int tt[T], et[T], Nt[T][YA];
                double g[T][NLP], gprev[T];
#pragma unroll
                for (int j = 0; j < T; j++) {
                    tt[j] = c0 + 64 * j + lane + 1;
                    const int tc = tt[j] <= K ? tt[j] : K;
                    const int *rt = rec + tc * RS;
                    et[j] = rt[0];
                    double h0 = L[et[j]];
                    if (YR > 0) {
#pragma unroll
                        for (int r = 0; r < YA; r++) {
                            if (r < yh) {
                                Nt[j][r] = rt[1 + r];
                                h0 -= L[Nt[j][r]];
                            } else {
                                Nt[j][r] = 0;
                            }
                        }
                    } else {
                        for (int r = 0; r < yh; r++) h0 -= L[rt[1 + r]];
                    }
                    gprev[j] = l0 == 2 ? h0 : G[(size_t)(l0 - 1) * KS + tc];
#pragma unroll
                    for (int q = 0; q < NLP; q++) g[j][q] = h0;
                }
                // sources of earlier chunks, SB at a time through LDS
                for (int sb = 1; sb <= c0; sb += SB) {
                    const int ns = min(SB, c0 - sb + 1);
                    for (int k = lane; k < nlp * SB; k += 64) {
                        const int q = k >> sbs, sl = k & (SB - 1);
                        stage[sl * NLP + q] =
                            (sl < ns && q < nl) ? G[(size_t)(l0 - 1 + q) * KS + sb + sl] : 0.0;
                    }
                    wave_sync();
                    for (int sl = 0; sl < ns; sl++) {
                        const int *rs = rec + (sb + sl) * RS;
                        const int es = rs[0];
                        double hs[T];
#pragma unroll
                        for (int j = 0; j < T; j++) hs[j] = L[et[j] - es];
                        if (YR > 0) {
#pragma unroll
                            for (int r = 0; r < YA; r++) {
                                if (r < yh) {
                                    const int nsr = rs[1 + r];
#pragma unroll
                                    for (int j = 0; j < T; j++) hs[j] -= L[Nt[j][r] - nsr];
                                }
                            }
                        } else {
                            for (int r = 0; r < yh; r++) {
                                const int nsr = rs[1 + r];
#pragma unroll
                                for (int j = 0; j < T; j++) {
                                    const int tc = tt[j] <= K ? tt[j] : K;
                                    hs[j] -= L[rec[tc * RS + 1 + r] - nsr];
                                }
                            }
                        }
                        const double *gs = stage + sl * NLP;
#pragma unroll
                        for (int q = 0; q < NLP; q += 2) {
                            if (q < nl) {
                                const double2 v = *(const double2 *)(gs + q);
#pragma unroll
                                for (int j = 0; j < T; j++) {
                                    g[j][q] = fmin(g[j][q], v.x + hs[j]);
                                    g[j][q + 1] = fmin(g[j][q + 1], v.y + hs[j]);
                                }
                            }
                        }
                    }
                    wave_sync();
                }
                // sources inside the chunk, in order
#pragma unroll
                for (int jo = 0; jo < T; jo++) {
                    const int sbeg = c0 + 64 * jo + 1;
                    const int send = min(c0 + 64 * jo + 64, K);
                    for (int s = sbeg; s <= send; s++) {
                        const int ln = s - sbeg;
                        if (lane == ln) {
                            pub[0] = gprev[jo];
#pragma unroll
                            for (int q = 1; q < NLP; q++) pub[q] = g[jo][q - 1];
                        }
                        wave_sync();
                        const int *rs = rec + s * RS;
                        const int es = rs[0];
#pragma unroll
                        for (int j = jo; j < T; j++) {
                            if (j == jo && lane <= ln) continue;
                            double hs = L[et[j] - es];
                            if (YR > 0) {
#pragma unroll
                                for (int r = 0; r < YA; r++)
                                    if (r < yh) hs -= L[Nt[j][r] - rs[1 + r]];
                            } else {
                                const int tc = tt[j] <= K ? tt[j] : K;
                                for (int r = 0; r < yh; r++) hs -= L[rec[tc * RS + 1 + r] - rs[1 + r]];
                            }
#pragma unroll
                            for (int q = 0; q < NLP; q += 2) {
                                if (q < nl) {
                                    const double2 v = *(const double2 *)(pub + q);
                                    g[j][q] = fmin(g[j][q], v.x + hs);
                                    g[j][q + 1] = fmin(g[j][q + 1], v.y + hs);
                                }
                            }
                        }
                        wave_sync();
                    }
                }
                // the chunk's layers become sources for later chunks
#pragma unroll
                for (int j = 0; j < T; j++) {
                    if (tt[j] <= K) {
                        if (l0 == 2) G[(size_t)KS + tt[j]] = gprev[j];
#pragma unroll
                        for (int q = 0; q < NLP; q++)
                            if (q < nl) G[(size_t)(l0 + q) * KS + tt[j]] = g[j][q];
                    }
                }
                global_sync();
            }
        }

        // ---- I_l = (L[n] - sum_r L[q_r] - G_l(K)) / n, normalised by ln min(l, yhat) ----
        double sq = 0.0;
        for (int r = 0; r < yh; r++) sq += L[rec[K * RS + 1 + r]];
        double *Aout = a.A + (size_t)po * a.ASUM + a.aoff[yi];
        for (int l = 2 + lane; l <= x; l += 64) {
            const double I = (L[n] - sq - G[(size_t)l * KS + K]) / (double)n;
            const int norm = min(l, yh);
            Aout[l - 2] = norm >= 2 ? I / log((double)norm) : 0.0;
        }
        wave_sync();
    }
}

// ------------------------------------------------------------------ dispatch

namespace {

typedef void (*dp_kernel_t)(DpArgs);

template <int NL, int YR>
dp_kernel_t pick_T(int T) {
    (void)T;
    if constexpr (NL <= 4) return k_dp64<NL, YR, 1>;
    else return k_dp64<NL, YR, 2>;
}

template <int NL>
dp_kernel_t pick_YR(int YR, int T) {
    switch (YR) {
        case 2: return pick_T<NL, 2>(T);
        case 4: return pick_T<NL, 4>(T);
        case 8: return pick_T<NL, 8>(T);
        case 16: return pick_T<NL, 16>(T);
        case 40: return pick_T<NL, 40>(T);
        default: return pick_T<NL, 0>(T);
    }
}

dp_kernel_t pick(int NL, int YR, int T) {
    switch (NL) {
        case 1: return pick_YR<1>(YR, T);
        case 2: return pick_YR<2>(YR, T);
        case 4: return pick_YR<4>(YR, T);
        case 8: return pick_YR<8>(YR, T);
        case 12: return pick_YR<12>(YR, T);
        case 16: return pick_YR<16>(YR, T);
        case 24: return pick_YR<24>(YR, T);
        default: return pick_YR<36>(YR, T);
    }
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
    static const int NLS[] = {1, 2, 4, 8, 12, 16, 24, 36};
    static const int YRS[] = {2, 4, 8, 16, 40};
    DpPlan p;
    const int y = yi + 2, x = g.B / y;
    const int kh = g.khat_host[yi];
    p.NL = round_up_in(x - 1, NLS, 8, 36);
    p.YR = round_up_in(y, YRS, 5, 0);
    p.T = p.NL <= 4 ? 1 : 2;
    const int NLP = (p.NL + 1) & ~1;
    p.KS = kh + 1;
    p.RS = y + 1;
    p.x = x;
    p.slot = (size_t)(x + 1) * (size_t)p.KS;
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
