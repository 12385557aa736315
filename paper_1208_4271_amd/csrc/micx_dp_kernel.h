// micx_dp_kernel.h -- the OptimizeXAxis dynamic program (Albanese et al. 2012,
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
//    partitions into at most l columns, and I_l = H(Q) - G_l(K)/n.  Layers
//    2..x-1 are needed at every target; layer x only at t = K.
//
// Value types.  V = double runs the DP in FP64.  V = uint32_t runs it in
// 32-bit fixed point: the table holds T[j] = round(S * j ln j) mod 2^32 for a
// per-row-count scale S chosen so that every candidate G_{l-1}(s) + h(s,t)
// (at most e_t ln(yhat) in exact arithmetic) stays below 2^32.  Integer sums
// are exact, so the DP finds the exact optimum of the rounded costs; each
// cost is off by at most (yhat+1)/2 units, so G_l(K)/S is within
// l (yhat+1) / (2S) of the true optimum.  The host uses this form only where
// that bound, in units of M, is below the requested tolerance.
//
// Layout.  Lanes own targets t, T per lane (a chunk of 64T targets).  The
// layers of a pass (up to NL) live in registers, as do the target's
// cumulative counts (up to YR rows).  Counts are kept as byte offsets into the
// L table (count times sizeof(V)), so the table address of a cost term is one
// difference of two counts.  Sources from earlier chunks are final:
// their layer values are staged from the item's G table (global, layer-major)
// into LDS, SB sources at a time, and read back as wavefront-uniform
// broadcasts.  Sources inside the chunk are taken in order; the lane that
// owns a source broadcasts its layer values through scalar registers
// (readlane).
#pragma once

#include <stdlib.h>

#include <algorithm>
#include <type_traits>

#include "micx_device.h"

namespace micx {

struct DpArgs {
    int n, NY, KSUM, ASUM;
    int yi, x, RS, KS;           // class: row count y = yi+2, x(y), count-record stride, G row stride
    int nitems, npairs, SB;      // items of the class = 2 * npairs
    PairSource ps;
    const int *koff, *aoff;
    const int *cbuf, *sbuf, *K, *src, *Yh;   // per item: ends, K, which ends, yhat
    const unsigned char *lab;    // row labels in column order, [item][y-2][p]
    size_t lab_row;
    int lab16;
    double *A;
    const double *xlogx;         // FP64 table j ln j
    const uint32_t *fxtab;       // fixed-point table of the class (uint32 form)
    double inv_scale;            // 1 / S (uint32 form)
    void *scratch;
    size_t slot_bytes;           // G table bytes per wavefront
    // items from several groups of a batch stream (the GR instances): 3 ints
    // per item (group, y-2, pair*2+orientation); n is then the largest n of
    // the launch
    const DpGroup *groups;
    const int *gitems;
    int compat;                  // MICX_COMPAT_* flags (MICX_COMPAT_NORM_BY_Y acts here)
    int lds_L, lds_stage, lds_wave;
    // the FP64 recheck of near-tied items: a list of the class's items
    // (pair*2+orientation; the GR instances take gitems) and its length, both
    // in device memory, or null: every item
    const int *ilist, *icount;
    int *dbg;                    // debug instances: the count tables, (KS*RS) ints per item
    // cooperative instances (one item per workgroup): the shared region after
    // the table holds the count records (lds_rec bytes), then the chunk
    // completion flags, the per-wave minima and the abort flag, then the
    // superclump flags of the count-table build (lds_flags bytes); each
    // wave's staging buffer follows.  status: bit 1 set if a wait gave up.
    int lds_rec, lds_flags;
    int *status;
};

// A wait on another wave's chunk gives up after this many sleeps (about 0.5 s,
// hundreds of times a chunk's time): the kernel then ends in bounded time
// and the status word reports it.
constexpr int kCoSpinMax = 1 << 23;

template <class V> struct DpVal;

template <> struct DpVal<double> {
    static constexpr int PK = 2;    // values per 16-byte LDS access
    static constexpr int SP = 1;    // sources merged per minimum
    __device__ static double mn(double a, double b) { return fmin(a, b); }
    __device__ static double big() { return INFINITY; }
    __device__ static double real(double g, double) { return g; }
    // value of lane `src` (uniform) in every lane
    __device__ static double bcast(double v, int src) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    }
};

template <> struct DpVal<uint32_t> {
    static constexpr int PK = 4;
    static constexpr int SP = 2;    // two sources per v_min3_u32
    __device__ static uint32_t mn(uint32_t a, uint32_t b) { return a < b ? a : b; }
    __device__ static uint32_t big() { return 0xffffffffu; }
    __device__ static double real(uint32_t g, double inv_scale) { return (double)g * inv_scale; }
    __device__ static uint32_t bcast(uint32_t v, int src) { return (uint32_t)__builtin_amdgcn_readlane((int)v, src); }
};

// Build-time tuning knob: MICX_DP_GROUP (16-byte layer packs per scheduling
// group).
#ifndef MICX_DP_GROUP
#define MICX_DP_GROUP 4
#endif

// No occupancy target is set: the compiler's own register allocation was
// measured faster than every target that compiles without spills, and the
// build rejects any DP kernel that spills (spill code placed inside a
// divergent region leaves the slots of inactive lanes unwritten).

template <class V>
struct alignas(16) Pack {
    V v[DpVal<V>::PK];
};

// DBG: a debug instance that writes each item's cumulative count table (as
// counts) to a.dbg and skips the DP (bit-exact readback of item 10a).
// CO: a cooperative instance -- the waves of a workgroup share one item: the
// count table is built once, the chunks of every pass are dealt round-robin
// to the waves, and a chunk's sources from earlier chunks are staged as soon
// as those chunks' completion flags (LDS) show them final; each chunk's own
// triangle stays in order.  For items with thousands of superclumps, whose
// one-wave time would otherwise bound a whole launch.
template <class V, int NL, int YR, int T, bool GR, bool DBG = false, bool CO = false>
__global__ __launch_bounds__((CO && sizeof(V) == 4) ? 512 : 256) void k_dp(DpArgs a) {
    using DV = DpVal<V>;
    constexpr int PK = DV::PK;
    constexpr int NLP = (NL + PK - 1) / PK * PK;
    constexpr bool FX = std::is_same<V, uint32_t>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nmax = a.n, SB = a.SB;
    const int sbs = __builtin_ctz(SB);
    // the wavefront index is uniform across the wave; saying so keeps the item
    // index, its sizes and pointers in scalar registers and its branches scalar
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    V *L = (V *)smem;
    constexpr int VB = (int)sizeof(V);
    // Table reads by LDS address.  A target's counts are kept with the
    // table's LDS base added, so the address of a cost term is one difference.
    typedef __attribute__((address_space(3))) const V *lds_v;
    const int lbase = (int)(uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char *)smem;
    auto LA = [&](int addr) -> V { return *(lds_v)(uintptr_t)(uint32_t)addr; };
    auto LB = [&](int b) -> V { return LA(lbase + b); };     // entry at byte offset b
    for (int j = threadIdx.x; j <= nmax; j += blockDim.x) {
        if constexpr (FX) L[j] = a.fxtab[j];
        else L[j] = a.xlogx[j];
    }
    __syncthreads();
    const int wpb = blockDim.x >> 6;
    V *stage;                                                  // SB x NLP, or labels and flags
    int *rec;                                                  // (K+1) x RS: e_t, N_t[0..RS-2]
    int *done = nullptr, *abort_flag = nullptr;                // cooperative: chunk flags
    V *wmin = nullptr;                                         // cooperative: per-wave minima
    unsigned char *coflags = nullptr;                          // cooperative: superclump flags
    if constexpr (CO) {
        unsigned char *sh = smem + a.lds_L;
        rec = (int *)sh;
        done = (int *)(sh + a.lds_rec);
        wmin = (V *)(sh + a.lds_rec + 4 * kCoChunks);
        abort_flag = (int *)(sh + a.lds_rec + 4 * kCoChunks + 8 * 16);
        coflags = sh + a.lds_rec + kCoMeta;
        stage = (V *)(sh + a.lds_rec + kCoMeta + a.lds_flags + (size_t)wv * a.lds_stage);
        if (threadIdx.x == 0) *abort_flag = 0;
    } else {
        unsigned char *wb = smem + a.lds_L + (size_t)wv * a.lds_wave;
        stage = (V *)wb;
        rec = (int *)(wb + a.lds_stage);
    }
    const int gw = CO ? blockIdx.x : blockIdx.x * wpb + wv;
    const int nw = CO ? gridDim.x : gridDim.x * wpb;
    V *G = (V *)((unsigned char *)a.scratch + (size_t)gw * a.slot_bytes);
    if constexpr (CO) __syncthreads();

    int nitems = a.nitems;
    if (a.icount) nitems = min(nitems, __builtin_amdgcn_readfirstlane(*a.icount));
    for (int wi = gw; wi < nitems; wi += nw) {
        // the item: its sample count n, columns x, G-table and count-record
        // strides, superclump count K, rows yhat and buffers
        int n, x, KS, RS, K, yh, ycls;
        const int *ends;
        const unsigned char *lb8;
        bool l16;
        double *Aout;
        if constexpr (GR) {
            const int *d = a.gitems + 3 * (size_t)wi;
            const int gi = __builtin_amdgcn_readfirstlane(d[0]);
            const int yi = __builtin_amdgcn_readfirstlane(d[1]);
            const int po = __builtin_amdgcn_readfirstlane(d[2]);
            const DpGroup &gr = a.groups[gi];
            const size_t it = (size_t)po * gr.NY + yi;
            n = gr.n;
            ycls = yi + 2;
            x = gr.xcnt[yi];
            KS = gr.khat[yi] + 1;
            RS = rec_stride(YR, ycls);
            K = __builtin_amdgcn_readfirstlane(gr.K[it]);
            yh = __builtin_amdgcn_readfirstlane(gr.Yh[it]);
            ends = (gr.src[it] ? gr.sbuf : gr.cbuf) + (size_t)po * gr.KSUM + gr.koff[yi];
            lb8 = gr.lab + it * gr.lab_row;
            l16 = gr.lab16 != 0;
            Aout = gr.A + (size_t)po * gr.ASUM + gr.aoff[yi];
        } else {
            const int po = a.ilist ? __builtin_amdgcn_readfirstlane(a.ilist[wi]) : wi;
            const int yi = a.yi, NY = a.NY;
            const size_t it = (size_t)po * NY + yi;
            n = a.n;
            ycls = yi + 2;
            x = a.x;
            KS = a.KS;
            RS = a.RS;
            K = __builtin_amdgcn_readfirstlane(a.K[it]);
            yh = __builtin_amdgcn_readfirstlane(a.Yh[it]);
            ends = (a.src[it] ? a.sbuf : a.cbuf) + (size_t)po * a.KSUM + a.koff[yi];
            lb8 = a.lab + it * a.lab_row;
            l16 = a.lab16 != 0;
            Aout = a.A + (size_t)po * a.ASUM + a.aoff[yi];
        }

        // ---- cumulative counts (item 10a); rows beyond yhat stay 0 ----
        // A flag per superclump start gives each point its superclump; the
        // point's row label (stored in column order by the partition kernel)
        // selects the count, and LDS atomics count.  (Cooperative: wave 0
        // builds the shared table while the others wait.)
        unsigned char *F = CO ? coflags : (unsigned char *)stage;
        if (CO && wv != 0) {
            // the other waves skip the build
        } else if constexpr (NL < 20) {
            // Every lane takes a run of consecutive points: one 16-byte load
            // of labels (the first loads are issued before the table is
            // cleared); a wavefront prefix sum of the lanes' flag counts
            // gives each point its superclump.  (Passes of 20 layers or more
            // keep the scan below: this one's registers would lower their
            // occupancy, and the scan is a few percent of their time.)
            const int lbytes = l16 ? 2 * n : n;
            constexpr int LG = 4;                       // label loads in flight per lane
            uint4 lv[LG];
            auto load_labels = [&](int c0) {
#pragma unroll
                for (int i = 0; i < LG; i++) {
                    const int off = ((c0 + i) * 64 + lane) * 16;
                    lv[i] = off < lbytes ? *(const uint4 *)(lb8 + off) : make_uint4(0, 0, 0, 0);
                }
            };
            load_labels(0);
            {
                const uint4 z = make_uint4(0, 0, 0, 0);
                for (int k = lane; k < (n + 15) >> 4; k += 64) ((uint4 *)F)[k] = z;
                for (int k = lane; k < ((K + 1) * RS + 3) >> 2; k += 64) ((uint4 *)rec)[k] = z;
            }
            wave_sync();
            for (int t = lane; t < K; t += 64) {
                const int et = ends[t];
                rec[(t + 1) * RS] = et * VB;
                if (t + 1 < K) F[et] = 1;
            }
            wave_sync();
            {
                // chunk c of the label row: 1 KiB, 16 bytes per lane (PPL points)
                auto count_chunk = [&](auto ppl, int c, const uint4 &lab4, int &carry) {
                    constexpr int PPL = decltype(ppl)::value;
                    const int p0 = (c * 64 + lane) * PPL;
                    uint32_t fw[PPL / 4];
                    if (p0 < n) {
                        if constexpr (PPL == 16) {
                            const uint4 f = *(const uint4 *)(F + p0);
                            fw[0] = f.x; fw[1] = f.y; fw[2] = f.z; fw[3] = f.w;
                        } else {
                            const uint2 f = *(const uint2 *)(F + p0);
                            fw[0] = f.x; fw[1] = f.y;
                        }
                    } else {
#pragma unroll
                        for (int w = 0; w < PPL / 4; w++) fw[w] = 0;
                    }
                    int cnt = 0;   // flags are 0 or 1: a word's byte sum is its top byte times 0x01010101
#pragma unroll
                    for (int w = 0; w < PPL / 4; w++) cnt += (int)((fw[w] * 0x01010101u) >> 24);
                    const int incl = wave_incl_scan(cnt, lane);
                    int sc = carry + incl - cnt;            // flags before this lane's first point
                    const uint32_t lw[4] = {lab4.x, lab4.y, lab4.z, lab4.w};
#pragma unroll
                    for (int k = 0; k < PPL; k++) {
                        sc += (int)((fw[k >> 2] >> (8 * (k & 3))) & 1u);
                        const int lab = PPL == 16 ? (int)((lw[k >> 2] >> (8 * (k & 3))) & 0xffu)
                                                  : (int)((lw[k >> 1] >> (16 * (k & 1))) & 0xffffu);
                        if (p0 + k < n) atomicAdd(&rec[(sc + 1) * RS + 1 + lab], VB);
                    }
                    carry += __builtin_amdgcn_readlane(incl, 63);
                };
                auto count_all = [&](auto ppl) {
                    int carry = 0;
                    const int nch = (lbytes + 1023) >> 10;
                    for (int c0 = 0; c0 < nch; c0 += LG) {
                        if (c0 > 0) load_labels(c0);
#pragma unroll
                        for (int i = 0; i < LG; i++)
                            if (c0 + i < nch) count_chunk(ppl, c0 + i, lv[i], carry);
                    }
                };
                if (l16) count_all(std::integral_constant<int, 8>());
                else count_all(std::integral_constant<int, 16>());
            }
            wave_sync();
        } else {
            // one point per lane and step: a ballot of the flags
            const uint16_t *lb16 = (const uint16_t *)lb8;
            for (int k = lane; k < (K + 1) * RS; k += 64) rec[k] = 0;
            for (int p = lane; p < n; p += 64) F[p] = 0;
            wave_sync();
            for (int t = lane; t < K; t += 64) {
                const int et = ends[t];
                rec[(t + 1) * RS] = et * VB;
                if (t + 1 < K) F[et] = 1;
            }
            wave_sync();
            int carry = 0;
            for (int p0 = 0; p0 < n; p0 += 64) {
                const int p = p0 + lane;
                const int lab = p < n ? (l16 ? (int)lb16[p] : (int)lb8[p]) : 0;
                const bool f = p < n && F[p] != 0;
                const uint64_t bal = __ballot(f);
                const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                      __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                if (p < n) atomicAdd(&rec[(carry + below + (f ? 1 : 0) + 1) * RS + 1 + lab], VB);
                carry += __popcll(bal);
            }
            wave_sync();
        }
        if (CO && wv != 0) {
        } else if (yh >= 8) {
            // one row per lane, eight superclumps per step (loads issued together)
            for (int r = lane; r < yh; r += 64) {
                int *col = rec + 1 + r;
                int run = 0, t = 1;
                for (; t + 7 <= K; t += 8) {
                    int v[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) v[u] = col[(t + u) * RS];
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        run += v[u];
                        col[(t + u) * RS] = run;
                    }
                }
                for (; t <= K; t++) {
                    run += col[t * RS];
                    col[t * RS] = run;
                }
            }
        } else {
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
        }
        wave_sync();
        if constexpr (CO) {
            for (int k = lane; k < kCoChunks; k += 64)
                if (wv == 0) done[k] = 0;
            __syncthreads();
        }
        if constexpr (DBG) {
            // records of y+1 ints (the padding dropped)
            const int W = ycls + 1;
            int *o = a.dbg + (size_t)wi * KS * W;
            for (int k = lane; k < (K + 1) * W; k += 64) o[k] = rec[(k / W) * RS + k % W] / VB;
            continue;
        }

        // column cost h(s,t) with both records read from LDS (any row count):
        // the records (a multiple of four ints each) as 16-byte vectors, four
        // table reads in flight per vector (entries past yhat are zero in both
        // records: L[0] = 0)
        auto hcost = [&](int s, int t) -> V {
            if constexpr (YR > 0 && !rec_vector(YR)) {
                const int *rs = rec + s * RS, *rt = rec + t * RS;
                V acc = LB(rt[0] - rs[0]);
                for (int r = 0; r < yh; r++) acc -= LB(rt[1 + r] - rs[1 + r]);
                return acc;
            }
            const int4 *rs = (const int4 *)(rec + s * RS), *rt = (const int4 *)(rec + t * RS);
            const int4 a0 = rt[0], b0 = rs[0];
            const V acc = LB(a0.x - b0.x);
            V sub = LB(a0.y - b0.y) + (LB(a0.z - b0.z) + LB(a0.w - b0.w));
            const int nq = (yh + 4) >> 2;
            for (int q = 1; q < nq; q++) {
                const int4 u = rt[q], v = rs[q];
                sub += (LB(u.x - v.x) + LB(u.y - v.y)) + (LB(u.z - v.z) + LB(u.w - v.w));
            }
            return acc - sub;
        };

        V best = DV::big();
        bool pairs_done = false;
        if constexpr (NL == 1 && !CO) if (x == 3) {
            // ---- x = 3: one full layer, whose sources are all final from the
            // start (G_1(s) = h(0,s)).  The (s,t) pairs are spread over all
            // lanes, each cost computed once, and layer 2 is an LDS minimum per
            // target; a target-per-lane pass would compute every cost on a
            // lane whether or not its target lies after the source, and leave
            // the lanes past K idle.
            // (three arrays of K+1 values in the staging buffer, which the
            // host sizes for them)
            V *G1 = (V *)stage, *G2 = G1 + (K + 1), *HK = G2 + (K + 1);
            for (int t = lane; t <= K; t += 64) {
                const V h = t == 0 ? (V)0 : hcost(0, t);
                G1[t] = h;   // G_1(t), G_1(0) = 0
                G2[t] = h;   // source 0's candidate for G_2(t), G_2(0) = 0
            }
            wave_sync();
            if (lane == 0) HK[0] = G1[K];   // h(0,K)
            // pairs 1 <= s < t <= K, row s holding t = s+1..K
            const int np = K * (K - 1) / 2;
            int s0 = 1, r0 = 0;
            for (int p = lane; p < np; p += 64) {
                while (p >= r0 + K - s0) {
                    r0 += K - s0;
                    s0++;
                }
                const int t = s0 + 1 + (p - r0);
                const V h = hcost(s0, t);
                if constexpr (FX) atomicMin((unsigned *)(G2 + t), (unsigned)(G1[s0] + h));
                else atomicMin((double *)(G2 + t), (double)(G1[s0] + h));
                if (t == K) HK[s0] = h;
            }
            wave_sync();
            if (lane == 0) G[(size_t)2 * KS + K] = G2[K];
            // last layer at t = K: G_3(K) = min_s G_2(s) + h(s,K), G_2(0) = 0
            for (int s1 = lane; s1 < K; s1 += 64) best = DV::mn(best, G2[s1] + HK[s1]);
            global_sync();   // lane 0's G_2(K) store before the epilogue's loads
            pairs_done = true;
        }
        if (!pairs_done) {
            // ---- full layers l = 2..x-1 for every target (item 10b costs, OptimizeXAxis) ----
            // (NL = 0 is the shape for x = 2, where no layer is needed at every target)
            // cooperative: the pass number whose chunk flags a wave waits for
            int pass = 0;
            // waits until chunk ci has finished pass `pass` (cooperative only)
            auto wait_chunk = [&](int ci) {
                int spins = 0;
                while (__hip_atomic_load(done + ci, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < pass) {
                    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kCoSpinMax) {
                        if (lane == 0) {
                            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            atomicOr(a.status, 2);
                        }
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            };
            if constexpr (NL > 0)
            for (int l0 = 2; l0 <= x - 1; l0 += NL) {
                const int nl = min(NL, x - l0);
                const int nlp = (nl + PK - 1) / PK * PK;
                pass++;
                // chunks of 64 T targets; one wave per item puts the partial
                // chunk first (targets 1..r), so that its idle lanes meet no
                // earlier-chunk sources (cooperative passes keep aligned chunks,
                // which their chunk flags index)
                const int first = CO ? 64 * T : K - (K - 1) / (64 * T) * (64 * T);
                for (int c0 = 0, cend = min(first, K); c0 < K; c0 = cend, cend = min(cend + 64 * T, K)) {
                    if (CO && (c0 / (64 * T)) % wpb != wv) continue;   // another wave's chunk
                    int tt[T], et[T];
                    int Nt[T][YR > 0 ? YR : 1];
                    V g[T][NLP], gprev[T];
    #pragma unroll
                    for (int j = 0; j < T; j++) {
                        tt[j] = c0 + 64 * j + lane + 1;
                        const int tc = tt[j] <= cend ? tt[j] : cend;
                        const int *rt = rec + tc * RS;
                        et[j] = rt[0] + lbase;
                        V h0 = LA(et[j]);
                        if constexpr (YR > 0) {
    #pragma unroll
                            for (int r = 0; r < YR; r++) {
                                Nt[j][r] = rt[1 + r] + lbase;
                                h0 -= LA(Nt[j][r]);
                            }
                        } else {
                            h0 = hcost(0, tc);   // record 0 is all zeros
                        }
                        gprev[j] = l0 == 2 ? h0 : G[(size_t)(l0 - 1) * KS + tc];
    #pragma unroll
                        for (int q = 0; q < NLP; q++) g[j][q] = h0;
                    }
                    // h(s, t_j) for this lane's targets (count rows from registers or LDS)
                    auto hsrc = [&](int s, V (&out)[T]) {
                        if constexpr (YR > 0 && !rec_vector(YR)) {
                            const int *rs = rec + s * RS;
                            const int es = rs[0];
    #pragma unroll
                            for (int j = 0; j < T; j++) out[j] = LA(et[j] - es);
    #pragma unroll
                            for (int r = 0; r < YR; r++) {
                                const int nsr = rs[1 + r];
    #pragma unroll
                                for (int j = 0; j < T; j++) out[j] -= LA(Nt[j][r] - nsr);
                            }
                        } else if constexpr (YR > 0) {
                            // the source's record as 16-byte broadcast reads, each
                            // consumed before the next (entry 0 is e_s, entry 1+r
                            // row r's count)
                            const int4 *rs4 = (const int4 *)(rec + s * RS);
    #pragma unroll
                            for (int q = 0; q < (YR + 4) / 4; q++) {
                                const int4 v = rs4[q];
                                const int w[4] = {v.x, v.y, v.z, v.w};
    #pragma unroll
                                for (int e = 0; e < 4; e++) {
                                    const int i = 4 * q + e;
                                    if (i == 0) {
    #pragma unroll
                                        for (int j = 0; j < T; j++) out[j] = LA(et[j] - w[e]);
                                    } else if (i <= YR) {
    #pragma unroll
                                        for (int j = 0; j < T; j++) out[j] -= LA(Nt[j][i - 1] - w[e]);
                                    }
                                }
                            }
                        } else {
    #pragma unroll
                            for (int j = 0; j < T; j++) out[j] = hcost(s, tt[j] <= cend ? tt[j] : cend);
                        }
                    };
                    // sources of earlier chunks, SB at a time through LDS.  The
                    // next sources' costs are gathered while this step's cells
                    // update; the fixed-point form merges two sources per min3
                    // (a missing partner carries the largest value and cost 0).
                    constexpr int SP = DV::SP;
                    for (int sb = 1; sb <= c0; sb += SB) {
                        const int ns = min(SB, c0 - sb + 1);
                        // cooperative: the block's sources are final once the
                        // chunk of its last source has finished this pass (a
                        // chunk finishes only after every earlier one)
                        if constexpr (CO) wait_chunk((sb + ns - 2) / (64 * T));
                        for (int k = lane; k < nlp * SB; k += 64) {
                            const int q = k >> sbs, sl = k & (SB - 1);
                            stage[sl * NLP + q] = (sl < ns && q < nl)
                                                      ? G[(size_t)(l0 - 1 + q) * KS + sb + sl]
                                                      : DV::big();
                        }
                        wave_sync();
                        V hc[SP][T], hn[SP][T];
    #pragma unroll
                        for (int u = 0; u < SP; u++) {
                            if (u < ns) hsrc(sb + u, hc[u]);
                            else {
    #pragma unroll
                                for (int j = 0; j < T; j++) hc[u][j] = 0;
                            }
                        }
                        for (int sl = 0; sl < ns; sl += SP) {
    #pragma unroll
                            for (int u = 0; u < SP; u++) {
                                const int nx = sl + SP + u;
                                if (nx < ns) hsrc(sb + nx, hn[u]);
                                else {
    #pragma unroll
                                    for (int j = 0; j < T; j++) hn[u][j] = 0;
                                }
                            }
    #pragma unroll
                            for (int q = 0; q < NLP; q += PK) {
                                Pack<V> v[SP];
    #pragma unroll
                                for (int u = 0; u < SP; u++) v[u] = *(const Pack<V> *)(stage + (sl + u) * NLP + q);
    #pragma unroll
                                for (int j = 0; j < T; j++)
    #pragma unroll
                                    for (int e = 0; e < PK; e++) {
                                        V m = g[j][q + e];
    #pragma unroll
                                        for (int u = 0; u < SP; u++) m = DV::mn(m, v[u].v[e] + hc[u][j]);
                                        g[j][q + e] = m;
                                    }
                                if ((q / PK + 1) % MICX_DP_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
                            }
    #pragma unroll
                            for (int u = 0; u < SP; u++)
    #pragma unroll
                                for (int j = 0; j < T; j++) hc[u][j] = hn[u][j];
                        }
                        wave_sync();
                    }
                    // sources inside the chunk, in order: the lane that owns source s
                    // holds its final layers; they are broadcast to the wave through
                    // scalar registers, and the next source's costs are gathered
                    // while this source's cells update
    #pragma unroll
                    for (int jo = 0; jo < T; jo++) {
                        const int sbeg = c0 + 64 * jo + 1;
                        // the chunk's last target is no source for any target of this chunk
                        const int send = min(c0 + 64 * jo + 64, cend - 1);
                        V hs[T], hn[T];
                        if (sbeg <= send) hsrc(sbeg, hs);
                        for (int s = sbeg; s <= send; s++) {
                            const int ln = s - sbeg;
                            if (s < send) hsrc(s + 1, hn);
    #pragma unroll
                            for (int q0 = 0; q0 < NL; q0 += 8) {
                                V src[8];
    #pragma unroll
                                for (int e = 0; e < 8; e++)
                                    if (q0 + e < NL) src[e] = DV::bcast(q0 + e == 0 ? gprev[jo] : g[jo][q0 + e - 1], ln);
    #pragma unroll
                                for (int j = jo; j < T; j++) {
                                    if (j == jo && lane <= ln) continue;
    #pragma unroll
                                    for (int e = 0; e < 8; e++)
                                        if (q0 + e < NL) g[j][q0 + e] = DV::mn(g[j][q0 + e], src[e] + hs[j]);
                                }
                            }
    #pragma unroll
                            for (int j = 0; j < T; j++) hs[j] = hn[j];
                        }
                    }
                    // the chunk's layers become sources for later chunks
    #pragma unroll
                    for (int j = 0; j < T; j++) {
                        if (tt[j] <= cend) {
                            if (l0 == 2) G[(size_t)KS + tt[j]] = gprev[j];
    #pragma unroll
                            for (int q = 0; q < NLP; q++)
                                if (q < nl) G[(size_t)(l0 + q) * KS + tt[j]] = g[j][q];
                        }
                    }
                    global_sync();
                    if constexpr (CO) {
                        // release: the chunk's layers of this pass are in G
                        if (lane == 0)
                            __hip_atomic_store(done + c0 / (64 * T), pass, __ATOMIC_RELEASE,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
            if constexpr (CO) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }

            // ---- last layer only at t = K: G_x(K) = min_{0 <= s < K} G_{x-1}(s) + h(s,K) ----
            for (int s = lane + (CO ? 64 * wv : 0); s < K; s += (CO ? 64 * wpb : 64)) {
                V gs = 0;   // G_{x-1}(0) = 0
                if (s > 0) gs = (x == 2) ? hcost(0, s) : G[(size_t)(x - 1) * KS + s];
                best = DV::mn(best, gs + hcost(s, K));
            }
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) best = DV::mn(best, (V)__shfl_xor(best, d, 64));
        if constexpr (CO) {
            // the waves' minima, combined by wave 0, which writes the scores
            if (lane == 0) wmin[wv] = best;
            __syncthreads();
            if (wv != 0) {
                __syncthreads();   // the item's end (wave 0 writes the scores)
                continue;
            }
            for (int w = 1; w < wpb; w++) best = DV::mn(best, wmin[w]);
        }

        // ---- I_l = (L[n] - sum_r L[q_r] - G_l(K)) / n in FP64, normalised by ln min(l, yhat) ----
        // H(Q) term: the rows' q ln q summed over lanes (a butterfly, so every
        // lane holds the same sum)
        double sq = 0.0;
        for (int r = lane; r < yh; r += 64) sq += a.xlogx[rec[K * RS + 1 + r] / VB];
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) sq += __shfl_xor(sq, d, 64);
        const double Ln = a.xlogx[n];
        for (int l = 2 + lane; l <= x; l += 64) {
            const V Gl = (l == x) ? best : G[(size_t)l * KS + K];
            const double I = (Ln - sq - DV::real(Gl, a.inv_scale)) / (double)n;
            const int norm = min(l, (a.compat & MICX_COMPAT_NORM_BY_Y) ? ycls : yh);
            // ln(norm) = (norm ln norm) / norm from the j ln j table
            Aout[l - 2] = norm >= 2 ? I * (double)norm / a.xlogx[norm] : 0.0;
        }
        wave_sync();
        if constexpr (CO) __syncthreads();   // the item's end: rec and G are reused
    }
}

typedef void (*dp_kernel_t)(DpArgs);

}  // namespace micx
