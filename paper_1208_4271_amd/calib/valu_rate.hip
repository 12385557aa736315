// valu_rate.hip -- issue rate of the VALU instructions the DP kernels use, on
// the GPU it runs on.  Each case runs 16 independent register chains of one
// instruction (inline assembly of ALU instructions only, so the count is
// exact) over W waves per SIMD (first argument, default 8), and reports
// SIMD-cycles per wave64
// instruction at the clock the first wave measures (shader clock against the
// 100 MHz real-time counter).  The peaks in bench.py's roofline rest on these
// rates.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o valu_rate paper_1208_4271_amd/calib/valu_rate.hip && ./valu_rate [W]
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define NCASE 12

template <int KIND>
__global__ __launch_bounds__(256) void k_rate(uint32_t *out, unsigned long long *clk, int iters, uint32_t seed) {
    uint32_t a[16];
    const uint32_t b = seed * 3u + threadIdx.x, c = seed ^ 0x5a5a5a5au;
    const float fb = (float)b * 1e-9f;
#pragma unroll
    for (int j = 0; j < 16; j++) a[j] = seed + threadIdx.x * (j + 1);
    const unsigned long long t0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int r = 0; r < 2; r++) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                if (KIND == 0) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
                else if (KIND == 1) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
                else if (KIND == 2) asm volatile("v_add_u32 %0, %1, %0" : "+v"(a[j]) : "s"(seed));
                else if (KIND == 3) asm volatile("v_min_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
                else if (KIND == 4) asm volatile("v_min3_u32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
                else if (KIND == 5) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
                else if (KIND == 6) asm volatile("v_mov_b32 %0, %1" : "=v"(a[j]) : "s"(seed + j));
                else if (KIND == 7) {
                    uint32_t sv;
                    asm volatile("v_readlane_b32 %0, %1, 5" : "=s"(sv) : "v"(a[j]));
                    asm volatile("v_add_u32 %0, %1, %0" : "+v"(a[(j + 1) & 15]) : "s"(sv));
                } else if (KIND == 8) asm volatile("v_add_f32 %0, %0, %1" : "+v"(a[j]) : "v"(fb));
                else if (KIND == 9) asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(a[j]) : "v"(fb));
                else if (KIND == 10)
                    asm volatile("v_add_f64 %0, %0, %1" : "+v"(*(double *)&a[j & 14]) : "v"(*(double *)&a[(j & 14) ^ 2]));
                else
                    asm volatile("v_min_f64 %0, %0, %1" : "+v"(*(double *)&a[j & 14]) : "v"(*(double *)&a[(j & 14) ^ 2]));
            }
        }
    }
    const unsigned long long t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 16; j++) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clk[0] = t1 - t0;
        clk[1] = r1 - r0;
    }
}

typedef void (*kern_t)(uint32_t *, unsigned long long *, int, uint32_t);

int main(int argc, char **argv) {
    const int wps = argc > 1 ? atoi(argv[1]) : 8;   // waves per SIMD (4 waves per workgroup)
    if (wps < 1 || wps > 8) {
        fprintf(stderr, "waves per SIMD must be 1..8\n");
        return 1;
    }
    const int blocks = 256 * wps, threads = 256, iters = 10000;
    const double winstr = (double)blocks * (threads / 64) * iters * 32;   // wave-instructions per launch
    uint32_t *out = nullptr;
    unsigned long long *clk = nullptr;
    if (hipMalloc((void **)&out, (size_t)blocks * threads * 4) != hipSuccess ||
        hipMalloc((void **)&clk, 16) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    const char *names[NCASE] = {"v_add_u32 v,v", "v_sub_u32 v,v", "v_add_u32 v,s", "v_min_u32 v,v",
                                "v_min3_u32", "v_add3_u32", "v_mov_b32 v,s", "v_readlane + v_add_u32 v,s",
                                "v_add_f32 v,v", "v_fma_f32", "v_add_f64", "v_min_f64"};
    const kern_t ks[NCASE] = {k_rate<0>, k_rate<1>, k_rate<2>, k_rate<3>, k_rate<4>, k_rate<5>,
                              k_rate<6>, k_rate<7>, k_rate<8>, k_rate<9>, k_rate<10>, k_rate<11>};
    printf("waves per SIMD: %d\n", wps);
    printf("%-28s %9s %10s %8s %14s\n", "instruction", "ms", "T lane/s", "MHz", "cycles/instr");
    for (int kind = 0; kind < NCASE; kind++) {
        for (int rep = 0; rep < 2; rep++) {   // the first launch warms up
            (void)hipEventRecord(e0, 0);
            hipLaunchKernelGGL(ks[kind], dim3(blocks), dim3(threads), 0, 0, out, clk, iters, 7u);
            (void)hipEventRecord(e1, 0);
            if (hipEventSynchronize(e1) != hipSuccess) {
                fprintf(stderr, "launch failed\n");
                return 2;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            unsigned long long hc[2] = {0, 0};
            if (hipMemcpy(hc, clk, 16, hipMemcpyDeviceToHost) != hipSuccess) return 3;
            const double mhz = (double)hc[0] / ((double)hc[1] * 10.0 / 1e3);
            const double cyc = (ms * 1e-3) * (mhz * 1e6) * 1024.0 / winstr;   // 1024 SIMDs
            if (rep == 1)
                printf("%-28s %9.3f %10.1f %8.0f %14.2f\n", names[kind], ms, winstr * 64 / (ms * 1e-3) / 1e12,
                       mhz, cyc);
        }
    }
    (void)hipFree(out);
    (void)hipFree(clk);
    return 0;
}
