// Register-only issue-rate probe of the integer instructions the pointwise
// product is made of, for the ceiling its roofline is priced against.  No
// memory traffic inside the timed loop: every thread keeps eight independent
// accumulators in registers, so the only limit is how fast the SIMDs issue
// the instruction.
//   kind 0: v_add_u32 (a full-rate VALU operation; calibrates the clock)
//   kind 1: v_mad_u64_u32 alone
//   kind 2: v_mad_u64_u32 followed by v_addc_co_u32 of its carry, the
//           two-instruction limb multiply-accumulate of the pointwise kernel
#include <hip/hip_runtime.h>

#include "../../include/tft.h"
#include "kernels.hpp"

// Written only when a probe's accumulators hit one particular value; visible
// outside this file, so the compiler must keep the work that feeds it.
__device__ uint64_t tft_alu_rate_sink;
// Shader-clock counter (s_memtime) and 100 MHz real-time counter
// (s_memrealtime) at the start and end of workgroup 0's first wave.
__device__ uint64_t tft_alu_rate_clock[4];

namespace {

constexpr uint32_t kThreads = 256;
constexpr int kChains = 8;

template <int KIND>
__global__ void __launch_bounds__(kThreads) alu_rate_kernel(uint32_t iters, uint32_t seed) {
    const uint32_t t = threadIdx.x + blockIdx.x * kThreads;
    const bool timer = blockIdx.x == 0 && threadIdx.x < 64u;
    uint64_t c0 = 0, r0 = 0;
    if (timer) {
        c0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    uint32_t a[kChains], cy[kChains];
    uint64_t acc[kChains], cc[kChains] = {};
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        a[k] = (t * 2654435761u) ^ (seed + (uint32_t)k * 0x9E3779B9u);
        acc[k] = a[k];
        cy[k] = 0u;
    }
    const uint32_t b = seed | 1u;
    for (uint32_t i = 0; i < iters; ++i) {
        if constexpr (KIND == 0) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
        } else if constexpr (KIND == 1) {
#pragma unroll
            // a carry register of its own per chain (live after the loop), so
            // that no two multiply-adds in flight write the same one
            for (int k = 0; k < kChains; ++k)
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[k]), "=s"(cc[k]) : "v"(a[k]), "v"(b));
        } else {
            // four multiply-adds, then their four carry additions (three
            // instructions between a carry's write and its read)
#pragma unroll
            for (int k0 = 0; k0 < kChains; k0 += 4) {
                uint64_t c0, c1, c2, c3;
                asm volatile(
                    "v_mad_u64_u32 %0, %4, %8, %12, %0\n\t"
                    "v_mad_u64_u32 %1, %5, %9, %12, %1\n\t"
                    "v_mad_u64_u32 %2, %6, %10, %12, %2\n\t"
                    "v_mad_u64_u32 %3, %7, %11, %12, %3"
                    : "+v"(acc[k0]), "+v"(acc[k0 + 1]), "+v"(acc[k0 + 2]), "+v"(acc[k0 + 3]), "=&s"(c0), "=&s"(c1),
                      "=&s"(c2), "=&s"(c3)
                    : "v"(a[k0]), "v"(a[k0 + 1]), "v"(a[k0 + 2]), "v"(a[k0 + 3]), "v"(b));
                asm volatile(
                    "v_addc_co_u32_e64 %0, %4, %0, 0, %4\n\t"
                    "v_addc_co_u32_e64 %1, %5, %1, 0, %5\n\t"
                    "v_addc_co_u32_e64 %2, %6, %2, 0, %6\n\t"
                    "v_addc_co_u32_e64 %3, %7, %3, 0, %7"
                    : "+v"(cy[k0]), "+v"(cy[k0 + 1]), "+v"(cy[k0 + 2]), "+v"(cy[k0 + 3]), "+s"(c0), "+s"(c1),
                      "+s"(c2), "+s"(c3));
            }
        }
    }
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += acc[k] + a[k] + cy[k] + cc[k];
    if (s == 0x0123456789ABCDEFull) tft_alu_rate_sink = s;  // keeps the loop; practically never taken
    if (timer) {
        const uint64_t c1 = __builtin_amdgcn_s_memtime();
        const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
        if (threadIdx.x == 0u) {
            tft_alu_rate_clock[0] = c0;
            tft_alu_rate_clock[1] = c1;
            tft_alu_rate_clock[2] = r0;
            tft_alu_rate_clock[3] = r1;
        }
    }
}

template <int KIND>
hipError_t launch(uint32_t blocks, uint32_t iters, hipStream_t st) {
    hipLaunchKernelGGL(alu_rate_kernel<KIND>, dim3(blocks), dim3(kThreads), 0, st, iters, 0x5851F42Du);
    return hipGetLastError();
}

hipError_t launch_kind(uint32_t kind, uint32_t blocks, uint32_t iters, hipStream_t st) {
    switch (kind) {
        case 0: return launch<0>(blocks, iters, st);
        case 1: return launch<1>(blocks, iters, st);
        default: return launch<2>(blocks, iters, st);
    }
}

}  // namespace

extern "C" int tft_alu_rate(uint32_t kind, uint32_t blocks, uint32_t iters, float *ms, uint64_t *lane_ops,
                            double *clock_hz, void *stream) {
    if (kind > 2 || blocks == 0 || iters == 0 || !ms || !lane_ops || !clock_hz) return TFT_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_kind(kind, blocks, iters / 8u + 1u, st);  // untimed warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_kind(kind, blocks, iters, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    uint64_t clk[4] = {};
    if (e == hipSuccess) e = hipMemcpyFromSymbol(clk, HIP_SYMBOL(tft_alu_rate_clock), sizeof clk, 0, hipMemcpyDeviceToHost);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return tft::device_error(e, "alu rate probe");
    *lane_ops = (uint64_t)blocks * kThreads * iters * kChains;
    *clock_hz = clk[3] > clk[2] ? (double)(clk[1] - clk[0]) * 1e8 / (double)(clk[3] - clk[2]) : 0.0;
    return TFT_OK;
}
