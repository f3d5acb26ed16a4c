// Issue-rate probes behind the roofline ceiling of the pair kernels: the
// shader cycles a SIMD spends per wave64 FP32 FMA (all operands in VGPRs, and
// with one SGPR operand) and per v_rsq_f32, and the shader clock while the
// FMA probe runs.  Eight independent dependency chains per lane and eight
// waves per SIMD (the pair kernels' occupancy) keep each probe on issue
// throughput; with fewer waves the rate drops (3.5 cycles per FMA at four).
// Measurement support for the roofline only; no part of the force path.
#include "probe.h"

namespace nbk {

constexpr int kProbeChains = 8;
constexpr int kProbeThreads = 256;

// MODE 0: v_fma_f32 with VGPR operands; 1: v_fma_f32 with one SGPR operand;
// 2: v_rsq_f32.  Thread 0 of block 0 records the shader-cycle counter and the
// fixed-rate wall counter around its loop.
template <int MODE>
__global__ __launch_bounds__(kProbeThreads) void k_probe(float *out, long long *clk, int iters, float a,
                                                         float b)
{
    float v[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) v[k] = 1.0f + 1e-3f * (float)threadIdx.x + (float)k;
    float av = a, bv = b;
    if (MODE == 0) {
        // the multiplier and addend as VGPR values, as the pair arithmetic has them
        asm volatile("v_mov_b32 %0, %1" : "=v"(av) : "s"(a));
        asm volatile("v_mov_b32 %0, %1" : "=v"(bv) : "s"(b));
    }
    const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
    long long c0 = 0, w0 = 0;
    if (timer) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) {
            if (MODE == 2) v[k] = __builtin_amdgcn_rsqf(v[k]);
            else v[k] = __builtin_fmaf(v[k], av, bv);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += v[k];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
    if (timer) {
        clk[2 * MODE] = clock64() - c0;
        clk[2 * MODE + 1] = wall_clock64() - w0;
    }
}

hipError_t launch_probe(int mode, float *out, long long *clk, int blocks, int iters, hipStream_t s)
{
    const dim3 grid((unsigned)blocks), block(kProbeThreads);
    switch (mode) {
    case 0: hipLaunchKernelGGL(k_probe<0>, grid, block, 0, s, out, clk, iters, 0.999f, 1e-3f); break;
    case 1: hipLaunchKernelGGL(k_probe<1>, grid, block, 0, s, out, clk, iters, 0.999f, 1e-3f); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, grid, block, 0, s, out, clk, iters, 0.999f, 1e-3f); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nbk
