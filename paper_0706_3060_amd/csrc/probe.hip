// Issue-rate probes behind the roofline ceiling of the pair kernels: the
// shader cycles a SIMD spends per wave64 instruction of the kinds the pair
// sequences are made of, and the shader clock while the FMA probe runs.
// Every probe runs independent dependency chains per lane at eight waves per
// SIMD (the most a SIMD holds) and times itself in shader cycles (s_memtime
// over the fixed-rate s_memrealtime).  Measurement support for the roofline
// only; no part of the force path.
//
// Modes (cycles per instruction unless noted):
//   0  v_fma_f32, all operands in VGPRs (the multiplier and addend shared by the chains)
//   1  v_fma_f32 with one SGPR operand
//   2  v_rsq_f32
//   3  one v_rsq_f32 interleaved with 13 independent FMAs (cycles per group of 14)
//   4  v_fma_f32 whose multiplier and addend are distinct VGPRs rotating over the chains
//   5  v_mov_b32 with a DPP row rotation (a cross-lane move on the VALU)
//   6  ds_bpermute_b32 (a cross-lane move through the LDS crossbar)
#include "probe.h"

namespace nbk {

constexpr int kProbeThreads = 256;

// per-lane value kept in a VGPR (the compiler would otherwise fold uniform values into SGPRs)
__device__ __forceinline__ float in_vgpr(float x)
{
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "v"(x));
    return v;
}

template <int MODE>
__global__ __launch_bounds__(kProbeThreads) void k_probe(float *out, long long *clk, int iters, float a,
                                                         float b)
{
    constexpr int K = 8;
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = 1.0f + 1e-3f * (float)threadIdx.x + (float)k;
    float av = a, bv = b;
    if (MODE == 0 || MODE == 3) {
        av = in_vgpr(a + 0.0f * (float)threadIdx.x);
        bv = in_vgpr(b + 0.0f * (float)threadIdx.x);
    }
    float am[16], bm[16];
    if (MODE == 4) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            am[k] = in_vgpr(a - 1e-6f * (float)k);
            bm[k] = in_vgpr(b + 1e-6f * (float)k);
        }
    }
    const int bp_addr = (((int)threadIdx.x + 1) & 63) * 4;
    const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
    long long c0 = 0, w0 = 0;
    if (timer) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    for (int i = 0; i < iters; ++i) {
        if (MODE == 0 || MODE == 1) {
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = __builtin_fmaf(v[k], av, bv);
        } else if (MODE == 2) {
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = __builtin_amdgcn_rsqf(v[k]);
        } else if (MODE == 3) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                v[k] = __builtin_amdgcn_rsqf(v[k]);
#pragma unroll
                for (int t = 0; t < 13; ++t) {
                    const int c = 8 + (13 * k + t) % 8;
                    v[c] = __builtin_fmaf(v[c], av, bv);
                }
            }
        } else if (MODE == 4) {
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = __builtin_fmaf(v[k], am[k], bm[(k + 7) & 15]);
        } else if (MODE == 5) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[k] = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v[k]), 0x121,
                                                                          0xF, 0xF, false));
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[k] = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(bp_addr, __builtin_bit_cast(int, v[k])));
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
    if (timer) {
        clk[0] = clock64() - c0;
        clk[1] = wall_clock64() - w0;
    }
}

// instructions of the measured kind per loop iteration and lane (mode 3: groups of 14)
int probe_units_per_iter(int mode)
{
    switch (mode) {
    case 3: return 8;
    case 4: return 16;
    default: return 8;
    }
}

hipError_t launch_probe(int mode, float *out, long long *clk, int blocks, int iters, hipStream_t s)
{
    const dim3 grid((unsigned)blocks), block(kProbeThreads);
    const float a = 0.999f, b = 1e-3f;
    switch (mode) {
    case 0: hipLaunchKernelGGL(k_probe<0>, grid, block, 0, s, out, clk, iters, a, b); break;
    case 1: hipLaunchKernelGGL(k_probe<1>, grid, block, 0, s, out, clk, iters, a, b); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, grid, block, 0, s, out, clk, iters, a, b); break;
    case 3: hipLaunchKernelGGL(k_probe<3>, grid, block, 0, s, out, clk, iters, a, b); break;
    case 4: hipLaunchKernelGGL(k_probe<4>, grid, block, 0, s, out, clk, iters, a, b); break;
    case 5: hipLaunchKernelGGL(k_probe<5>, grid, block, 0, s, out, clk, iters, a, b); break;
    case 6: hipLaunchKernelGGL(k_probe<6>, grid, block, 0, s, out, clk, iters, a, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nbk
