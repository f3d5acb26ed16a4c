// Interface of the issue-rate probes (probe.hip) to the host runtime.
#pragma once
#include <hip/hip_runtime.h>

namespace nbk {

// mode 0: FP32 FMA with VGPR operands; 1: with one SGPR operand; 2: v_rsq_f32.
// out: [blocks * 256] floats (keeps the chains live); clk: [6], the shader
// cycles and wall-counter ticks of each mode's timing wave.
hipError_t launch_probe(int mode, float *out, long long *clk, int blocks, int iters, hipStream_t s);

}  // namespace nbk
