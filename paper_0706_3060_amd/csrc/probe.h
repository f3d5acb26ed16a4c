// Interface of the issue-rate probes (probe.hip) to the host runtime.
#pragma once
#include <hip/hip_runtime.h>

namespace nbk {

// Probe modes 0..6 (see probe.hip).  out: [blocks * 256] floats (keeps the
// chains live); clk: [2], the shader cycles and wall-counter ticks of the
// timing wave of the last launch.
constexpr int kProbeModes = 7;
hipError_t launch_probe(int mode, float *out, long long *clk, int blocks, int iters, hipStream_t s);
// measured instructions (mode 3: groups of one rsq and 13 FMAs) per loop iteration and lane
int probe_units_per_iter(int mode);

}  // namespace nbk
