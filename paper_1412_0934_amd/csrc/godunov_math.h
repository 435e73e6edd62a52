// Device arithmetic shared by the forward and adjoint kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace gd {

// Reciprocal and reciprocal square root: the hardware estimate refined by one
// Newton-Raphson iteration in FP64, which squares its relative error: the
// gfx950 estimates are within about 5e-8 of the true value, one iteration
// brings them within about 4e-15 (a few tens of ulp, measured over 2^20
// operands spanning 40 binades), far inside the 1e-12 the step is held to.
// The FP32 estimate is already within an ulp. Operands are normal, finite
// numbers here (densities, pressures and wave-speed gaps).

__device__ __forceinline__ double fast_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double fast_rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double t = fma(-(0.5 * x) * y, y, 0.5);
    return fma(y, t, y);
}

__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

}  // namespace gd
