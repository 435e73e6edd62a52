// Device arithmetic shared by the forward and adjoint kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace gd {

// Reciprocal and reciprocal square root: the hardware estimate refined by
// Newton-Raphson iterations (two for FP64, which square the relative error
// each time; the FP32 estimate is already within an ulp). Operands are
// normal, finite numbers here (densities, pressures and wave-speed gaps).

__device__ __forceinline__ double fast_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double fast_rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    double t = fma(-h * y, y, 0.5);
    y = fma(y, t, y);
    t = fma(-h * y, y, 0.5);
    return fma(y, t, y);
}

__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

}  // namespace gd
