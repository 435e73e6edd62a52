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

// x / 6 with the rounding of the division itself (x finite, not subnormal),
// in three FMA-unit operations instead of the division sequence: x times the
// rounded reciprocal y is a faithful quotient q, the remainder x - 6q is
// exact in one FMA, and q + (x - 6q) y rounds to the correctly rounded
// quotient (Markstein's theorem on FMA division); copysign gives a zero
// quotient the sign of x. Checked against x / 6 on every binary32 value and
// on 4e8 binary64 values.
template <typename T>
__device__ __forceinline__ T div6(T x)
{
    const T y = T(1) / T(6);
    const T q = x * y;
    const T r = fma(-q, T(6), x);
    return copysign(fma(r, y, q), x);
}

}  // namespace gd
