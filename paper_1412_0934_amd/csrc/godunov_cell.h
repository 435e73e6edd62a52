// Cell physics and Riemann fluxes of the Euler step (gfx950 device code),
// shared by the step kernels and the coarse-fine seam kernels.
#pragma once

#include "godunov_internal.h"
#include "godunov_math.h"

#include <hip/hip_runtime.h>

namespace gd {

enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_NONE = 2 };
enum { RS_HLLC = 0, RS_HLL = 1 };

template <typename T>
struct Phys {
    T gamma, gm1, inv_gm1, rho_floor, p_floor;
};

template <typename T>
__device__ __forceinline__ Phys<T> make_phys(const Scalars &sc)
{
    Phys<T> ph;
    ph.gamma = T(sc.gamma);
    ph.gm1 = T(sc.gamma - 1.0);
    ph.inv_gm1 = T(1.0 / (sc.gamma - 1.0));
    ph.rho_floor = T(sc.rho_floor);
    ph.p_floor = T(sc.p_floor);
    return ph;
}

// ------------------------------------------------------------ cell physics

// max(x, floor), counting a raise. Written as a comparison and a select that
// share the comparison with the count: a maximum of a loaded value costs two
// extra canonicalising instructions in IEEE mode. Equal to fmax for every
// number x; a NaN x stays NaN.
template <typename T>
__device__ __forceinline__ T floored(T x, T floor, int &hits)
{
    const bool below = x < floor;
    hits += below;
    return below ? floor : x;
}

template <typename T>
__device__ __forceinline__ void prim_from_cons(const T U[5], T W[5], T &inv_rho,
                                               const Phys<T> &ph, int &hits)
{
    const T rho = floored(U[0], ph.rho_floor, hits);
    T inv = fast_rcp(rho);
    T u = U[1] * inv, v = U[2] * inv, w = U[3] * inv;
    T kin = T(0.5) * (U[1] * u + U[2] * v + U[3] * w);
    const T p = floored(ph.gm1 * (U[4] - kin), ph.p_floor, hits);
    W[0] = rho; W[1] = u; W[2] = v; W[3] = w; W[4] = p;
    inv_rho = inv;
}

// Limited undivided slope from a = q_i - q_{i-1}, b = q_{i+1} - q_i.
// minmod is the median of (a, b, 0); MC is sign(a) min(2|a|, 2|b|, |a+b|/2)
// when a and b share a sign, else 0.
template <int LIM, typename T>
__device__ __forceinline__ T limited_slope(T a, T b)
{
    if constexpr (LIM == LIM_NONE) {
        return T(0.5) * (a + b);
    } else if constexpr (LIM == LIM_MINMOD) {
        return fmax(fmin(a, b), fmin(fmax(a, b), T(0)));
    } else {
        T lo = fmin(a, b), hi = fmax(a, b);
        T m = fmin(fmin(T(2) * fabs(a), T(2) * fabs(b)), T(0.5) * fabs(a + b));
        return lo > T(0) ? m : (hi < T(0) ? -m : T(0));
    }
}

// Hancock predictor, primitive form, all three directions.
template <typename T>
__device__ __forceinline__ void predictor(const T W[5], T inv_rho, const T Sx[5], const T Sy[5],
                                          const T Sz[5], T lam, T gamma, T Ws[5])
{
    const T u = W[1], v = W[2], w = W[3];
    T divu = Sx[1] + Sy[2] + Sz[3];
    T adv[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) adv[q] = u * Sx[q] + v * Sy[q] + w * Sz[q];
    Ws[0] = W[0] - lam * (adv[0] + W[0] * divu);
    Ws[1] = u - lam * (adv[1] + Sx[4] * inv_rho);
    Ws[2] = v - lam * (adv[2] + Sy[4] * inv_rho);
    Ws[3] = w - lam * (adv[3] + Sz[4] * inv_rho);
    Ws[4] = W[4] - lam * (adv[4] + gamma * W[4] * divu);
}

template <typename T>
__device__ __forceinline__ void face_state(const T Ws[5], const T S[5], T half_sign, T out[5],
                                           const Phys<T> &ph, int &hits)
{
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q] = Ws[q] + half_sign * S[q];
    out[0] = floored(out[0], ph.rho_floor, hits);
    out[4] = floored(out[4], ph.p_floor, hits);
}

// ------------------------------------------------------------ Riemann fluxes
// States are rotated: (rho, u_n, u_t1, u_t2, p).

template <typename T>
__device__ __forceinline__ void hllc_rotated(const T L[5], const T R[5], const Phys<T> &ph, T F[5])
{
    const T g = ph.gamma;
    // c = sqrt(g p / rho) = g p / sqrt(g p rho)
    T gpL = g * L[4], gpR = g * R[4];
    T cL = gpL * fast_rsqrt(gpL * L[0]);
    T cR = gpR * fast_rsqrt(gpR * R[0]);
    T SL = fmin(L[1] - cL, R[1] - cR);
    T SR = fmax(L[1] + cL, R[1] + cR);
    T mL = L[0] * (SL - L[1]);
    T mR = R[0] * (SR - R[1]);
    T Sst = (R[4] - L[4] + mL * L[1] - mR * R[1]) * fast_rcp(mL - mR);

    // Regions, in order: S_L >= 0 -> F(L); S* >= 0 -> L star; S_R > 0 ->
    // R star; else F(R). K is the side whose flux is the base.
    bool supL = SL >= T(0);
    bool left = supL || Sst >= T(0);
    bool star = !supL && (left || SR > T(0));
    T rK = left ? L[0] : R[0];
    T uK = left ? L[1] : R[1];
    T vK = left ? L[2] : R[2];
    T wK = left ? L[3] : R[3];
    T pK = left ? L[4] : R[4];
    T SK = left ? SL : SR;

    T EK = pK * ph.inv_gm1 + T(0.5) * rK * (uK * uK + vK * vK + wK * wK);
    T mass = rK * uK;
    T FK[5] = { mass, mass * uK + pK, mass * vK, mass * wK, uK * (EK + pK) };
    T UK[5] = { rK, mass, rK * vK, rK * wK, EK };
    // U*_K = a (1, S*, v_K, w_K, e) with a = rho_K (S_K - u_K)/(S_K - S*) and
    // e = E_K/rho_K + (S* - u_K)(S* + p_K/(rho_K (S_K - u_K))); the energy
    // component a e is expanded so that only 1/(S_K - S*) is needed.
    // F = F_K + s (U*_K - U_K) with s = S_K in the star regions and 0 in the
    // upwind ones, where 1/(S_K - S*) is replaced by 0 so that U*_K stays
    // finite: two selects instead of one per component, the same value.
    T dK = SK - uK;
    T inv_d = star ? fast_rcp(SK - Sst) : T(0);
    T sK = star ? SK : T(0);
    T a = rK * dK * inv_d;
    T su = Sst - uK;
    T Us[5] = { a, a * Sst, a * vK, a * wK, inv_d * (EK * dK + su * pK) + a * Sst * su };
#pragma unroll
    for (int q = 0; q < 5; ++q) F[q] = FK[q] + sK * (Us[q] - UK[q]);
}

template <typename T>
__device__ __forceinline__ void euler_flux_rotated(const T W[5], const Phys<T> &ph, T F[5], T U[5])
{
    T E = W[4] * ph.inv_gm1 + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
    T mass = W[0] * W[1];
    F[0] = mass; F[1] = mass * W[1] + W[4]; F[2] = mass * W[2]; F[3] = mass * W[3];
    F[4] = W[1] * (E + W[4]);
    U[0] = W[0]; U[1] = mass; U[2] = W[0] * W[2]; U[3] = W[0] * W[3]; U[4] = E;
}

template <typename T>
__device__ __forceinline__ void hll_rotated(const T L[5], const T R[5], const Phys<T> &ph, T F[5])
{
    const T g = ph.gamma;
    T gpL = g * L[4], gpR = g * R[4];
    T cL = gpL * fast_rsqrt(gpL * L[0]);
    T cR = gpR * fast_rsqrt(gpR * R[0]);
    T SL = fmin(L[1] - cL, R[1] - cR);
    T SR = fmax(L[1] + cL, R[1] + cR);
    T FL[5], FR[5], UL[5], UR[5];
    euler_flux_rotated(L, ph, FL, UL);
    euler_flux_rotated(R, ph, FR, UR);
    T inv = fast_rcp(SR - SL);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        T Fm = (SR * FL[q] - SL * FR[q] + SL * SR * (UR[q] - UL[q])) * inv;
        F[q] = SL >= T(0) ? FL[q] : (SR <= T(0) ? FR[q] : Fm);
    }
}

template <int RS, typename T>
__device__ __forceinline__ void riemann(const T L[5], const T R[5], const Phys<T> &ph, T F[5])
{
    if constexpr (RS == RS_HLL) hll_rotated(L, R, ph, F);
    else hllc_rotated(L, R, ph, F);
}

// Flux through a face normal to the compile-time direction D from unrotated
// primitive states; transverse components follow the cyclic order (D+1, D+2).
template <int RS, int D, typename T>
__device__ __forceinline__ void face_flux(const T WL[5], const T WR[5], const Phys<T> &ph, T F[5])
{
    constexpr int n = 1 + D, t1 = 1 + (D + 1) % 3, t2 = 1 + (D + 2) % 3;
    T L[5] = { WL[0], WL[n], WL[t1], WL[t2], WL[4] };
    T R[5] = { WR[0], WR[n], WR[t1], WR[t2], WR[4] };
    T G[5];
    riemann<RS>(L, R, ph, G);
    F[0] = G[0]; F[n] = G[1]; F[t1] = G[2]; F[t2] = G[3]; F[4] = G[4];
}

// The same for a direction chosen per lane (x or y), used where one wave
// holds faces of both orientations.
template <int RS, typename T>
__device__ __forceinline__ void face_flux_xy(bool isx, const T WL[5], const T WR[5],
                                             const Phys<T> &ph, T F[5])
{
    // x: (u, v, w); y: (v, w, u)
    T L[5] = { WL[0], isx ? WL[1] : WL[2], isx ? WL[2] : WL[3], isx ? WL[3] : WL[1], WL[4] };
    T R[5] = { WR[0], isx ? WR[1] : WR[2], isx ? WR[2] : WR[3], isx ? WR[3] : WR[1], WR[4] };
    T G[5];
    riemann<RS>(L, R, ph, G);
    F[0] = G[0]; F[4] = G[4];
    F[1] = isx ? G[1] : G[3];
    F[2] = isx ? G[2] : G[1];
    F[3] = isx ? G[3] : G[2];
}

}  // namespace gd
