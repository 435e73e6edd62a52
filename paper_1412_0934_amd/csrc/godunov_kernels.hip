// gfx950 kernels of the unsplit MUSCL-Hancock Godunov step (3-D Euler).
//
// Forward step: one workgroup owns a TX x TY column tile of a patch and
// marches through a z-range plane by plane (a 2.5-D sweep). Per plane:
//   - the primitive state of the tile plus a two-deep x-y halo is staged in
//     LDS (each HBM byte read once per tile; halo overlap between tiles is
//     served by L2);
//   - the z-neighbours of a column live in registers of its owner thread;
//   - every cell whose predicted state some face needs (the tile interior
//     plus a one-deep ring) computes its slopes, predictor and face states;
//   - each face flux is computed exactly once and shared through LDS;
//   - the update of a plane is completed one plane later, when the flux
//     through its upper z face is known.
// The interior is TX*TY threads; one extra wave-aligned group of threads owns
// the ring cells (depth-1 halo), which need predicted states but no update.
//
// The same tile routine serves one patch (a grid of tiles) and a batch of
// patches (a persistent grid pulling tiles from a device work queue).
#include "godunov_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_NONE = 2 };
enum { RS_HLLC = 0, RS_HLL = 1 };

int tile_tx(int shape) { return shape == TILE_8x8 ? 8 : (shape == TILE_32x8 ? 32 : 16); }
int tile_ty(int shape) { return shape == TILE_8x8 ? 8 : (shape == TILE_32x8 ? 8 : 16); }

template <typename T>
struct Phys {
    T gamma, gm1, rho_floor, p_floor;
};

constexpr int tile_threads(int tx, int ty) { return tx * ty + ((2 * (tx + ty) + 63) / 64) * 64; }

template <int TX, int TY>
struct TileGeom {
    static constexpr int NINT = TX * TY;
    static constexpr int NRING = ((2 * (TX + TY) + 63) / 64) * 64;
    static constexpr int NT = NINT + NRING;
};

// ------------------------------------------------------------ cell physics

template <typename T>
__device__ __forceinline__ void prim_from_cons(const T U[5], T W[5], T &inv_rho,
                                               const Phys<T> &ph, int &hits)
{
    T rho = U[0];
    if (rho < ph.rho_floor) { rho = ph.rho_floor; ++hits; }
    T inv = T(1) / rho;
    T u = U[1] * inv, v = U[2] * inv, w = U[3] * inv;
    T kin = T(0.5) * (U[1] * u + U[2] * v + U[3] * w);
    T p = ph.gm1 * (U[4] - kin);
    if (p < ph.p_floor) { p = ph.p_floor; ++hits; }
    W[0] = rho; W[1] = u; W[2] = v; W[3] = w; W[4] = p;
    inv_rho = inv;
}

template <int LIM, typename T>
__device__ __forceinline__ T limited_slope(T a, T b)
{
    if constexpr (LIM == LIM_NONE) {
        return T(0.5) * (a + b);
    } else {
        bool pos = a > T(0) && b > T(0);
        bool neg = a < T(0) && b < T(0);
        if constexpr (LIM == LIM_MINMOD) {
            T m = fabs(a) <= fabs(b) ? a : b;
            return (pos || neg) ? m : T(0);
        } else {
            T m = fmin(fmin(T(2) * fabs(a), T(2) * fabs(b)), T(0.5) * fabs(a + b));
            return pos ? m : (neg ? -m : T(0));
        }
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
__device__ __forceinline__ void face_state(const T Ws[5], const T S[5], T sign, T out[5],
                                           const Phys<T> &ph, int &hits)
{
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q] = Ws[q] + sign * T(0.5) * S[q];
    if (out[0] < ph.rho_floor) { out[0] = ph.rho_floor; ++hits; }
    if (out[4] < ph.p_floor) { out[4] = ph.p_floor; ++hits; }
}

// ------------------------------------------------------------ Riemann fluxes
// States are rotated: (rho, u_n, u_t1, u_t2, p).

template <typename T>
__device__ __forceinline__ void hllc_rotated(const T L[5], const T R[5], const Phys<T> &ph, T F[5])
{
    const T g = ph.gamma;
    T cL = sqrt(g * L[4] / L[0]);
    T cR = sqrt(g * R[4] / R[0]);
    T SL = fmin(L[1] - cL, R[1] - cR);
    T SR = fmax(L[1] + cL, R[1] + cR);
    T mL = L[0] * (SL - L[1]);
    T mR = R[0] * (SR - R[1]);
    T Sst = (R[4] - L[4] + mL * L[1] - mR * R[1]) / (mL - mR);

    // Region logic in the order: S_L >= 0 -> F(L); S* >= 0 -> L star;
    // S_R > 0 -> R star; else F(R). The side K whose flux is the base:
    bool supL = SL >= T(0);
    bool left = supL || Sst >= T(0);
    bool star = !supL && (left || SR > T(0));
    T rK = left ? L[0] : R[0];
    T uK = left ? L[1] : R[1];
    T vK = left ? L[2] : R[2];
    T wK = left ? L[3] : R[3];
    T pK = left ? L[4] : R[4];
    T SK = left ? SL : SR;
    T mK = left ? mL : mR;

    T EK = pK / ph.gm1 + T(0.5) * rK * (uK * uK + vK * vK + wK * wK);
    T mass = rK * uK;
    T FK[5] = { mass, mass * uK + pK, mass * vK, mass * wK, uK * (EK + pK) };
    T UK[5] = { rK, rK * uK, rK * vK, rK * wK, EK };
    T a = mK / (SK - Sst);
    T e = EK / rK + (Sst - uK) * (Sst + pK / mK);
    T Us[5] = { a, a * Sst, a * vK, a * wK, a * e };
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        T Fs = FK[q] + SK * (Us[q] - UK[q]);
        F[q] = star ? Fs : FK[q];
    }
}

template <typename T>
__device__ __forceinline__ void euler_flux_rotated(const T W[5], const Phys<T> &ph, T F[5], T U[5])
{
    T E = W[4] / ph.gm1 + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
    T mass = W[0] * W[1];
    F[0] = mass; F[1] = mass * W[1] + W[4]; F[2] = mass * W[2]; F[3] = mass * W[3];
    F[4] = W[1] * (E + W[4]);
    U[0] = W[0]; U[1] = W[0] * W[1]; U[2] = W[0] * W[2]; U[3] = W[0] * W[3]; U[4] = E;
}

template <typename T>
__device__ __forceinline__ void hll_rotated(const T L[5], const T R[5], const Phys<T> &ph, T F[5])
{
    const T g = ph.gamma;
    T cL = sqrt(g * L[4] / L[0]);
    T cR = sqrt(g * R[4] / R[0]);
    T SL = fmin(L[1] - cL, R[1] - cR);
    T SR = fmax(L[1] + cL, R[1] + cR);
    T FL[5], FR[5], UL[5], UR[5];
    euler_flux_rotated(L, ph, FL, UL);
    euler_flux_rotated(R, ph, FR, UR);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        T Fm = (SR * FL[q] - SL * FR[q] + SL * SR * (UR[q] - UL[q])) / (SR - SL);
        F[q] = SL >= T(0) ? FL[q] : (SR <= T(0) ? FR[q] : Fm);
    }
}

// Flux through a face normal to direction d (0, 1, 2; may differ per lane)
// from unrotated primitive states. The transverse components follow the
// cyclic order (d+1, d+2).
template <int RS, typename T>
__device__ __forceinline__ void face_flux(int d, const T WL[5], const T WR[5], const Phys<T> &ph,
                                          T F[5])
{
    T L[5], R[5], G[5];
    L[0] = WL[0]; R[0] = WR[0]; L[4] = WL[4]; R[4] = WR[4];
    L[1] = d == 0 ? WL[1] : (d == 1 ? WL[2] : WL[3]);
    L[2] = d == 0 ? WL[2] : (d == 1 ? WL[3] : WL[1]);
    L[3] = d == 0 ? WL[3] : (d == 1 ? WL[1] : WL[2]);
    R[1] = d == 0 ? WR[1] : (d == 1 ? WR[2] : WR[3]);
    R[2] = d == 0 ? WR[2] : (d == 1 ? WR[3] : WR[1]);
    R[3] = d == 0 ? WR[3] : (d == 1 ? WR[1] : WR[2]);
    if constexpr (RS == RS_HLL) hll_rotated(L, R, ph, G);
    else hllc_rotated(L, R, ph, G);
    F[0] = G[0]; F[4] = G[4];
    F[1] = d == 0 ? G[1] : (d == 1 ? G[3] : G[2]);
    F[2] = d == 0 ? G[2] : (d == 1 ? G[1] : G[3]);
    F[3] = d == 0 ? G[3] : (d == 1 ? G[2] : G[1]);
}

// ------------------------------------------------------------ addressing

__device__ __forceinline__ int wrap_once(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct InputView {
    int64_t vstride;          // elements between variables
    int32_t sy, sz;           // row and plane strides
    int32_t nx, ny, nz, ng, periodic;

    __device__ __forceinline__ int64_t cell(int i, int j, int k) const
    {
        if (periodic) {
            i = wrap_once(wrap_once(i, nx), nx);
            j = wrap_once(wrap_once(j, ny), ny);
            k = wrap_once(wrap_once(k, nz), nz);
            return (int64_t)k * sz + (int64_t)j * sy + i;
        }
        return (int64_t)(k + ng) * sz + (int64_t)(j + ng) * sy + (i + ng);
    }
};

__device__ __forceinline__ InputView make_view(const PatchDesc &P)
{
    InputView v;
    v.nx = P.nx; v.ny = P.ny; v.nz = P.nz; v.ng = P.ng; v.periodic = P.periodic;
    int gx = P.periodic ? P.nx : P.nx + 2 * P.ng;
    int gy = P.periodic ? P.ny : P.ny + 2 * P.ng;
    int gz = P.periodic ? P.nz : P.nz + 2 * P.ng;
    v.sy = gx;
    v.sz = gx * gy;
    v.vstride = (int64_t)gx * gy * gz;
    return v;
}

template <typename T>
__device__ __forceinline__ void load_cons(const T *__restrict__ u, const InputView &v, int i, int j,
                                          int k, T U[5])
{
    int64_t c = v.cell(i, j, k);
#pragma unroll
    for (int q = 0; q < 5; ++q) U[q] = u[c + q * v.vstride];
}

// ------------------------------------------------------------ the tile march

template <typename T, int TX, int TY>
struct TileSmem {
    T w[5][TY + 4][TX + 4];     // primitives of the plane, two-deep halo
    T xp[5][TY][TX + 1];        // x+ face state of cell i-1 at [i]
    T yp[5][TY + 1][TX];        // y+ face state of cell j-1 at [j]
    T fx[5][TY][TX + 1];        // x flux through face i-1/2 at [i]
    T fy[5][TY + 1][TX];        // y flux through face j-1/2 at [j]
};

enum { ROLE_NONE = -1, ROLE_INT = 0, ROLE_BOTTOM = 1, ROLE_TOP = 2, ROLE_LEFT = 3, ROLE_RIGHT = 4 };

template <typename T, int LIM, int RS, int TX, int TY>
__device__ void godunov_tile(const PatchDesc &P, const T *__restrict__ u_in_base,
                             T *__restrict__ u_out_base, T *__restrict__ bflux_base, T dtdx, T lam,
                             const Phys<T> &ph, int x0, int y0, int z0, int z1,
                             TileSmem<T, TX, TY> &sm, int &hits)
{
    using Geo = TileGeom<TX, TY>;
    const int tid = threadIdx.x;
    const int ax = min(TX, P.nx - x0);
    const int ay = min(TY, P.ny - y0);
    const InputView view = make_view(P);
    const T *__restrict__ uin = u_in_base + P.in_off;

    // ---- role of this thread
    int ci = 0, cj = 0, role = ROLE_NONE;
    if (tid < Geo::NINT) {
        ci = tid % TX;
        cj = tid / TX;
        if (ci < ax && cj < ay) role = ROLE_INT;
    } else {
        int r = tid - Geo::NINT;
        if (r < ax) { ci = r; cj = -1; role = ROLE_BOTTOM; }
        else if (r < 2 * ax) { ci = r - ax; cj = ay; role = ROLE_TOP; }
        else if (r < 2 * ax + ay) { ci = -1; cj = r - 2 * ax; role = ROLE_LEFT; }
        else if (r < 2 * ax + 2 * ay) { ci = ax; cj = r - 2 * ax - ay; role = ROLE_RIGHT; }
    }
    const bool owner = role != ROLE_NONE;
    const bool interior = role == ROLE_INT;
    const int gi = x0 + ci, gj = y0 + cj;     // patch coordinates of the owned column

    // ---- depth-2 halo and depth-1 corner cells of a plane, one per thread
    int hi = 0, hj = 0;
    const int nhalo = 2 * ax + 2 * ay + 4;
    const bool halo = tid < nhalo;
    if (halo) {
        int h = tid;
        if (h < ax) { hi = h; hj = -2; }
        else if (h < 2 * ax) { hi = h - ax; hj = ay + 1; }
        else if (h < 2 * ax + ay) { hi = -2; hj = h - 2 * ax; }
        else if (h < 2 * ax + 2 * ay) { hi = ax + 1; hj = h - 2 * ax - ay; }
        else {
            int c = h - 2 * ax - 2 * ay;
            hi = (c & 1) ? ax : -1;
            hj = (c & 2) ? ay : -1;
        }
    }

    // boundary-flux sheets of this patch
    const bool want_flux = bflux_base != nullptr && P.flux_off >= 0;
    T *__restrict__ bf = want_flux ? bflux_base + P.flux_off : nullptr;
    const int64_t sxs = (int64_t)P.nz * P.ny, sys = (int64_t)P.nz * P.nx, szs = (int64_t)P.ny * P.nx;
    T *bxm = bf, *bxp = bf + 5 * sxs, *bym = bf + 10 * sxs, *byp = bym + 5 * sys;
    T *bzm = byp + 5 * sys, *bzp = bzm + 5 * szs;

    // ---- registers of the owned column
    T Wm[5], W0[5], Wp[5], inv0 = T(1), invp = T(1);
    T Ucur[5], Unext[5], Uprev[5];
    T zprev[5], dxy_prev[5], Fzm[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        Wm[q] = W0[q] = Wp[q] = T(0);
        Ucur[q] = Unext[q] = Uprev[q] = zprev[q] = dxy_prev[q] = Fzm[q] = T(0);
    }

    // prologue: planes z0-2 (interior only), z0-1 and z0
    if (owner) {
        T U[5], inv;
        if (interior) {
            load_cons(uin, view, gi, gj, z0 - 2, U);
            prim_from_cons(U, Wm, inv, ph, hits);
        }
        load_cons(uin, view, gi, gj, z0 - 1, U);
        prim_from_cons(U, W0, inv0, ph, hits);
        load_cons(uin, view, gi, gj, z0, Unext);
        prim_from_cons(Unext, Wp, invp, ph, hits);
    }

    const int lx = ci + 2, ly = cj + 2;
    for (int k = z0 - 1; k <= z1; ++k) {
        const bool pre = k < z0;
        const bool post = k == z1;

        if (!pre) {
            // shift the column registers and read plane k+1
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                Wm[q] = W0[q]; W0[q] = Wp[q];
                Uprev[q] = Ucur[q]; Ucur[q] = Unext[q];
            }
            inv0 = invp;
            if (interior || (owner && !post)) {
                load_cons(uin, view, gi, gj, k + 1, Unext);
                prim_from_cons(Unext, Wp, invp, ph, hits);
            }
        }

        // stage plane k in LDS
        if (owner) {
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.w[q][ly][lx] = W0[q];
        }
        if (!pre && !post && halo) {
            T U[5], Wh[5], invh;
            load_cons(uin, view, x0 + hi, y0 + hj, k, U);
            prim_from_cons(U, Wh, invh, ph, hits);
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.w[q][hj + 2][hi + 2] = Wh[q];
        }
        __syncthreads();

        if (pre || post) {
            // only the z face state of the interior is needed
            if (interior) {
                T Sx[5], Sy[5], Sz[5], Ws[5], st[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    T c = W0[q];
                    Sx[q] = limited_slope<LIM>(c - sm.w[q][ly][lx - 1], sm.w[q][ly][lx + 1] - c);
                    Sy[q] = limited_slope<LIM>(c - sm.w[q][ly - 1][lx], sm.w[q][ly + 1][lx] - c);
                    Sz[q] = limited_slope<LIM>(c - Wm[q], Wp[q] - c);
                }
                predictor(W0, inv0, Sx, Sy, Sz, lam, ph.gamma, Ws);
                if (pre) {
                    face_state(Ws, Sz, T(1), zprev, ph, hits);
                } else {
                    face_state(Ws, Sz, T(-1), st, ph, hits);
                    T Fz[5];
                    face_flux<RS>(2, zprev, st, ph, Fz);
                    if (want_flux && k == P.nz) {
#pragma unroll
                        for (int q = 0; q < 5; ++q) bzp[q * szs + (int64_t)gj * P.nx + gi] = Fz[q];
                    }
                    if (k > z0) {
                        T *out = u_out_base + P.out_off;
                        int64_t o = ((int64_t)(k - 1) * P.ny + gj) * P.nx + gi;
                        int64_t ostride = (int64_t)P.nx * P.ny * P.nz;
#pragma unroll
                        for (int q = 0; q < 5; ++q)
                            out[o + q * ostride] = Uprev[q] - dtdx * (dxy_prev[q] + (Fz[q] - Fzm[q]));
                    }
                }
            }
            __syncthreads();
            continue;
        }

        // ---- full plane: slopes, predictor, face states
        T xm[5], ym[5], zm[5], zp[5];
        if (owner) {
            T Sx[5], Sy[5], Sz[5], Ws[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                T c = W0[q];
                Sx[q] = limited_slope<LIM>(c - sm.w[q][ly][lx - 1], sm.w[q][ly][lx + 1] - c);
                Sy[q] = limited_slope<LIM>(c - sm.w[q][ly - 1][lx], sm.w[q][ly + 1][lx] - c);
                Sz[q] = limited_slope<LIM>(c - Wm[q], Wp[q] - c);
            }
            predictor(W0, inv0, Sx, Sy, Sz, lam, ph.gamma, Ws);
            T st[5];
            if (interior || role == ROLE_LEFT) {
                face_state(Ws, Sx, T(1), st, ph, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.xp[q][cj][ci + 1] = st[q];
            }
            if (interior || role == ROLE_BOTTOM) {
                face_state(Ws, Sy, T(1), st, ph, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.yp[q][cj + 1][ci] = st[q];
            }
            if (interior || role == ROLE_RIGHT) face_state(Ws, Sx, T(-1), xm, ph, hits);
            if (interior || role == ROLE_TOP) face_state(Ws, Sy, T(-1), ym, ph, hits);
            if (interior) {
                face_state(Ws, Sz, T(-1), zm, ph, hits);
                face_state(Ws, Sz, T(1), zp, ph, hits);
            }
        }
        __syncthreads();

        // ---- fluxes, each face once
        T Fz[5];
        if (interior) {
            T L[5], F[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) L[q] = sm.xp[q][cj][ci];
            face_flux<RS>(0, L, xm, ph, F);
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.fx[q][cj][ci] = F[q];
            if (want_flux && gi == 0) {
#pragma unroll
                for (int q = 0; q < 5; ++q) bxm[q * sxs + (int64_t)k * P.ny + gj] = F[q];
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) L[q] = sm.yp[q][cj][ci];
            face_flux<RS>(1, L, ym, ph, F);
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.fy[q][cj][ci] = F[q];
            if (want_flux && gj == 0) {
#pragma unroll
                for (int q = 0; q < 5; ++q) bym[q * sys + (int64_t)k * P.nx + gi] = F[q];
            }
            face_flux<RS>(2, zprev, zm, ph, Fz);
            if (want_flux && k == 0) {
#pragma unroll
                for (int q = 0; q < 5; ++q) bzm[q * szs + (int64_t)gj * P.nx + gi] = Fz[q];
            }
        } else if (role == ROLE_RIGHT || role == ROLE_TOP) {
            // the last x face (right ring) or y face (top ring) of the tile
            const bool isx = role == ROLE_RIGHT;
            T L[5], R[5], F[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                L[q] = isx ? sm.xp[q][cj][ax] : sm.yp[q][ay][ci];
                R[q] = isx ? xm[q] : ym[q];
            }
            face_flux<RS>(isx ? 0 : 1, L, R, ph, F);
            if (isx) {
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fx[q][cj][ax] = F[q];
                if (want_flux && gi == P.nx) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) bxp[q * sxs + (int64_t)k * P.ny + gj] = F[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fy[q][ay][ci] = F[q];
                if (want_flux && gj == P.ny) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) byp[q * sys + (int64_t)k * P.nx + gi] = F[q];
                }
            }
        }
        __syncthreads();

        // ---- x-y flux divergence; finish the plane below
        if (interior) {
            T dxy[5];
#pragma unroll
            for (int q = 0; q < 5; ++q)
                dxy[q] = (sm.fx[q][cj][ci + 1] - sm.fx[q][cj][ci]) + (sm.fy[q][cj + 1][ci] - sm.fy[q][cj][ci]);
            if (k > z0) {
                T *out = u_out_base + P.out_off;
                int64_t o = ((int64_t)(k - 1) * P.ny + gj) * P.nx + gi;
                int64_t ostride = (int64_t)P.nx * P.ny * P.nz;
#pragma unroll
                for (int q = 0; q < 5; ++q)
                    out[o + q * ostride] = Uprev[q] - dtdx * (dxy_prev[q] + (Fz[q] - Fzm[q]));
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                dxy_prev[q] = dxy[q];
                Fzm[q] = Fz[q];
                zprev[q] = zp[q];
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ Phys<T> make_phys(const Scalars &sc)
{
    Phys<T> ph;
    ph.gamma = T(sc.gamma);
    ph.gm1 = T(sc.gamma - 1.0);
    ph.rho_floor = T(sc.rho_floor);
    ph.p_floor = T(sc.p_floor);
    return ph;
}

__device__ __forceinline__ void flush_hits(int hits, unsigned long long *counter)
{
    if (hits) atomicAdd(counter, (unsigned long long)hits);
}

// One patch: blockIdx.x enumerates (segment, tile) with the z segment
// fastest, so consecutive workgroups share halo planes in L2.
template <typename T, int LIM, int RS, int TX, int TY>
__global__ __launch_bounds__(tile_threads(TX, TY)) void step_kernel(
    PatchDesc P, const T *__restrict__ u_in, T *__restrict__ u_out, T *__restrict__ bflux,
    const double *__restrict__ dt_dev, Scalars sc, unsigned long long *hits_ctr, int ntx, int nseg,
    int zlen)
{
    __shared__ TileSmem<T, TX, TY> sm;
    const Phys<T> ph = make_phys<T>(sc);
    const double dt = dt_dev ? *dt_dev : P.dt;
    const T dtdx = T(dt / P.dx), lam = T(dt / (2.0 * P.dx));
    const int item = blockIdx.x;
    const int seg = item % nseg;
    const int tile = item / nseg;
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int z0 = seg * zlen, z1 = min(z0 + zlen, P.nz);
    int hits = 0;
    godunov_tile<T, LIM, RS, TX, TY>(P, u_in, u_out, bflux, dtdx, lam, ph, x0, y0, z0, z1, sm, hits);
    flush_hits(hits, hits_ctr);
}

// A batch: a persistent grid; each workgroup pulls (patch, tile, z-range)
// items from an atomic counter until the table is exhausted. The last
// workgroup to leave resets the counter, so the next launch (or graph replay)
// starts from zero without a separate reset.
template <typename T, int LIM, int RS, int TX, int TY>
__global__ __launch_bounds__(tile_threads(TX, TY)) void step_batched_kernel(
    const PatchDesc *__restrict__ patches, const WorkItem *__restrict__ items, int nitems,
    const T *__restrict__ u_in, T *__restrict__ u_out, T *__restrict__ bflux,
    const double *__restrict__ dt_dev, Scalars sc, unsigned long long *hits_ctr, unsigned *queue)
{
    __shared__ TileSmem<T, TX, TY> sm;
    __shared__ int s_item;
    const Phys<T> ph = make_phys<T>(sc);
    int hits = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&queue[0], 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const PatchDesc P = patches[w.patch];
        const double dt = dt_dev ? *dt_dev : P.dt;
        const T dtdx = T(dt / P.dx), lam = T(dt / (2.0 * P.dx));
        godunov_tile<T, LIM, RS, TX, TY>(P, u_in, u_out, bflux, dtdx, lam, ph, w.x0, w.y0, w.z0,
                                         w.z1, sm, hits);
        __syncthreads();
    }
    flush_hits(hits, hits_ctr);
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned done = atomicAdd(&queue[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
        }
    }
}

// ------------------------------------------------------------ CFL reduction

template <typename T>
__device__ __forceinline__ double cell_signal(const T U[5], const Phys<T> &ph, int &hits)
{
    T W[5], inv;
    prim_from_cons(U, W, inv, ph, hits);
    T c = sqrt(ph.gamma * W[4] / W[0]);
    return (double)(fabs(W[1]) + fabs(W[2]) + fabs(W[3]) + T(3) * c);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide max of v (>= 0) folded into *smax_bits; the last block turns it
// into dt = cfl / smax and resets the accumulators.
__device__ void cfl_finish(double v, double cfl, double *dt_out, unsigned long long *smax_bits,
                           unsigned *done)
{
    __shared__ double part[16];
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) m = fmax(m, part[i]);
        atomicMax(smax_bits, (unsigned long long)__double_as_longlong(m));
        __threadfence();
        unsigned t = atomicAdd(done, 1u);
        if (t == gridDim.x - 1) {
            unsigned long long b = atomicAdd(smax_bits, 0ull);
            *dt_out = cfl / __longlong_as_double((long long)b);
            atomicExch(smax_bits, 0ull);
            atomicExch(done, 0u);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void cfl_kernel(const PatchDesc *__restrict__ patches,
                                                  const CflItem *__restrict__ items, int nitems,
                                                  const T *__restrict__ u, Scalars sc, double cfl,
                                                  double *dt_out, unsigned long long *smax_bits,
                                                  unsigned *done, unsigned long long *hits_ctr)
{
    const Phys<T> ph = make_phys<T>(sc);
    double vmax = 0.0;
    int hits = 0;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const CflItem c = items[it];
        const PatchDesc P = patches[c.patch];
        const InputView view = make_view(P);
        const T *base = u + P.in_off;
        const double inv_dx = 1.0 / P.dx;
        const int n = c.nrow * P.nx;
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            int i = e % P.nx, j = c.j0 + e / P.nx;
            T U[5];
            load_cons(base, view, i, j, c.k, U);
            vmax = fmax(vmax, cell_signal(U, ph, hits) * inv_dx);
        }
    }
    (void)hits_ctr;
    cfl_finish(vmax, cfl, dt_out, smax_bits, done);
}

template <typename T>
__global__ __launch_bounds__(256) void cfl_single_kernel(PatchDesc P, const T *__restrict__ u,
                                                         Scalars sc, double cfl, double *dt_out,
                                                         unsigned long long *smax_bits,
                                                         unsigned *done)
{
    const Phys<T> ph = make_phys<T>(sc);
    const InputView view = make_view(P);
    const T *base = u + P.in_off;
    const double inv_dx = 1.0 / P.dx;
    const int64_t ncell = (int64_t)P.nx * P.ny * P.nz;
    double vmax = 0.0;
    int hits = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ncell;
         e += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(e % P.nx);
        int64_t r = e / P.nx;
        int j = (int)(r % P.ny), k = (int)(r / P.ny);
        T U[5];
        load_cons(base, view, i, j, k, U);
        vmax = fmax(vmax, cell_signal(U, ph, hits) * inv_dx);
    }
    cfl_finish(vmax, cfl, dt_out, smax_bits, done);
}

// ------------------------------------------------------------ launchers

template <typename T, int LIM, int RS, int TX, int TY>
static int launch_step_t(const PatchDesc &P, const void *u_in, void *u_out, void *bflux,
                         const double *dt_dev, const Scalars &sc, unsigned long long *hits,
                         int zlen, hipStream_t s)
{
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    const int nseg = (P.nz + zlen - 1) / zlen;
    const int64_t nblocks = (int64_t)ntx * nty * nseg;
    if (nblocks <= 0 || nblocks > 0x7fffffff) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((step_kernel<T, LIM, RS, TX, TY>), dim3((unsigned)nblocks),
                       dim3(TileGeom<TX, TY>::NT), 0, s, P, (const T *)u_in, (T *)u_out, (T *)bflux,
                       dt_dev, sc, hits, ntx, nseg, zlen);
    return (int)hipGetLastError();
}

template <typename T, int LIM, int RS, int TX, int TY>
static int launch_batched_t(const PatchDesc *d_patches, const WorkItem *d_items, int nitems,
                            const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                            const Scalars &sc, unsigned long long *hits, unsigned *d_queue,
                            int grid, hipStream_t s)
{
    hipLaunchKernelGGL((step_batched_kernel<T, LIM, RS, TX, TY>), dim3(grid),
                       dim3(TileGeom<TX, TY>::NT), 0, s, d_patches, d_items, nitems,
                       (const T *)u_in, (T *)u_out, (T *)bflux, dt_dev, sc, hits, d_queue);
    return (int)hipGetLastError();
}

template <typename T, int LIM, int RS>
static int dispatch_shape_step(int shape, const PatchDesc &P, const void *u_in, void *u_out,
                               void *bflux, const double *dt_dev, const Scalars &sc,
                               unsigned long long *hits, int zlen, hipStream_t s)
{
    switch (shape) {
    case TILE_8x8: return launch_step_t<T, LIM, RS, 8, 8>(P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, s);
    case TILE_32x8: return launch_step_t<T, LIM, RS, 32, 8>(P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, s);
    default: return launch_step_t<T, LIM, RS, 16, 16>(P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, s);
    }
}

template <typename T, int LIM, int RS>
static int dispatch_shape_batched(int shape, const PatchDesc *d_patches, const WorkItem *d_items,
                                  int nitems, const void *u_in, void *u_out, void *bflux,
                                  const double *dt_dev, const Scalars &sc,
                                  unsigned long long *hits, unsigned *d_queue, int grid,
                                  hipStream_t s)
{
    switch (shape) {
    case TILE_8x8: return launch_batched_t<T, LIM, RS, 8, 8>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, s);
    case TILE_32x8: return launch_batched_t<T, LIM, RS, 32, 8>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, s);
    default: return launch_batched_t<T, LIM, RS, 16, 16>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, s);
    }
}

#define GD_DISPATCH_SCHEME(FN, T, ...)                                              \
    do {                                                                            \
        if (riemann == RS_HLL) {                                                    \
            if (limiter == LIM_MC) return FN<T, LIM_MC, RS_HLL>(__VA_ARGS__);       \
            if (limiter == LIM_NONE) return FN<T, LIM_NONE, RS_HLL>(__VA_ARGS__);   \
            return FN<T, LIM_MINMOD, RS_HLL>(__VA_ARGS__);                          \
        }                                                                           \
        if (limiter == LIM_MC) return FN<T, LIM_MC, RS_HLLC>(__VA_ARGS__);          \
        if (limiter == LIM_NONE) return FN<T, LIM_NONE, RS_HLLC>(__VA_ARGS__);      \
        return FN<T, LIM_MINMOD, RS_HLLC>(__VA_ARGS__);                             \
    } while (0)

int launch_step(int dtype, int limiter, int riemann, int shape, const PatchDesc &P,
                const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                const Scalars &sc, unsigned long long *hits, int zlen, hipStream_t s)
{
    if (dtype == 1)
        GD_DISPATCH_SCHEME(dispatch_shape_step, float, shape, P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, s);
    GD_DISPATCH_SCHEME(dispatch_shape_step, double, shape, P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, s);
}

int launch_step_batched(int dtype, int limiter, int riemann, int shape,
                        const PatchDesc *d_patches, const WorkItem *d_items, int nitems,
                        const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                        const Scalars &sc, unsigned long long *hits, unsigned *d_queue, int grid,
                        hipStream_t s)
{
    if (dtype == 1)
        GD_DISPATCH_SCHEME(dispatch_shape_batched, float, shape, d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, s);
    GD_DISPATCH_SCHEME(dispatch_shape_batched, double, shape, d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, s);
}

int launch_cfl(int dtype, const PatchDesc *d_patches, const CflItem *d_items, int nitems,
               const void *u, const Scalars &sc, double cfl, double *dt_out,
               unsigned long long *smax_bits, unsigned *done, int grid, hipStream_t s)
{
    if (dtype == 1)
        hipLaunchKernelGGL(cfl_kernel<float>, dim3(grid), dim3(256), 0, s, d_patches, d_items,
                           nitems, (const float *)u, sc, cfl, dt_out, smax_bits, done, nullptr);
    else
        hipLaunchKernelGGL(cfl_kernel<double>, dim3(grid), dim3(256), 0, s, d_patches, d_items,
                           nitems, (const double *)u, sc, cfl, dt_out, smax_bits, done, nullptr);
    return (int)hipGetLastError();
}

int launch_cfl_single(int dtype, const PatchDesc &P, const void *u, const Scalars &sc, double cfl,
                      double *dt_out, unsigned long long *smax_bits, unsigned *done,
                      hipStream_t s)
{
    const int64_t ncell = (int64_t)P.nx * P.ny * P.nz;
    int64_t blocks = (ncell + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    if (dtype == 1)
        hipLaunchKernelGGL(cfl_single_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, P,
                           (const float *)u, sc, cfl, dt_out, smax_bits, done);
    else
        hipLaunchKernelGGL(cfl_single_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, P,
                           (const double *)u, sc, cfl, dt_out, smax_bits, done);
    return (int)hipGetLastError();
}

template <typename T, int LIM, int RS>
static int occupancy_t(int shape, int device)
{
    (void)device;
    int n = 0;
    hipError_t e;
    switch (shape) {
    case TILE_8x8:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_batched_kernel<T, LIM, RS, 8, 8>, TileGeom<8, 8>::NT, 0);
        break;
    case TILE_32x8:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_batched_kernel<T, LIM, RS, 32, 8>, TileGeom<32, 8>::NT, 0);
        break;
    default:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_batched_kernel<T, LIM, RS, 16, 16>, TileGeom<16, 16>::NT, 0);
    }
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

int max_resident_blocks(int dtype, int limiter, int riemann, int shape, int device)
{
    if (dtype == 1) GD_DISPATCH_SCHEME(occupancy_t, float, shape, device);
    GD_DISPATCH_SCHEME(occupancy_t, double, shape, device);
}

}  // namespace gd
