// gfx950 kernels of one unsplit MUSCL-Hancock step of ideal MHD with
// hyperbolic-parabolic divergence cleaning (GLM), on a periodic box.
//
// The Euler step's method family (Sec. 2) carried to the MHD equations of the
// paper's Enzo solver (Sec. 4): conserved U = (rho, rho v, E, B, psi) with
// E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2; limited primitive slopes; the
// conservative MUSCL-Hancock half step, in which the upper- and lower-face
// values of a cell along each axis move by the same increment
//   dU = -dt/(2dx) sum_d [F_d(W + S_d/2) - F_d(W - S_d/2)];
// at every face the GLM 2x2 problem for (B_n, psi) fixes the normal field
//   B_n* = (B_nL + B_nR)/2 - (psi_R - psi_L)/(2 ch),
//   psi* = (psi_L + psi_R)/2 - ch (B_nR - B_nL)/2,
// whose fluxes are psi* and ch^2 B_n*, and the HLLD solver of Miyoshi and
// Kusano (2005) with that normal field gives the other seven fluxes; then
// U' = U - dt/dx ((dF_x + dF_y) + dF_z) and psi' <- psi' exp(-alpha ch dt/dx).
//
// Two launches per step over a library-owned scratch: predict (one thread per
// cell: 7-point stencil, slopes, half step, six predicted face states) and a
// flux sweep (z-marching column tiles: x and y faces through LDS, z faces in
// registers, the update, and optionally the signal speeds of the new state).
// Every value is written by one thread and the reductions are maxima:
// deterministic.
#include "godunov_internal.h"
#include "godunov_math.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

namespace mhd {

enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_NONE = 2 };
constexpr int NV = 9;

template <typename T>
struct Par {
    int nx, ny, nz, n;        // box and its cell count
    T gamma, gm1, inv_gm1, rho_floor, p_floor;
    T h;                      // dt / (2 dx)
    T c;                      // dt / dx
    T ch, ch2;                // cleaning speed and its square
    T damp;                   // exp(-alpha ch dt / dx)
};

// The step's time-dependent parameters (h, c, ch, ch^2, damp) when dt or ch
// come from device scalars: computed on the device by k_params, read by every
// kernel of the step.
template <typename T>
__device__ __forceinline__ void take_dynamic(Par<T> &P, const T *__restrict__ dyn)
{
    if (!dyn) return;
    P.h = dyn[0]; P.c = dyn[1]; P.ch = dyn[2]; P.ch2 = dyn[3]; P.damp = dyn[4];
}

template <typename T>
__device__ __forceinline__ T limited(int lim, T a, T b)
{
    if (lim == LIM_NONE) return T(0.5) * (a + b);
    if (!((a > T(0) && b > T(0)) || (a < T(0) && b < T(0)))) return T(0);
    if (lim == LIM_MINMOD) return fabs(a) <= fabs(b) ? a : b;
    T m = fmin(fmin(T(2) * fabs(a), T(2) * fabs(b)), T(0.5) * fabs(a + b));
    return a > T(0) ? m : -m;
}

// sqrt(x), x >= 0, from the hardware reciprocal square root refined by one
// Newton step (relative error within about 4e-15 in FP64)
template <typename T>
__device__ __forceinline__ T hw_sqrt(T x)
{
    return x > T(0) ? x * fast_rsqrt(x) : T(0);
}

// Divisions and square roots: EXACT = IEEE-rounded (the signal speeds behind
// dt and ch), else the refined hardware estimates (the step's arithmetic).
template <bool EXACT, typename T>
__device__ __forceinline__ void to_prim(const Par<T> &P, const T U[NV], T W[NV])
{
    T rho = U[0] < P.rho_floor ? P.rho_floor : U[0];
    T u, v, w;
    if constexpr (EXACT) {
        u = U[1] / rho; v = U[2] / rho; w = U[3] / rho;
    } else {
        const T ir = fast_rcp(rho);
        u = U[1] * ir; v = U[2] * ir; w = U[3] * ir;
    }
    T kin = T(0.5) * (U[1] * u + U[2] * v + U[3] * w);
    T mag = T(0.5) * (U[5] * U[5] + U[6] * U[6] + U[7] * U[7]);
    T p = P.gm1 * (U[4] - kin - mag);
    if (p < P.p_floor) p = P.p_floor;
    W[0] = rho; W[1] = u; W[2] = v; W[3] = w; W[4] = p;
    W[5] = U[5]; W[6] = U[6]; W[7] = U[7]; W[8] = U[8];
}

template <typename T>
__device__ __forceinline__ void to_cons(const Par<T> &P, const T W[NV], T U[NV])
{
    const T rho = W[0];
    U[0] = rho;
    U[1] = rho * W[1]; U[2] = rho * W[2]; U[3] = rho * W[3];
    U[4] = W[4] * P.inv_gm1 + T(0.5) * rho * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]) +
           T(0.5) * (W[5] * W[5] + W[6] * W[6] + W[7] * W[7]);
    U[5] = W[5]; U[6] = W[6]; U[7] = W[7]; U[8] = W[8];
}

// fast magnetosonic speed of the primitive state along the axis whose field
// component is bn
template <bool EXACT, typename T>
__device__ __forceinline__ T fast_speed(const Par<T> &P, const T W[NV], T bn)
{
    const T ir = EXACT ? T(1) / W[0] : fast_rcp(W[0]);
    const T a2 = P.gamma * W[4] * ir;
    const T b2 = (W[5] * W[5] + W[6] * W[6] + W[7] * W[7]) * ir;
    const T s = a2 + b2;
    T disc = s * s - T(4) * a2 * (bn * bn * ir);
    disc = disc < T(0) ? T(0) : disc;
    if constexpr (EXACT) return sqrt(T(0.5) * (s + sqrt(disc)));
    else return hw_sqrt(T(0.5) * (s + hw_sqrt(disc)));
}

// physical GLM-MHD flux along axis D
template <int D, typename T>
__device__ __forceinline__ void phys_flux(const Par<T> &P, const T W[NV], T F[NV])
{
    const T rho = W[0], p = W[4];
    const T un = W[1 + D], Bn = W[5 + D];
    const T B2 = W[5] * W[5] + W[6] * W[6] + W[7] * W[7];
    const T pT = p + T(0.5) * B2;
    const T uB = W[1] * W[5] + W[2] * W[6] + W[3] * W[7];
    const T E = p * P.inv_gm1 + T(0.5) * rho * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]) +
                T(0.5) * B2;
    F[0] = rho * un;
#pragma unroll
    for (int k = 0; k < 3; ++k) F[1 + k] = rho * un * W[1 + k] - Bn * W[5 + k] + (k == D ? pT : T(0));
    F[4] = (E + pT) * un - Bn * uB;
#pragma unroll
    for (int k = 0; k < 3; ++k) F[5 + k] = k == D ? W[8] : un * W[5 + k] - W[1 + k] * Bn;
    F[8] = P.ch2 * Bn;
}

// HLLD in the frame of the face: L, R = (rho, u_n, u_t1, u_t2, p, Bn, B_t1,
// B_t2) with the same Bn; fluxes of (rho, m_n, m_t1, m_t2, E, B_t1, B_t2).
template <typename T>
__device__ __forceinline__ void hlld(const Par<T> &P, const T L[8], const T R[8], T F[7])
{
    const T Bn = L[5];
    const T sgn = Bn > T(0) ? T(1) : (Bn < T(0) ? T(-1) : T(0));
    T Uc[2][8], Fc[2][7], pT[2], cf[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T *W = s ? R : L;
        const T rho = W[0], u = W[1], v = W[2], w = W[3], p = W[4], By = W[6], Bz = W[7];
        const T B2 = Bn * Bn + By * By + Bz * Bz;
        pT[s] = p + T(0.5) * B2;
        const T E = p * P.inv_gm1 + T(0.5) * rho * (u * u + v * v + w * w) + T(0.5) * B2;
        const T uB = u * Bn + v * By + w * Bz;
        Uc[s][0] = rho; Uc[s][1] = rho * u; Uc[s][2] = rho * v; Uc[s][3] = rho * w;
        Uc[s][4] = E; Uc[s][5] = Bn; Uc[s][6] = By; Uc[s][7] = Bz;
        Fc[s][0] = rho * u;
        Fc[s][1] = rho * u * u + pT[s] - Bn * Bn;
        Fc[s][2] = rho * u * v - Bn * By;
        Fc[s][3] = rho * u * w - Bn * Bz;
        Fc[s][4] = (E + pT[s]) * u - Bn * uB;
        Fc[s][5] = u * By - v * Bn;
        Fc[s][6] = u * Bz - w * Bn;
        const T Wf[NV] = { rho, u, v, w, p, Bn, By, Bz, T(0) };
        cf[s] = fast_speed<false>(P, Wf, Bn);
    }
    const T SL = fmin(L[1] - cf[0], R[1] - cf[1]);
    const T SR = fmax(L[1] + cf[0], R[1] + cf[1]);
    if (SL >= T(0)) {
        for (int q = 0; q < 7; ++q) F[q] = Fc[0][q];
        return;
    }
    if (SR <= T(0)) {
        for (int q = 0; q < 7; ++q) F[q] = Fc[1][q];
        return;
    }
    const T dL = (SL - L[1]) * L[0], dR = (SR - R[1]) * R[0];
    const T idd = fast_rcp(dR - dL);
    const T SM = (dR * R[1] - dL * L[1] - pT[1] + pT[0]) * idd;
    const T pTs = (dR * pT[0] - dL * pT[1] + dL * dR * (R[1] - L[1])) * idd;

    // single-star states
    T Us[2][8], sq[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T *W = s ? R : L;
        const T S = s ? SR : SL;
        const T rho = W[0], u = W[1], v = W[2], w = W[3], By = W[6], Bz = W[7];
        const T isd = fast_rcp(S - SM);
        const T rs = rho * (S - u) * isd;
        const T den = rho * (S - u) * (S - SM) - Bn * Bn;
        T vs = v, ws = w, Bys = By, Bzs = Bz;
        if (!(fabs(den) <= T(1e-12) * (rho * (S - u) * (S - u) + Bn * Bn))) {
            const T iden = fast_rcp(den);
            const T t = Bn * (SM - u) * iden;
            vs = v - By * t;
            ws = w - Bz * t;
            const T q = (rho * (S - u) * (S - u) - Bn * Bn) * iden;
            Bys = By * q;
            Bzs = Bz * q;
        }
        const T uB = u * Bn + v * By + w * Bz;
        const T uBs = SM * Bn + vs * Bys + ws * Bzs;
        const T Es = ((S - u) * Uc[s][4] - pT[s] * u + pTs * SM + Bn * (uB - uBs)) * isd;
        Us[s][0] = rs; Us[s][1] = rs * SM; Us[s][2] = rs * vs; Us[s][3] = rs * ws;
        Us[s][4] = Es; Us[s][5] = Bn; Us[s][6] = Bys; Us[s][7] = Bzs;
        sq[s] = hw_sqrt(rs);
    }
    const T SLs = SM - fabs(Bn) * fast_rcp(sq[0]);
    const T SRs = SM + fabs(Bn) * fast_rcp(sq[1]);
    // the side of the contact the face lies on: left when SM >= 0 (values are
    // selected, not indexed, so that everything stays in registers)
    const bool left = SM >= T(0);
    const T SK = left ? SL : SR;
    T UcK[8], UsK[8], Fs[7];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        UcK[q] = left ? Uc[0][q] : Uc[1][q];
        UsK[q] = left ? Us[0][q] : Us[1][q];
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const int c = q < 5 ? q : q + 1;
        Fs[q] = (left ? Fc[0][q] : Fc[1][q]) + SK * (UsK[c] - UcK[c]);
    }
    // outside the Alfven waves: the single-star flux of that side
    if ((left && SLs >= T(0)) || (!left && SRs <= T(0))) {
        for (int q = 0; q < 7; ++q) F[q] = Fs[q];
        return;
    }
    // between the Alfven waves: the double-star states
    const T irL = fast_rcp(Us[0][0]), irR = fast_rcp(Us[1][0]);
    const T vL = Us[0][2] * irL, wL = Us[0][3] * irL;
    const T vR = Us[1][2] * irR, wR = Us[1][3] * irR;
    const T ByL = Us[0][6], BzL = Us[0][7], ByR = Us[1][6], BzR = Us[1][7];
    const T iss = fast_rcp(sq[0] + sq[1]);
    const T vss = (sq[0] * vL + sq[1] * vR + (ByR - ByL) * sgn) * iss;
    const T wss = (sq[0] * wL + sq[1] * wR + (BzR - BzL) * sgn) * iss;
    const T Byss = (sq[0] * ByR + sq[1] * ByL + sq[0] * sq[1] * (vR - vL) * sgn) * iss;
    const T Bzss = (sq[0] * BzR + sq[1] * BzL + sq[0] * sq[1] * (wR - wL) * sgn) * iss;
    const T uBss = SM * Bn + vss * Byss + wss * Bzss;
    const T vK = left ? vL : vR, wK = left ? wL : wR;
    const T ByK = left ? ByL : ByR, BzK = left ? BzL : BzR;
    const T uBs = SM * Bn + vK * ByK + wK * BzK;
    const T rK = UsK[0], sqK = left ? sq[0] : sq[1];
    const T sgnK = left ? T(-1) : T(1);
    const T Uss[8] = { rK, rK * SM, rK * vss, rK * wss, UsK[4] + sgnK * sqK * (uBs - uBss) * sgn,
                       Bn, Byss, Bzss };
    const T SKs = left ? SLs : SRs;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const int c = q < 5 ? q : q + 1;
        F[q] = Fs[q] + SKs * (Uss[c] - UsK[c]);
    }
}

// GLM + HLLD flux through a face normal to D from unrotated primitive states
template <int D, typename T>
__device__ __forceinline__ void face_flux(const Par<T> &P, const T WL[NV], const T WR[NV], T F[NV])
{
    constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
    const T Bns = T(0.5) * (WL[5 + D] + WR[5 + D]) - (WR[8] - WL[8]) * fast_rcp(T(2) * P.ch);
    const T psis = T(0.5) * (WL[8] + WR[8]) - T(0.5) * P.ch * (WR[5 + D] - WL[5 + D]);
    const T L[8] = { WL[0], WL[1 + D], WL[1 + t1], WL[1 + t2], WL[4], Bns, WL[5 + t1], WL[5 + t2] };
    const T R[8] = { WR[0], WR[1 + D], WR[1 + t1], WR[1 + t2], WR[4], Bns, WR[5 + t1], WR[5 + t2] };
    T Fr[7];
    hlld(P, L, R, Fr);
    F[0] = Fr[0];
    F[1 + D] = Fr[1]; F[1 + t1] = Fr[2]; F[1 + t2] = Fr[3];
    F[4] = Fr[4];
    F[5 + D] = psis; F[5 + t1] = Fr[5]; F[5 + t2] = Fr[6];
    F[8] = P.ch2 * Bns;
}

__device__ __forceinline__ int wrap(int i, int n)
{
    if (i < 0) i += n;
    else if (i >= n) i -= n;
    if ((unsigned)i >= (unsigned)n) { i %= n; if (i < 0) i += n; }
    return i;
}

__device__ __forceinline__ int cell(int nx, int ny, int nz, int i, int j, int k)
{
    return (wrap(k, nz) * ny + wrap(j, ny)) * nx + wrap(i, nx);
}

template <bool EXACT, typename T>
__device__ __forceinline__ void load_prim(const Par<T> &P, const T *__restrict__ u, int c, T W[NV])
{
    T U[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) U[q] = u[q * P.n + c];
    to_prim<EXACT>(P, U, W);
}

// face-state scratch: fs[(d*2 + side)*9 + q][cell], side 0 the upper-face
// state W*+ and side 1 the lower-face state W*-; flux scratch: fl[d*9 + q][cell]
// holds the flux through the lower face of the cell along d.

// The upper- and lower-face values W +- S/2 of a cell along d, with the
// density and pressure floors.
template <typename T>
__device__ __forceinline__ void face_values(const Par<T> &P, const T W[NV], const T S[NV], T up[NV],
                                            T dn[NV])
{
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        up[q] = W[q] + T(0.5) * S[q];
        dn[q] = W[q] - T(0.5) * S[q];
    }
    up[0] = fmax(up[0], P.rho_floor); dn[0] = fmax(dn[0], P.rho_floor);
    up[4] = fmax(up[4], P.p_floor); dn[4] = fmax(dn[4], P.p_floor);
}

template <typename T, int LIM>
__global__ __launch_bounds__(256) void k_predict(Par<T> P, const T *__restrict__ dyn,
                                                 const T *__restrict__ u, T *__restrict__ fs)
{
    take_dynamic(P, dyn);
    const int i = blockIdx.x * 64 + threadIdx.x % 64;
    const int j = blockIdx.y * 4 + threadIdx.x / 64;
    const int k = blockIdx.z;
    if (i >= P.nx || j >= P.ny) return;
    const int c = (k * P.ny + j) * P.nx + i;
    T W[NV], dU[NV], S[3][NV];
    load_prim<false>(P, u, c, W);
#pragma unroll
    for (int q = 0; q < NV; ++q) dU[q] = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        {
            T Wm[NV], Wp[NV];
            load_prim<false>(P, u, cell(P.nx, P.ny, P.nz, i - (d == 0), j - (d == 1), k - (d == 2)), Wm);
            load_prim<false>(P, u, cell(P.nx, P.ny, P.nz, i + (d == 0), j + (d == 1), k + (d == 2)), Wp);
#pragma unroll
            for (int q = 0; q < NV; ++q) S[d][q] = limited<T>(LIM, W[q] - Wm[q], Wp[q] - W[q]);
        }
        T up[NV], dn[NV], Fu[NV], Fd[NV];
        face_values(P, W, S[d], up, dn);
        if (d == 0) { phys_flux<0>(P, up, Fu); phys_flux<0>(P, dn, Fd); }
        else if (d == 1) { phys_flux<1>(P, up, Fu); phys_flux<1>(P, dn, Fd); }
        else { phys_flux<2>(P, up, Fu); phys_flux<2>(P, dn, Fd); }
#pragma unroll
        for (int q = 0; q < NV; ++q) dU[q] -= Fu[q] - Fd[q];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T up[NV], dn[NV], Uu[NV], Ud[NV], Wu[NV], Wd[NV];
        face_values(P, W, S[d], up, dn);
        to_cons(P, up, Uu);
        to_cons(P, dn, Ud);
#pragma unroll
        for (int q = 0; q < NV; ++q) { Uu[q] += P.h * dU[q]; Ud[q] += P.h * dU[q]; }
        to_prim<false>(P, Uu, Wu);
        to_prim<false>(P, Ud, Wd);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            // streamed out: the sweep reads each value back once, long after
            __builtin_nontemporal_store(Wu[q], &fs[(size_t)((d * 2 + 0) * NV + q) * P.n + c]);
            __builtin_nontemporal_store(Wd[q], &fs[(size_t)((d * 2 + 1) * NV + q) * P.n + c]);
        }
    }
}

// ------------------------------------------------------------ flux sweep

// A workgroup owns a 16 x 16 column tile and marches up a z-range. Per plane,
// the predicted x-face states of the tile (and of one halo cell at each end
// of a row) are staged in LDS, every x face of the tile is evaluated once
// (faces on a tile border by both tiles) and its flux overwrites the left
// state it read; each cell takes its x flux difference; the same for y; the
// z face above a cell is evaluated in registers and serves the plane above
// as its lower face; then the update, and optionally the signal speeds of
// the new state for the next step's dt and cleaning speed.
constexpr int MTX = 16, MTY = 16, MT = MTX * MTY;
constexpr int MSLOT = (MTX + 1) * (MTY + 1);

template <typename T>
struct SweepSmem {
    T st[2][NV][MSLOT];      // [0] left state, then the flux; [1] right state
    double red[2][MT / 64];  // wave maxima of the speed reduction
};

template <typename T>
__device__ __forceinline__ void load_state(const Par<T> &P, const T *__restrict__ fs, int d,
                                           int side, int c, T W[NV])
{
#pragma unroll
    for (int q = 0; q < NV; ++q)
        W[q] = __builtin_nontemporal_load(&fs[(size_t)((d * 2 + side) * NV + q) * P.n + c]);
}

// Faces of one direction: slot s of the x pass is row s / (MTX+1), face
// s % (MTX+1) of that row (its right cell is tile column s % (MTX+1)); slot s
// of the y pass is column s % MTX, face s / MTX of that column.
template <int D, typename T>
__device__ __forceinline__ void sweep_pass(const Par<T> &P, const T *__restrict__ fs, int i, int j,
                                           int k, int tx, int ty, SweepSmem<T> &sm, T dF[NV])
{
    constexpr int NS = D == 0 ? (MTX + 1) * MTY : MTX * (MTY + 1);
    const int lo = D == 0 ? ty * (MTX + 1) + tx : ty * MTX + tx;        // the cell's lower face
    const int hi = D == 0 ? lo + 1 : lo + MTX;                         // its upper face
    const int c = cell(P.nx, P.ny, P.nz, i, j, k);
    {
        T W[NV];
        load_state(P, fs, D, 1, c, W);              // right state of the lower face
#pragma unroll
        for (int q = 0; q < NV; ++q) sm.st[1][q][lo] = W[q];
        load_state(P, fs, D, 0, c, W);              // left state of the upper face
#pragma unroll
        for (int q = 0; q < NV; ++q) sm.st[0][q][hi] = W[q];
        // the halo cells below the first and above the last cell of the row
        const int edge = D == 0 ? tx : ty;
        if (edge == 0) {
            load_state(P, fs, D, 0, cell(P.nx, P.ny, P.nz, i - (D == 0), j - (D == 1), k), W);
#pragma unroll
            for (int q = 0; q < NV; ++q) sm.st[0][q][lo] = W[q];
        }
        if (edge == (D == 0 ? MTX : MTY) - 1) {
            load_state(P, fs, D, 1, cell(P.nx, P.ny, P.nz, i + (D == 0), j + (D == 1), k), W);
#pragma unroll
            for (int q = 0; q < NV; ++q) sm.st[1][q][hi] = W[q];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NS; t += MT) {
        T WL[NV], WR[NV], F[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) { WL[q] = sm.st[0][q][t]; WR[q] = sm.st[1][q][t]; }
        face_flux<D>(P, WL, WR, F);
#pragma unroll
        for (int q = 0; q < NV; ++q) sm.st[0][q][t] = F[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) dF[q] = sm.st[0][q][hi] - sm.st[0][q][lo];
    __syncthreads();
}

// two waves per SIMD: the FP64 sweep sits at the 256-register limit
template <typename T>
__global__ __launch_bounds__(MT) __attribute__((amdgpu_waves_per_eu(2)))
void k_sweep(Par<T> P, const T *__restrict__ dyn,
                                              const T *__restrict__ u, const T *__restrict__ fs,
                                              T *__restrict__ out, int ntx, int nty, int zlen,
                                              int nitem, int per_xcd,
                                              unsigned long long *__restrict__ acc)
{
    __shared__ SweepSmem<T> sm;
    take_dynamic(P, dyn);
    // workgroups are dealt to the eight XCDs in turn: give each XCD a
    // contiguous range of work items, so that neighbouring tiles share its L2
    const int b = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (b >= nitem) return;
    const int bx = b % ntx, br = b / ntx;
    const int by = br % nty, bz = br / nty;
    const int tx = threadIdx.x % MTX, ty = threadIdx.x / MTX;
    const int i = bx * MTX + tx, j = by * MTY + ty;
    const bool own = i < P.nx && j < P.ny;
    const int k0 = bz * zlen, k1 = min(k0 + zlen, P.nz);

    // flux through the z face below the first plane
    T Flo[NV];
    {
        T WL[NV], WR[NV];
        load_state(P, fs, 2, 0, cell(P.nx, P.ny, P.nz, i, j, k0 - 1), WL);
        load_state(P, fs, 2, 1, cell(P.nx, P.ny, P.nz, i, j, k0), WR);
        face_flux<2>(P, WL, WR, Flo);
    }
    double smax = 0.0, dmax = 0.0;
    for (int k = k0; k < k1; ++k) {
        T dFx[NV], dFy[NV];
        sweep_pass<0>(P, fs, i, j, k, tx, ty, sm, dFx);
        sweep_pass<1>(P, fs, i, j, k, tx, ty, sm, dFy);
        T Fhi[NV];
        {
            T WL[NV], WR[NV];
            load_state(P, fs, 2, 0, cell(P.nx, P.ny, P.nz, i, j, k), WL);
            load_state(P, fs, 2, 1, cell(P.nx, P.ny, P.nz, i, j, k + 1), WR);
            face_flux<2>(P, WL, WR, Fhi);
        }
        if (own) {
            const int c = (k * P.ny + j) * P.nx + i;
            T U[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const T dFz = Fhi[q] - Flo[q];
                T v = u[(size_t)q * P.n + c] - P.c * ((dFx[q] + dFy[q]) + dFz);
                if (q == 8) v *= P.damp;
                __builtin_nontemporal_store(v, &out[(size_t)q * P.n + c]);
                U[q] = v;
            }
            if (acc) {
                T W[NV];
                to_prim<true>(P, U, W);
                double sum = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double v = (double)fabs(W[1 + d]) + (double)fast_speed<true>(P, W, W[5 + d]);
                    sum += v;
                    dmax = fmax(dmax, v);
                }
                smax = fmax(smax, sum);
            }
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) Flo[q] = Fhi[q];
    }
    if (!acc) return;
    // block maxima: wave maxima by shuffles, then the first wave over the waves
    for (int o = 32; o > 0; o >>= 1) {
        smax = fmax(smax, __shfl_xor(smax, o));
        dmax = fmax(dmax, __shfl_xor(dmax, o));
    }
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) { sm.red[0][w] = smax; sm.red[1][w] = dmax; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < MT / 64; ++q) {
            smax = fmax(smax, sm.red[0][q]);
            dmax = fmax(dmax, sm.red[1][q]);
        }
        atomicMax(&acc[0], (unsigned long long)__double_as_longlong(smax));
        atomicMax(&acc[1], (unsigned long long)__double_as_longlong(dmax));
    }
}

// max over cells of sum_d (|u_d| + cf_d) and of max_d (|u_d| + cf_d): block
// maxima through LDS, one atomicMax per block on the bit patterns of the
// non-negative doubles (which order like the values)
template <typename T>
__global__ __launch_bounds__(256) void k_speeds(Par<T> P, const T *__restrict__ u,
                                                unsigned long long *__restrict__ acc)
{
    __shared__ double red[2][256];
    double s = 0.0, m = 0.0;
    for (int c = blockIdx.x * 256 + threadIdx.x; c < P.n; c += gridDim.x * 256) {
        T W[NV];
        load_prim<true>(P, u, c, W);
        double sum = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = (double)fabs(W[1 + d]) + (double)fast_speed<true>(P, W, W[5 + d]);
            sum += v;
            m = fmax(m, v);
        }
        s = fmax(s, sum);
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&acc[0], (unsigned long long)__double_as_longlong(red[0][0]));
        atomicMax(&acc[1], (unsigned long long)__double_as_longlong(red[1][0]));
    }
}

// dt = cfl dx / smax and ch = max speed into device scalars; resets the
// accumulators for the next reduction
__global__ void k_speeds_finish(double cfl, double dx, unsigned long long *acc, double *dt_out,
                                double *ch_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double s = __longlong_as_double((long long)atomicExch(&acc[0], 0ull));
    const double m = __longlong_as_double((long long)atomicExch(&acc[1], 0ull));
    if (dt_out) *dt_out = cfl * dx / s;
    if (ch_out) *ch_out = m;
}

// dt and ch from device scalars (or the host values) -> the dynamic
// parameters (h, c, ch, ch^2, damp) of the step (one thread)
template <typename T>
__global__ void k_params(T *dyn, const double *dt_dev, const double *ch_dev, double dt_host,
                         double ch_host, double dx, double alpha)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double dt = dt_dev ? *dt_dev : dt_host;
    const double ch = ch_dev ? *ch_dev : ch_host;
    dyn[0] = (T)(dt / (2.0 * dx));
    dyn[1] = (T)(dt / dx);
    dyn[2] = (T)ch;
    dyn[3] = (T)(ch * ch);
    dyn[4] = (T)exp(-alpha * ch * dt / dx);
}

}  // namespace mhd

size_t mhd_scratch_bytes(int dtype, int nx, int ny, int nz)
{
    const size_t n = (size_t)nx * ny * nz;
    const size_t el = dtype == 0 ? 8 : 4;
    // six face states of 9 values per cell, plus the step's device-side
    // parameters
    return 6 * 9 * n * el + 512;
}

template <typename T>
static int run_mhd(int limiter, int nx, int ny, int nz, const void *u_in, void *u_out,
                   const MhdScalars &sc, const double *dt_dev, const double *ch_dev, void *scratch,
                   double cfl, double *dt_next, double *ch_next, unsigned long long *acc,
                   hipStream_t st)
{
    mhd::Par<T> P{};
    P.nx = nx; P.ny = ny; P.nz = nz; P.n = nx * ny * nz;
    P.gamma = (T)sc.gamma; P.gm1 = (T)(sc.gamma - 1.0); P.inv_gm1 = (T)(1.0 / (sc.gamma - 1.0));
    P.rho_floor = (T)sc.rho_floor; P.p_floor = (T)sc.p_floor;
    P.h = (T)(sc.dt / (2.0 * sc.dx));
    P.c = (T)(sc.dt / sc.dx);
    P.ch = (T)sc.ch; P.ch2 = (T)(sc.ch * sc.ch);
    P.damp = (T)exp(-sc.alpha * sc.ch * sc.dt / sc.dx);
    const size_t n = (size_t)P.n;
    T *fs = (T *)scratch;
    T *dyn = nullptr;
    if (dt_dev || ch_dev) {
        dyn = (T *)(((uintptr_t)(fs + 54 * n) + 255) & ~(uintptr_t)255);
        hipLaunchKernelGGL(mhd::k_params<T>, dim3(1), dim3(64), 0, st, dyn, dt_dev, ch_dev, sc.dt,
                           sc.ch, sc.dx, sc.alpha);
    }
    const T *u = (const T *)u_in;
    T *out = (T *)u_out;
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4, nz), block(256);
    switch (limiter) {
    case 1: hipLaunchKernelGGL((mhd::k_predict<T, 1>), grid, block, 0, st, P, dyn, u, fs); break;
    case 2: hipLaunchKernelGGL((mhd::k_predict<T, 2>), grid, block, 0, st, P, dyn, u, fs); break;
    default: hipLaunchKernelGGL((mhd::k_predict<T, 0>), grid, block, 0, st, P, dyn, u, fs); break;
    }
    // z-ranges: about 1024 work items, at least 2 planes each
    const int ntx = (nx + mhd::MTX - 1) / mhd::MTX, nty = (ny + mhd::MTY - 1) / mhd::MTY;
    int nseg = (1024 + ntx * nty - 1) / (ntx * nty);
    nseg = nseg < 1 ? 1 : (nseg > (nz + 1) / 2 ? (nz + 1) / 2 : nseg);
    const int zlen = (nz + nseg - 1) / nseg;
    nseg = (nz + zlen - 1) / zlen;
    const int nitem = ntx * nty * nseg, per_xcd = (nitem + 7) / 8;
    unsigned long long *a = dt_next || ch_next ? acc : nullptr;
    hipLaunchKernelGGL(mhd::k_sweep<T>, dim3(8 * per_xcd), dim3(mhd::MT), 0, st, P, dyn, u, fs, out,
                       ntx, nty, zlen, nitem, per_xcd, a);
    if (a)
        hipLaunchKernelGGL(mhd::k_speeds_finish, dim3(1), dim3(64), 0, st, cfl, sc.dx, a, dt_next,
                           ch_next);
    return (int)hipGetLastError();
}

int launch_mhd_step(int dtype, int limiter, int nx, int ny, int nz, const void *u_in, void *u_out,
                    const MhdScalars &sc, const double *dt_dev, const double *ch_dev,
                    void *scratch, double cfl, double *dt_next, double *ch_next,
                    unsigned long long *acc, hipStream_t s)
{
    if (dtype == 0)
        return run_mhd<double>(limiter, nx, ny, nz, u_in, u_out, sc, dt_dev, ch_dev, scratch, cfl,
                               dt_next, ch_next, acc, s);
    return run_mhd<float>(limiter, nx, ny, nz, u_in, u_out, sc, dt_dev, ch_dev, scratch, cfl,
                          dt_next, ch_next, acc, s);
}

template <typename T>
static int run_speeds(int nx, int ny, int nz, const void *u, const MhdScalars &sc, double cfl,
                      double *dt_dev, double *ch_dev, unsigned long long *acc, hipStream_t st)
{
    mhd::Par<T> P{};
    P.nx = nx; P.ny = ny; P.nz = nz; P.n = nx * ny * nz;
    P.gamma = (T)sc.gamma; P.gm1 = (T)(sc.gamma - 1.0); P.inv_gm1 = (T)(1.0 / (sc.gamma - 1.0));
    P.rho_floor = (T)sc.rho_floor; P.p_floor = (T)sc.p_floor;
    int blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(mhd::k_speeds<T>, dim3(blocks), dim3(256), 0, st, P, (const T *)u, acc);
    hipLaunchKernelGGL(mhd::k_speeds_finish, dim3(1), dim3(64), 0, st, cfl, sc.dx, acc, dt_dev,
                       ch_dev);
    return (int)hipGetLastError();
}

int launch_mhd_speeds(int dtype, int nx, int ny, int nz, const void *u, const MhdScalars &sc,
                      double cfl, double *dt_dev, double *ch_dev, unsigned long long *acc,
                      hipStream_t s)
{
    if (dtype == 0) return run_speeds<double>(nx, ny, nz, u, sc, cfl, dt_dev, ch_dev, acc, s);
    return run_speeds<float>(nx, ny, nz, u, sc, cfl, dt_dev, ch_dev, acc, s);
}

}  // namespace gd
