// gfx950 kernels of the seams of a two-level AMR step around the batched
// Godunov step: ghost fill of the fine patches, refluxing at coarse-fine
// faces and averaging down (Sec. 3: the patches handed to the GPU carry
// boundary cells taken from the neighbouring grids; Sec. 4: the step returns
// the boundary fluxes that flux correction between levels needs).
//
// All three are gathers driven by tables the host builds once per hierarchy:
//   fill     one thread per cell of a fine patch's ghosted box (interior
//            cells return at once): the value of the fine cell at the same
//            place if a fine patch covers it, else the coarse parent;
//   reflux   one thread per uncovered coarse cell that shares a face with a
//            fine patch: for each such face, in a fixed order, the coarse
//            flux is recomputed from the old coarse state and swapped for
//            the mean of the four fine boundary fluxes;
//   average  one thread per covered coarse cell: the mean of its eight
//            children, summed as a fixed pairwise tree.
// The work is a few percent of the step's and bound by latency and HBM
// gathers, so the kernels stay plain: no LDS staging, 32-bit indexing.
#include "godunov_cell.h"
#include "godunov_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

namespace {

constexpr int FILL_BLOCK = 256;
constexpr int SEAM_BLOCK = 128;

__device__ __forceinline__ int wrap(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

template <typename T>
__global__ __launch_bounds__(FILL_BLOCK) void fill_kernel(AmrTables t, const T *__restrict__ coarse,
                                                          T *__restrict__ fine)
{
    const AmrFillItem it = t.fill[blockIdx.x];
    const AmrPatch P = t.patches[it.patch];
    const int gx = P.n[0] + 4, gy = P.n[1] + 4, gz = P.n[2] + 4;
    const int box = gx * gy * gz;
    const int idx = it.start + (int)threadIdx.x;
    if (idx >= box) return;
    const int ii = idx % gx, jj = (idx / gx) % gy, kk = idx / (gx * gy);
    if (ii >= 2 && ii < gx - 2 && jj >= 2 && jj < gy - 2 && kk >= 2 && kk < gz - 2) return;
    // global fine cell, periodic over the fine extent of the coarse box
    const int fx = wrap(2 * P.lo[0] + ii - 2, 2 * t.nc[0]);
    const int fy = wrap(2 * P.lo[1] + jj - 2, 2 * t.nc[1]);
    const int fz = wrap(2 * P.lo[2] + kk - 2, 2 * t.nc[2]);
    const int cidx = ((fz >> 1) * t.nc[1] + (fy >> 1)) * t.nc[0] + (fx >> 1);
    const int q = t.owner[cidx];
    const T *src;
    int64_t vs;
    if (q >= 0) {
        const AmrPatch Q = t.patches[q];
        const int qx = Q.n[0] + 4, qy = Q.n[1] + 4;
        const int li = fx - 2 * Q.lo[0] + 2, lj = fy - 2 * Q.lo[1] + 2, lk = fz - 2 * Q.lo[2] + 2;
        src = fine + Q.in_off + ((int64_t)lk * qy + lj) * qx + li;
        vs = (int64_t)qx * qy * (Q.n[2] + 4);
    } else {
        src = coarse + cidx;
        vs = (int64_t)t.nc[0] * t.nc[1] * t.nc[2];
    }
    T *dst = fine + P.in_off + idx;
    const int64_t dvs = box;
    T v[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = src[c * vs];
#pragma unroll
    for (int c = 0; c < 5; ++c) dst[c * dvs] = v[c];
}

// Primitive state of coarse cell (x, y, z) of the periodic box.
template <typename T>
__device__ __forceinline__ void coarse_prim(const AmrTables &t, const T *__restrict__ u, int x, int y,
                                            int z, const Phys<T> &ph, T W[5], T &inv)
{
    const int64_t n = (int64_t)t.nc[0] * t.nc[1] * t.nc[2];
    const int c = (wrap(z, t.nc[2]) * t.nc[1] + wrap(y, t.nc[1])) * t.nc[0] + wrap(x, t.nc[0]);
    T U[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) U[q] = u[c + q * n];
    int unused = 0;
    prim_from_cons(U, W, inv, ph, unused);
}

// Predicted face state of coarse cell c on its upper (half = +1/2) or lower
// (half = -1/2) face along d: limited slopes on all three axes, the Hancock
// half step, then W* + half S_d -- the arithmetic of the step kernels.
template <typename T, int LIM>
__device__ __forceinline__ void coarse_face_state(const AmrTables &t, const T *__restrict__ u, const int c[3], int d,
                                  T half, T lam, const Phys<T> &ph, T out[5])
{
    T W[5], inv, S[3][5];
    coarse_prim(t, u, c[0], c[1], c[2], ph, W, inv);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T Wm[5], Wp[5], unused;
        coarse_prim(t, u, c[0] - (a == 0), c[1] - (a == 1), c[2] - (a == 2), ph, Wm, unused);
        coarse_prim(t, u, c[0] + (a == 0), c[1] + (a == 1), c[2] + (a == 2), ph, Wp, unused);
#pragma unroll
        for (int q = 0; q < 5; ++q) S[a][q] = limited_slope<LIM>(W[q] - Wm[q], Wp[q] - W[q]);
    }
    T Ws[5], Sd[5];
    predictor(W, inv, S[0], S[1], S[2], lam, ph.gamma, Ws);
    // value selects keep S in registers (a pointer select would not)
#pragma unroll
    for (int q = 0; q < 5; ++q) Sd[q] = d == 0 ? S[0][q] : (d == 1 ? S[1][q] : S[2][q]);
    int unused = 0;
    face_state(Ws, Sd, half, out, ph, unused);
}

template <typename T, int LIM, int RS>
__device__ __forceinline__ void coarse_face_flux(const AmrTables &t, const T *__restrict__ u, int right, int d,
                                 T lam, const Phys<T> &ph, T F[5])
{
    const int cr[3] = { right % t.nc[0], (right / t.nc[0]) % t.nc[1], right / (t.nc[0] * t.nc[1]) };
    const int cl[3] = { cr[0] - (d == 0), cr[1] - (d == 1), cr[2] - (d == 2) };
    T WL[5], WR[5];
    coarse_face_state<T, LIM>(t, u, cl, d, T(0.5), lam, ph, WL);
    coarse_face_state<T, LIM>(t, u, cr, d, T(-0.5), lam, ph, WR);
    // rotate to (rho, u_n, u_t1, u_t2, p) with the cyclic order (d+1, d+2),
    // as face_flux<RS, d> does, through value selects (a runtime axis index
    // into the state arrays would put them in private memory)
    T Lr[5] = { WL[0], d == 0 ? WL[1] : (d == 1 ? WL[2] : WL[3]),
               d == 0 ? WL[2] : (d == 1 ? WL[3] : WL[1]), d == 0 ? WL[3] : (d == 1 ? WL[1] : WL[2]),
               WL[4] };
    T Rr[5] = { WR[0], d == 0 ? WR[1] : (d == 1 ? WR[2] : WR[3]),
                d == 0 ? WR[2] : (d == 1 ? WR[3] : WR[1]), d == 0 ? WR[3] : (d == 1 ? WR[1] : WR[2]),
                WR[4] };
    T G[5];
    riemann<RS>(Lr, Rr, ph, G);
    F[0] = G[0];
    F[1] = d == 0 ? G[1] : (d == 1 ? G[3] : G[2]);
    F[2] = d == 0 ? G[2] : (d == 1 ? G[1] : G[3]);
    F[3] = d == 0 ? G[3] : (d == 1 ? G[2] : G[1]);
    F[4] = G[4];
}

template <typename T, int LIM, int RS>
__global__ __launch_bounds__(SEAM_BLOCK) void seam_kernel(AmrTables t, const T *__restrict__ coarse_old,
                                                          T *__restrict__ coarse_new,
                                                          const T *__restrict__ fine_out,
                                                          const T *__restrict__ fine_flux,
                                                          Scalars sc, double dx, double dt_host,
                                                          const double *dt_dev)
{
    const int g = blockIdx.x * SEAM_BLOCK + threadIdx.x;
    const int64_t n = (int64_t)t.nc[0] * t.nc[1] * t.nc[2];
    if (g < t.ncells) {
        const double dt = dt_dev ? *dt_dev : dt_host;
        const T c = T(dt / dx), lam = T(dt / (2.0 * dx));
        const Phys<T> ph = make_phys<T>(sc);
        const int o = t.cells[g];
        T U[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) U[q] = coarse_new[o + q * n];
        for (int f = t.cell_start[g]; f < t.cell_start[g + 1]; ++f) {
            const AmrFace fc = t.faces[f];
            const int d = fc.dside >> 1, upper_side = fc.dside & 1;
            T Fc[5];
            coarse_face_flux<T, LIM, RS>(t, coarse_old, fc.right, d, lam, ph, Fc);
            const T *b = fine_flux + fc.fine;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const T *v = b + (int64_t)q * fc.vstride;
                T Ff = ((v[0] + v[1]) + (v[fc.row] + v[fc.row + 1])) * T(0.25);
                U[q] += upper_side ? c * (Ff - Fc[q]) : c * (Fc[q] - Ff);
            }
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) coarse_new[o + q * n] = U[q];
        return;
    }
    const int a = g - t.ncells;
    if (a >= t.ncover) return;
    const AmrCover cv = t.cover[a];
    const AmrPatch P = t.patches[cv.patch];
    const int64_t sy = P.n[0], sz = (int64_t)P.n[0] * P.n[1], vs = sz * P.n[2];
    const T *ch = fine_out + cv.child;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T *v = ch + q * vs;
        T z0 = (v[0] + v[1]) + (v[sy] + v[sy + 1]);
        T z1 = (v[sz] + v[sz + 1]) + (v[sz + sy] + v[sz + sy + 1]);
        coarse_new[cv.coarse + q * n] = (z0 + z1) * T(0.125);
    }
}

__global__ void set_scalar_kernel(double *dst, double v) { *dst = v; }

template <typename T, int LIM, int RS>
int launch_seam_t(const AmrTables &t, const void *coarse_old, void *coarse_new, const void *fine_out,
                  const void *fine_flux, const Scalars &sc, double dx, double dt,
                  const double *dt_dev, hipStream_t s)
{
    const int total = t.ncells + t.ncover;
    if (total == 0) return 0;
    hipLaunchKernelGGL((seam_kernel<T, LIM, RS>), dim3((total + SEAM_BLOCK - 1) / SEAM_BLOCK),
                       dim3(SEAM_BLOCK), 0, s, t, (const T *)coarse_old, (T *)coarse_new,
                       (const T *)fine_out, (const T *)fine_flux, sc, dx, dt, dt_dev);
    return (int)hipGetLastError();
}

template <typename T>
int launch_seam_d(int limiter, int riemann, const AmrTables &t, const void *co, void *cn,
                  const void *fo, const void *ff, const Scalars &sc, double dx, double dt,
                  const double *dt_dev, hipStream_t s)
{
#define GD_SEAM(L, R) return launch_seam_t<T, L, R>(t, co, cn, fo, ff, sc, dx, dt, dt_dev, s)
    if (riemann == RS_HLL) {
        if (limiter == LIM_MINMOD) GD_SEAM(LIM_MINMOD, RS_HLL);
        if (limiter == LIM_MC) GD_SEAM(LIM_MC, RS_HLL);
        GD_SEAM(LIM_NONE, RS_HLL);
    }
    if (limiter == LIM_MINMOD) GD_SEAM(LIM_MINMOD, RS_HLLC);
    if (limiter == LIM_MC) GD_SEAM(LIM_MC, RS_HLLC);
    GD_SEAM(LIM_NONE, RS_HLLC);
#undef GD_SEAM
}

}  // namespace

int launch_amr_fill(int dtype, const AmrTables &t, const void *coarse, void *fine, hipStream_t s)
{
    if (t.nfill == 0) return 0;
    if (dtype == 1)
        hipLaunchKernelGGL(fill_kernel<float>, dim3(t.nfill), dim3(FILL_BLOCK), 0, s, t,
                           (const float *)coarse, (float *)fine);
    else
        hipLaunchKernelGGL(fill_kernel<double>, dim3(t.nfill), dim3(FILL_BLOCK), 0, s, t,
                           (const double *)coarse, (double *)fine);
    return (int)hipGetLastError();
}

int launch_amr_seam(int dtype, int limiter, int riemann, const AmrTables &t, const void *coarse_old,
                    void *coarse_new, const void *fine_out, const void *fine_flux,
                    const Scalars &sc, double dx_coarse, double dt, const double *dt_dev,
                    hipStream_t s)
{
    if (dtype == 1)
        return launch_seam_d<float>(limiter, riemann, t, coarse_old, coarse_new, fine_out, fine_flux,
                                    sc, dx_coarse, dt, dt_dev, s);
    return launch_seam_d<double>(limiter, riemann, t, coarse_old, coarse_new, fine_out, fine_flux,
                                 sc, dx_coarse, dt, dt_dev, s);
}

int launch_set_scalar(double *dst, double v, hipStream_t s)
{
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, s, dst, v);
    return (int)hipGetLastError();
}

}  // namespace gd
