// gfx950 kernels of the seams of a two-level AMR step around the batched
// Godunov step: ghost fill of the fine patches, refluxing at coarse-fine
// faces and averaging down (Sec. 3: the patches handed to the GPU carry
// boundary cells taken from the neighbouring grids; Sec. 4: the step returns
// the boundary fluxes that flux correction between levels needs).
//
// All three are gathers driven by tables the host builds once per hierarchy:
//   fill     one thread per coarse cell of the shell around a fine patch
//            (whose eight children are that patch's ghost cells): the
//            children from the fine patch covering the shell cell, else the
//            limited linear prolongation of the coarse cell;
//   reflux   one thread per side of each coarse-fine face recomputes that
//            side's predicted face state from the old coarse state (staged
//            in the plan's scratch); then one thread per uncovered coarse
//            cell next to a fine patch takes, face by face in a fixed order,
//            the coarse flux from those states and swaps it for the mean of
//            the four fine boundary fluxes;
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

// i in [-n, 2n): one conditional add or subtract, no division (fine ghost
// positions lie in [-2, 2 nc + 1) of a fine extent 2 nc >= 2)
__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// One thread per cell of the one-coarse-cell shell around a patch (its two
// fine ghost layers are exactly the eight children of each shell cell):
// the eight children come from the fine patch covering the shell cell, or
// from the limited linear prolongation of the coarse cell, whose slopes are
// computed once for all eight.
template <typename T>
__global__ __launch_bounds__(FILL_BLOCK) void fill_kernel(AmrTables t, const T *__restrict__ coarse,
                                                          T *__restrict__ fine)
{
    const AmrFillItem it = t.fill[blockIdx.x];
    const AmrPatch P = t.patches[it.patch];
    const int sx = P.n[0] / 2 + 2, sy = P.n[1] / 2 + 2, sz = P.n[2] / 2 + 2;
    const int idx = it.start + (int)threadIdx.x;
    if (idx >= sx * sy * sz) return;
    const int ci = idx % sx, cj = (idx / sx) % sy, ck = idx / (sx * sy);
    if (ci >= 1 && ci < sx - 1 && cj >= 1 && cj < sy - 1 && ck >= 1 && ck < sz - 1) return;
    const int nx = t.nc[0], ny = t.nc[1], nz = t.nc[2];
    // the shell cell, periodic over the coarse box
    const int cx = wrap(P.lo[0] + ci - 1, nx), cy = wrap(P.lo[1] + cj - 1, ny);
    const int cz = wrap(P.lo[2] + ck - 1, nz);
    const int cidx = (cz * ny + cy) * nx + cx;
    const int q = t.owner[cidx];
    const int gx = P.n[0] + 4, gy = P.n[1] + 4;
    const int64_t dvs = (int64_t)gx * gy * (P.n[2] + 4);
    // child (a, b, c) of the shell cell: ghost-box cell (2ci + a, 2cj + b, 2ck + c)
    T *dst = fine + P.in_off + ((int64_t)(2 * ck) * gy + 2 * cj) * gx + 2 * ci;
    if (q >= 0) {
        // the fine patch covering the shell cell holds all eight children
        const AmrPatch Q = t.patches[q];
        const int qx = Q.n[0] + 4, qy = Q.n[1] + 4;
        const int li = 2 * (cx - Q.lo[0]) + 2, lj = 2 * (cy - Q.lo[1]) + 2, lk = 2 * (cz - Q.lo[2]) + 2;
        const T *src = fine + Q.in_off + ((int64_t)lk * qy + lj) * qx + li;
        const int64_t vs = (int64_t)qx * qy * (Q.n[2] + 4);
#pragma unroll
        for (int c = 0; c < 5; ++c)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        dst[c * dvs + ((int64_t)k * gy + j) * gx + i] =
                            src[c * vs + ((int64_t)k * qy + j) * qx + i];
        return;
    }
    // limited linear prolongation: per variable the minmod slope along each
    // axis from the periodic neighbours; a child adds a quarter of each with
    // the sign of the half of the coarse cell it lies in, so the eight
    // children average back to the coarse value
    const int64_t vs = (int64_t)nx * ny * nz;
    const int ox = nx, oy = nx * ny;
    const int xm = cx > 0 ? -1 : nx - 1, xp = cx < nx - 1 ? 1 : 1 - nx;
    const int ym = cy > 0 ? -ox : (ny - 1) * ox, yp = cy < ny - 1 ? ox : (1 - ny) * ox;
    const int zm = cz > 0 ? -oy : (nz - 1) * oy, zp = cz < nz - 1 ? oy : (1 - nz) * oy;
    const T *c0 = coarse + cidx;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const T *u = c0 + c * vs;
        const T uc = u[0];
        const T Sx = limited_slope<LIM_MINMOD>(uc - u[xm], u[xp] - uc);
        const T Sy = limited_slope<LIM_MINMOD>(uc - u[ym], u[yp] - uc);
        const T Sz = limited_slope<LIM_MINMOD>(uc - u[zm], u[zp] - uc);
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const T tx = i ? Sx : -Sx, ty = j ? Sy : -Sy, tz = k ? Sz : -Sz;
                    dst[c * dvs + ((int64_t)k * gy + j) * gx + i] = uc + T(0.25) * ((tx + ty) + tz);
                }
    }
}

// Primitive state of coarse cell (x, y, z) of the periodic box.
template <typename T>
__device__ __forceinline__ void coarse_prim(const AmrTables &t, const T *__restrict__ u, int x, int y,
                                            int z, const Phys<T> &ph, T W[5], T &inv)
{
    const int64_t n = (int64_t)t.nc[0] * t.nc[1] * t.nc[2];
    // x, y, z lie in [-2, nc + 1): two conditional wraps cover nc >= 1
    const int c = (wrap(wrap(z, t.nc[2]), t.nc[2]) * t.nc[1] + wrap(wrap(y, t.nc[1]), t.nc[1])) * t.nc[0] +
                  wrap(wrap(x, t.nc[0]), t.nc[0]);
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

// Variable index of component k of a state rotated to (rho, u_n, u_t1,
// u_t2, p) with the cyclic order (d+1, d+2), as face_flux<RS, d> uses. The
// rotation is done through memory addresses: with runtime d, selects between
// register array elements are turned back into indexed private arrays.
__device__ __forceinline__ int rotated_var(int k, int d)
{
    if (k == 0 || k == 4) return k;
    int v = k + d;
    return v > 3 ? v - 3 : v;
}

// Thread g < nfaces: the left state of face g (upper face state of the cell
// below it along d); thread nfaces + g: its right state. Written to the
// plan's scratch, already rotated, as [side][component][face].
template <typename T, int LIM>
__global__ __launch_bounds__(SEAM_BLOCK) void face_state_kernel(AmrTables t,
                                                                const T *__restrict__ coarse_old,
                                                                Scalars sc, double dx, double dt_host,
                                                                const double *dt_dev)
{
    const int g = blockIdx.x * SEAM_BLOCK + threadIdx.x;
    if (g >= 2 * t.nfaces) return;
    // the two sides of a face in neighbouring lanes: their stencils share the
    // cells next to the face, so a wave fetches those lines once
    const int side = g & 1, f = g >> 1;
    const double dt = dt_dev ? *dt_dev : dt_host;
    const T lam = T(dt / (2.0 * dx));
    const Phys<T> ph = make_phys<T>(sc);
    const AmrFace fc = t.faces[f];
    const int d = fc.dside >> 1, r = fc.right;
    const int c[3] = { r % t.nc[0] - (d == 0 && !side), (r / t.nc[0]) % t.nc[1] - (d == 1 && !side),
                       r / (t.nc[0] * t.nc[1]) - (d == 2 && !side) };
    T W[5];
    coarse_face_state<T, LIM>(t, coarse_old, c, d, side ? T(-0.5) : T(0.5), lam, ph, W);
    T *fs = (T *)t.fstate + (int64_t)side * 5 * t.nfaces + f;
    // variable q sits at rotated component k with rotated_var(k, d) = q
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        int k = q;
        if (q >= 1 && q <= 3) k = q - d < 1 ? q - d + 3 : q - d;
        fs[(int64_t)k * t.nfaces] = W[q];
    }
}

// Threads below ncells: refluxing of one uncovered cell, its faces in table
// order (coarse flux from the staged face states, applied component by
// component in the rotated frame); the rest: averaging down of one covered
// cell.
template <typename T, int RS>
__global__ __launch_bounds__(SEAM_BLOCK) void seam_kernel(AmrTables t, T *__restrict__ coarse_new,
                                                          const T *__restrict__ fine_out,
                                                          const T *__restrict__ fine_flux,
                                                          Scalars sc, double dx, double dt_host,
                                                          const double *dt_dev)
{
    const int g = blockIdx.x * SEAM_BLOCK + threadIdx.x;
    const int64_t n = (int64_t)t.nc[0] * t.nc[1] * t.nc[2];
    if (g < t.ncells) {
        const double dt = dt_dev ? *dt_dev : dt_host;
        const T c = T(dt / dx);
        const Phys<T> ph = make_phys<T>(sc);
        T *U = coarse_new + t.cells[g];
        const T *fs = (const T *)t.fstate;
        for (int f = t.cell_start[g]; f < t.cell_start[g + 1]; ++f) {
            const AmrFace fc = t.faces[f];
            const int d = fc.dside >> 1, upper_side = fc.dside & 1;
            T Lr[5], Rr[5], G[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                Lr[k] = fs[(int64_t)k * t.nfaces + f];
                Rr[k] = fs[(int64_t)(5 + k) * t.nfaces + f];
            }
            riemann<RS>(Lr, Rr, ph, G);
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int q = rotated_var(k, d);
                const T *v = fine_flux + fc.fine + (int64_t)q * fc.vstride;
                T Ff = ((v[0] + v[1]) + (v[fc.row] + v[fc.row + 1])) * T(0.25);
                U[q * n] += upper_side ? c * (Ff - G[k]) : c * (G[k] - Ff);
            }
        }
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
    if (t.nfaces > 0) {
        hipLaunchKernelGGL((face_state_kernel<T, LIM>), dim3((2 * t.nfaces + SEAM_BLOCK - 1) / SEAM_BLOCK),
                           dim3(SEAM_BLOCK), 0, s, t, (const T *)coarse_old, sc, dx, dt, dt_dev);
        int e = (int)hipGetLastError();
        if (e) return e;
    }
    const int total = t.ncells + t.ncover;
    if (total == 0) return 0;
    hipLaunchKernelGGL((seam_kernel<T, RS>), dim3((total + SEAM_BLOCK - 1) / SEAM_BLOCK),
                       dim3(SEAM_BLOCK), 0, s, t, (T *)coarse_new, (const T *)fine_out,
                       (const T *)fine_flux, sc, dx, dt, dt_dev);
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
