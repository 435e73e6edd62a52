// gfx950 kernels of the Godunov step with piecewise-parabolic reconstruction
// (the PPM member of the reconstructions the paper lists beside PLM and TVD,
// Sec. 2; Enzo's hydro solver, Sec. 4).
//
// Per axis and primitive variable the parabola of Colella & Woodward (1984)
// replaces the limited slope of the PLM step: interface values
// a_{i+1/2} = (a_i + a_{i+1})/2 - (da_{i+1} - da_i)/6 with MC-limited (or,
// unlimited, central) slopes da, then -- limited variant -- flattening at a
// local extremum and the overshoot corrections a_L = 3a - 2a_R or
// a_R = 3a - 2a_L. The Hancock half step uses the slopes a_R - a_L; the face
// states are W* + (a_R - W) on the upper face and W* + (a_L - W) on the lower.
// With characteristic tracing (GD_PPM_CT, GD_PPM_CT_UNLIMITED) the face states
// along each axis come instead from the waves of the primitive system along
// that axis (speeds u - c, u, u + c): the edge value plus, for each wave moving
// towards the face, its eigenvector times its projection of (the parabolas'
// average over the part of the cell the wave sweeps in dt - the edge value)
// (Colella & Woodward 1984), plus the Hancock step's terms of the two other
// axes.
//
// A patch takes one launch per step (ppm_tile_kernel, the tile march of the
// PLM step with the parabola: the face states stay in LDS and registers), and
// so does a batch (ppm_batched_kernel: the same march over a persistent work
// queue of the batch's tiles). Periodic boxes thinner than two cells, whose
// wrapped stencils the march does not cover, take two launches per step over
// a scratch of 30 values per predicted cell:
//   ppm_predict  16 x 16 column tiles of the cells whose face states some
//                face needs (the interior and, for a ghosted patch, the face
//                ghosts of depth 1), marching in z: each plane converted to
//                primitives once into LDS, the column's z neighbours in
//                registers; per axis the five-cell stencil -> edges, then the
//                predictor and the six floored face states, stored SoA;
//   ppm_update   one thread per interior cell: its six face fluxes from the
//                staged states (a face shared by two cells is evaluated by
//                both from the same inputs, so both get the same bits), the
//                update, the boundary-flux sheets.
#include "godunov_cell.h"
#include "godunov_internal.h"
#include "godunov_tile.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace gd {

namespace {

constexpr int PPM_BLOCK = 256;
enum { PPM_LIMITED = 0, PPM_CENTRAL = 1 };

// Addressing of a patch's input: ghosted [5][nz+2ng][ny+2ng][nx+2ng], or a
// periodic box [5][nz][ny][nx] whose neighbours wrap (coordinates in
// [-2n, 3n) here).
struct Addr {
    int nx, ny, nz, ng, periodic;
    int gx, gy;
    int64_t vs;

    __device__ __forceinline__ static int wrap(int i, int n)
    {
        i = i < 0 ? i + n : (i >= n ? i - n : i);
        return i < 0 ? i + n : (i >= n ? i - n : i);
    }
    __device__ __forceinline__ int64_t at(int i, int j, int k) const
    {
        if (periodic) return ((int64_t)wrap(k, nz) * ny + wrap(j, ny)) * nx + wrap(i, nx);
        return ((int64_t)(k + ng) * gy + (j + ng)) * gx + (i + ng);
    }
};

__device__ __forceinline__ Addr make_addr(const PatchDesc &P)
{
    Addr a;
    a.nx = P.nx; a.ny = P.ny; a.nz = P.nz; a.ng = P.ng; a.periodic = P.periodic;
    a.gx = P.periodic ? P.nx : P.nx + 2 * P.ng;
    a.gy = P.periodic ? P.ny : P.ny + 2 * P.ng;
    const int gz = P.periodic ? P.nz : P.nz + 2 * P.ng;
    a.vs = (int64_t)a.gx * a.gy * gz;
    return a;
}

// The scratch box of a patch: the interior for a periodic box, the interior
// plus one layer (whose face-ghost cells are predicted) for a ghosted one.
struct Box {
    int e, bx, by, bz;
    int64_t n;
};

__device__ __forceinline__ Box make_box(const PatchDesc &P)
{
    Box b;
    b.e = P.periodic ? 0 : 1;
    b.bx = P.nx + 2 * b.e; b.by = P.ny + 2 * b.e; b.bz = P.nz + 2 * b.e;
    b.n = (int64_t)b.bx * b.by * b.bz;
    return b;
}

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

template <int MODE, typename T>
__device__ __forceinline__ T ppm_slope(T am, T a0, T ap)
{
    if constexpr (MODE == PPM_CENTRAL) return T(0.5) * (ap - am);
    else return limited_slope<LIM_MC>(a0 - am, ap - a0);
}

// Interface value between the cells holding a0 and ap.
template <int MODE, typename T>
__device__ __forceinline__ T ppm_interface(T am, T a0, T ap, T app)
{
    T d0 = ppm_slope<MODE>(am, a0, ap);
    T d1 = ppm_slope<MODE>(a0, ap, app);
    return T(0.5) * (a0 + ap) - div6(d1 - d0);
}

template <int MODE, typename T>
__device__ __forceinline__ void ppm_edges(T amm, T am, T a0, T ap, T app, T &aL, T &aR)
{
    T l = ppm_interface<MODE>(amm, am, a0, ap);
    T r = ppm_interface<MODE>(am, a0, ap, app);
    if constexpr (MODE == PPM_LIMITED) {
        if ((r - a0) * (a0 - l) <= T(0)) {
            l = a0;
            r = a0;
        } else {
            T D = r - l, m = a0 - T(0.5) * (l + r);
            // the threshold rounded as the division D^2 / 6 (and -(D^2) / 6 is
            // its exact negative), so that the branch matches the definition
            const T t = div6(D * D);
            if (D * m > t) l = T(3) * a0 - T(2) * r;
            else if (-t > D * m) r = T(3) * a0 - T(2) * l;
        }
    }
    aL = l;
    aR = r;
}

// The parabola's average over the last s of the cell minus a_R (upper face,
// s > 0), or over the first -s of the cell minus a_L (lower face, s < 0).
template <bool UPPER, typename T>
__device__ __forceinline__ T ppm_sweep_minus_edge(T aL, T aR, T a0, T s)
{
    const T da = aR - aL, a6 = T(6) * (a0 - T(0.5) * (aL + aR));
    if constexpr (UPPER) return T(-0.5) * s * (da - (T(1) - s * T(2.0 / 3.0)) * a6);
    else return T(-0.5) * s * (da + (T(1) + s * T(2.0 / 3.0)) * a6);
}

// The traced state on the upper (UPPER) or lower face along axis D of a cell
// with primitive state W, parabola edges aL, aR, sound speed c and 1/c, and
// dt/dx = cfl; eigenvectors in (rho, u_n, u_t1, u_t2, p):
// r_-+ = (1, -+c/rho, 0, 0, c^2), l_-+ = (0, -+rho/(2c), 0, 0, 1/(2c^2));
// entropy r = (1, 0, 0, 0, 0), l = (1, 0, 0, 0, -1/c^2); shear: the transverse
// velocities.
template <int D, bool UPPER, typename T>
__device__ __forceinline__ void ppm_trace(const T W[5], const T aL[5], const T aR[5], T c, T inv_c,
                                          T inv_rho, T cfl, T out[5])
{
    constexpr int n = 1 + D, t1 = 1 + (D + 1) % 3, t2 = 1 + (D + 2) % 3;
    const T un = W[n];
    const T s[3] = { (un - c) * cfl, un * cfl, (un + c) * cfl };
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q] = UPPER ? aR[q] : aL[q];
    const T half_rho_ic = T(0.5) * W[0] * inv_c, half_ic2 = T(0.5) * inv_c * inv_c;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        const bool towards = UPPER ? s[w] > T(0) : s[w] < T(0);
        if (!towards) continue;
        const T Dn = ppm_sweep_minus_edge<UPPER>(aL[n], aR[n], W[n], s[w]);
        const T Dp = ppm_sweep_minus_edge<UPPER>(aL[4], aR[4], W[4], s[w]);
        if (w == 1) {
            // entropy and shear waves
            out[0] += ppm_sweep_minus_edge<UPPER>(aL[0], aR[0], W[0], s[w]) -
                      T(2) * half_ic2 * Dp;
            out[t1] += ppm_sweep_minus_edge<UPPER>(aL[t1], aR[t1], W[t1], s[w]);
            out[t2] += ppm_sweep_minus_edge<UPPER>(aL[t2], aR[t2], W[t2], s[w]);
        } else {
            const T sg = w == 0 ? T(-1) : T(1);
            const T beta = sg * half_rho_ic * Dn + half_ic2 * Dp;
            out[0] += beta;
            out[n] += sg * c * inv_rho * beta;
            out[4] += c * c * beta;
        }
    }
}

// The Hancock half step's terms from the slopes a_R - a_L along axis D alone:
// W* - W = -dt/(2dx) (C_x + C_y + C_z), C_D = A_D(W) (a_R,D - a_L,D).
template <int D, typename T>
__device__ __forceinline__ void hancock_axis_term(const T W[5], T inv_rho, const T aL[5],
                                                  const T aR[5], T gamma, T C[5])
{
    constexpr int n = 1 + D;
    const T Sn = aR[n] - aL[n], Sp = aR[4] - aL[4];
#pragma unroll
    for (int q = 0; q < 5; ++q) C[q] = W[n] * (aR[q] - aL[q]);
    C[0] += W[0] * Sn;
    C[n] += Sp * inv_rho;
    C[4] += gamma * W[4] * Sn;
}

// The two face states of a cell along axis D by characteristic tracing, each
// with the Hancock terms of the two other axes (E1, E2), floored.
template <int D, int E1, int E2, typename T>
__device__ __forceinline__ void ppm_traced_faces(const T W[5], T inv_rho, const T aL[3][5],
                                                 const T aR[3][5], T c, T inv_c, T lam,
                                                 const Phys<T> &ph, T lo[5], T hi[5], int &hits)
{
    ppm_trace<D, false>(W, aL[D], aR[D], c, inv_c, inv_rho, T(2) * lam, lo);
    ppm_trace<D, true>(W, aL[D], aR[D], c, inv_c, inv_rho, T(2) * lam, hi);
    T C1[5], C2[5];
    hancock_axis_term<E1>(W, inv_rho, aL[E1], aR[E1], ph.gamma, C1);
    hancock_axis_term<E2>(W, inv_rho, aL[E2], aR[E2], ph.gamma, C2);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T tr = -lam * (C1[q] + C2[q]);
        lo[q] += tr;
        hi[q] += tr;
    }
    lo[0] = floored(lo[0], ph.rho_floor, hits);
    lo[4] = floored(lo[4], ph.p_floor, hits);
    hi[0] = floored(hi[0], ph.rho_floor, hits);
    hi[4] = floored(hi[4], ph.p_floor, hits);
}

template <typename T>
__device__ __forceinline__ void load_prim(const T *__restrict__ u, const Addr &A, int i, int j, int k,
                                          const Phys<T> &ph, T W[5], T &inv, int &hits)
{
    const int64_t o = A.at(i, j, k);
    T U[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) U[q] = u[o + q * A.vs];
    prim_from_cons(U, W, inv, ph, hits);
}

__device__ __forceinline__ void count_hits(int hits, unsigned long long *counter)
{
    if (hits) atomicAdd(counter, (unsigned long long)hits);
}

// Tiles of the predict kernel: PT x PT columns of the scratch box marching
// through up to PZ planes; each plane of the tile and a two-deep x-y halo is
// converted to primitives once and staged in LDS, and each column keeps the
// primitives of planes k-2 .. k+2 in registers.
constexpr int PT = 16, PZ = 16, PLW = PT + 4;
constexpr int PPM_HALO = PLW * PLW - PT * PT;          // 144 halo cells per plane

template <typename T>
struct PpmSmem {
    T w[5][PLW][PLW];
};

template <typename T>
__device__ __forceinline__ void load_raw(const T *__restrict__ u, const Addr &A, int i, int j, int k,
                                         T U[5])
{
    const int64_t o = A.at(i, j, k);
#pragma unroll
    for (int q = 0; q < 5; ++q) U[q] = u[o + q * A.vs];
}

// Two waves per SIMD: the FP64 tracing variant would otherwise take 256 VGPRs
// and 30-38 AGPRs (one wave) and runs 16% slower than with a few spills.
template <typename T, int MODE, bool CT>
__global__ __launch_bounds__(PT * PT) __attribute__((amdgpu_waves_per_eu(2))) void ppm_predict_kernel(
    PatchDesc P, const T *__restrict__ u_base, T *__restrict__ scratch, const double *dt_dev,
    Scalars sc, unsigned long long *hits_ctr)
{
    __shared__ PpmSmem<T> sm;
    int x0, y0, z0, z1;
    {
        const Box Bq = make_box(P);
        const int ntx = (Bq.bx + PT - 1) / PT, nty = (Bq.by + PT - 1) / PT;
        const int b = blockIdx.x, tile = b % (ntx * nty), seg = b / (ntx * nty);
        x0 = (tile % ntx) * PT;
        y0 = (tile / ntx) * PT;
        z0 = seg * PZ;
        z1 = min(z0 + PZ, Bq.bz);
    }
    const Box B = make_box(P);
    const Addr A = make_addr(P);
    const T *__restrict__ u = u_base + P.in_off;
    const Phys<T> ph = make_phys<T>(sc);
    const double dt = dt_dev ? *dt_dev : P.dt;
    const T lam = T(dt / (2.0 * P.dx));
    const int e = B.e;
    int hits = 0;

    // this thread's column (box coordinates bi, bj) and halo cell
    const int tid = threadIdx.x, ci = tid % PT, cj = tid / PT;
    const int bi = x0 + ci, bj = y0 + cj;
    // the stencils of the box's cells reach box coordinates -2 .. bx+1
    const bool col_load = bi <= B.bx + 1 && bj <= B.by + 1;
    int hx = 0, hy = 0;
    if (tid < 2 * PLW) { hy = tid / PLW; hx = tid % PLW; }
    else if (tid < 4 * PLW) { hy = PT + 2 + (tid - 2 * PLW) / PLW; hx = (tid - 2 * PLW) % PLW; }
    else if (tid < PPM_HALO) {
        const int r = tid - 4 * PLW, c = r & 3;
        hy = 2 + (r >> 2);
        hx = c < 2 ? c : PT + c;
    }
    const int hbi = x0 + hx - 2, hbj = y0 + hy - 2;
    const bool halo_load = tid < PPM_HALO && hbi <= B.bx + 1 && hbj <= B.by + 1;
    bool predicted = bi < B.bx && bj < B.by;
    if (!P.periodic) {
        const int i = bi - e, j = bj - e;
        const int di = i < 0 ? -i : (i >= P.nx ? i - P.nx + 1 : 0);
        const int dj = j < 0 ? -j : (j >= P.ny ? j - P.ny + 1 : 0);
        predicted = predicted && di + dj <= 1;
    }

    // z window of the column: planes zc-2 .. zc+2 of the current plane zc
    T win[5][5], winv[5], Upf[5], Hpf[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        winv[p] = T(1);
#pragma unroll
        for (int q = 0; q < 5; ++q) win[p][q] = T(0);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) Upf[q] = Hpf[q] = T(0);
    const int zc0 = z0 - e;
    if (col_load) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            T U[5];
            load_raw(u, A, bi - e, bj - e, zc0 - 2 + p, U);
            prim_from_cons(U, win[p], winv[p], ph, hits);
        }
        load_raw(u, A, bi - e, bj - e, zc0 + 2, Upf);
    }
    if (halo_load) load_raw(u, A, hbi - e, hbj - e, zc0, Hpf);

    const int lx = ci + 2, ly = cj + 2;
    for (int kb = z0; kb < z1; ++kb) {
        const int zc = kb - e;
        if (col_load) {
            prim_from_cons(Upf, win[4], winv[4], ph, hits);
            if (kb + 1 < z1) load_raw(u, A, bi - e, bj - e, zc + 3, Upf);
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.w[q][ly][lx] = win[2][q];
        }
        if (halo_load) {
            T Wh[5], invh;
            prim_from_cons(Hpf, Wh, invh, ph, hits);
            if (kb + 1 < z1) load_raw(u, A, hbi - e, hbj - e, zc + 1, Hpf);
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.w[q][hy][hx] = Wh[q];
        }
        __syncthreads();

        bool out_here = predicted;
        if (!P.periodic) {
            const int dk = zc < 0 ? -zc : (zc >= P.nz ? zc - P.nz + 1 : 0);
            const int i = bi - e, j = bj - e;
            const int di = i < 0 ? -i : (i >= P.nx ? i - P.nx + 1 : 0);
            const int dj = j < 0 ? -j : (j >= P.ny ? j - P.ny + 1 : 0);
            out_here = out_here && di + dj + dk <= 1;
        }
        if (out_here) {
            const T *W = win[2];
            T aL[3][5], aR[3][5], S[3][5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                ppm_edges<MODE>(sm.w[q][ly][lx - 2], sm.w[q][ly][lx - 1], W[q], sm.w[q][ly][lx + 1],
                                sm.w[q][ly][lx + 2], aL[0][q], aR[0][q]);
                ppm_edges<MODE>(sm.w[q][ly - 2][lx], sm.w[q][ly - 1][lx], W[q], sm.w[q][ly + 1][lx],
                                sm.w[q][ly + 2][lx], aL[1][q], aR[1][q]);
                ppm_edges<MODE>(win[0][q], win[1][q], W[q], win[3][q], win[4][q], aL[2][q], aR[2][q]);
#pragma unroll
                for (int d = 0; d < 3; ++d) S[d][q] = aR[d][q] - aL[d][q];
            }
            T *__restrict__ out = scratch + ((int64_t)kb * B.by + bj) * B.bx + bi;
            if constexpr (CT) {
                const T gp = ph.gamma * W[4];
                const T r = fast_rsqrt(gp * W[0]);
                const T c = gp * r, inv_c = W[0] * r;      // sqrt(gamma p / rho) and its inverse
                T lo[5], hi[5];
                ppm_traced_faces<0, 1, 2>(W, winv[2], aL, aR, c, inv_c, lam, ph, lo, hi, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    out[(int64_t)(0 * 5 + q) * B.n] = lo[q];
                    out[(int64_t)(1 * 5 + q) * B.n] = hi[q];
                }
                ppm_traced_faces<1, 0, 2>(W, winv[2], aL, aR, c, inv_c, lam, ph, lo, hi, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    out[(int64_t)(2 * 5 + q) * B.n] = lo[q];
                    out[(int64_t)(3 * 5 + q) * B.n] = hi[q];
                }
                ppm_traced_faces<2, 0, 1>(W, winv[2], aL, aR, c, inv_c, lam, ph, lo, hi, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    out[(int64_t)(4 * 5 + q) * B.n] = lo[q];
                    out[(int64_t)(5 * 5 + q) * B.n] = hi[q];
                }
            } else {
                T Ws[5];
                predictor(W, winv[2], S[0], S[1], S[2], lam, ph.gamma, Ws);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    T lo[5], hi[5];
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        lo[q] = Ws[q] + (aL[d][q] - W[q]);
                        hi[q] = Ws[q] + (aR[d][q] - W[q]);
                    }
                    lo[0] = floored(lo[0], ph.rho_floor, hits);
                    lo[4] = floored(lo[4], ph.p_floor, hits);
                    hi[0] = floored(hi[0], ph.rho_floor, hits);
                    hi[4] = floored(hi[4], ph.p_floor, hits);
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        out[(int64_t)((2 * d) * 5 + q) * B.n] = lo[q];
                        out[(int64_t)((2 * d + 1) * 5 + q) * B.n] = hi[q];
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            winv[p] = winv[p + 1];
#pragma unroll
            for (int q = 0; q < 5; ++q) win[p][q] = win[p + 1][q];
        }
    }
    count_hits(hits, hits_ctr);
}

// Scratch index of cell (i, j, k) of the box (periodic boxes wrap).
__device__ __forceinline__ int64_t box_at(const Box &B, const PatchDesc &P, int i, int j, int k)
{
    if (P.periodic) {
        i = i < 0 ? i + P.nx : (i >= P.nx ? i - P.nx : i);
        j = j < 0 ? j + P.ny : (j >= P.ny ? j - P.ny : j);
        k = k < 0 ? k + P.nz : (k >= P.nz ? k - P.nz : k);
        return ((int64_t)k * P.ny + j) * P.nx + i;
    }
    return ((int64_t)(k + 1) * B.by + (j + 1)) * B.bx + (i + 1);
}

template <typename T>
__device__ __forceinline__ void load_state(const T *__restrict__ s, int64_t n, int slot, T W[5])
{
#pragma unroll
    for (int q = 0; q < 5; ++q) W[q] = s[(int64_t)(slot * 5 + q) * n];
}

template <typename T, int RS>
__global__ __launch_bounds__(PPM_BLOCK) void ppm_update_kernel(
    PatchDesc P, const T *__restrict__ u_base, const T *__restrict__ scratch,
    T *__restrict__ out_base, T *__restrict__ bflux_base, const double *dt_dev, Scalars sc)
{
    const int start = blockIdx.x * PPM_BLOCK;
    const int64_t ncell = (int64_t)P.nx * P.ny * P.nz;
    const int idx = start + (int)threadIdx.x;
    if (idx >= ncell) return;
    const int i = idx % P.nx, j = (idx / P.nx) % P.ny, k = idx / (P.nx * P.ny);
    const Box B = make_box(P);
    const T *__restrict__ s = scratch;
    const Phys<T> ph = make_phys<T>(sc);
    const double dt = dt_dev ? *dt_dev : P.dt;
    const T c = T(dt / P.dx);
    const int64_t me = box_at(B, P, i, j, k);

    T Fm[3][5], Fp[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int di = d == 0, dj = d == 1, dk = d == 2;
        const int64_t left = box_at(B, P, i - di, j - dj, k - dk);
        const int64_t right = box_at(B, P, i + di, j + dj, k + dk);
        T WL[5], WR[5];
        load_state(s + left, B.n, 2 * d + 1, WL);
        load_state(s + me, B.n, 2 * d, WR);
        if (d == 0) face_flux<RS, 0>(WL, WR, ph, Fm[d]);
        else if (d == 1) face_flux<RS, 1>(WL, WR, ph, Fm[d]);
        else face_flux<RS, 2>(WL, WR, ph, Fm[d]);
        load_state(s + me, B.n, 2 * d + 1, WL);
        load_state(s + right, B.n, 2 * d, WR);
        if (d == 0) face_flux<RS, 0>(WL, WR, ph, Fp[d]);
        else if (d == 1) face_flux<RS, 1>(WL, WR, ph, Fp[d]);
        else face_flux<RS, 2>(WL, WR, ph, Fp[d]);
    }
    const Addr A = make_addr(P);
    const T *__restrict__ u = u_base + P.in_off + A.at(i, j, k);
    T *__restrict__ o = out_base + P.out_off + idx;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        T div = ((Fp[0][q] - Fm[0][q]) + (Fp[1][q] - Fm[1][q])) + (Fp[2][q] - Fm[2][q]);
        o[(int64_t)q * ncell] = u[(int64_t)q * A.vs] - c * div;
    }
    if (bflux_base && P.flux_off >= 0) {
        T *bf = bflux_base + P.flux_off;
        const int64_t sx = (int64_t)P.nz * P.ny, sy = (int64_t)P.nz * P.nx, sz = (int64_t)P.ny * P.nx;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            if (i == 0) bf[q * sx + (int64_t)k * P.ny + j] = Fm[0][q];
            if (i == P.nx - 1) bf[5 * sx + q * sx + (int64_t)k * P.ny + j] = Fp[0][q];
            if (j == 0) bf[10 * sx + q * sy + (int64_t)k * P.nx + i] = Fm[1][q];
            if (j == P.ny - 1) bf[10 * sx + 5 * sy + q * sy + (int64_t)k * P.nx + i] = Fp[1][q];
            if (k == 0) bf[10 * sx + 10 * sy + q * sz + (int64_t)j * P.nx + i] = Fm[2][q];
            if (k == P.nz - 1) bf[10 * sx + 10 * sy + 5 * sz + q * sz + (int64_t)j * P.nx + i] = Fp[2][q];
        }
    }
}


// ------------------------------------------------------------ fused PPM tile

// One launch per step for a single patch with the Hancock PPM reconstruction
// (GD_PPM, GD_PPM_UNLIMITED): the tile march of the PLM step kernel
// (godunov_tile) with the parabola in place of the limited slope, so that the
// face states never leave the chip. A workgroup owns a TX x TY column tile and
// a z-range; interior and ring columns keep planes k-2 .. k+2 of their column
// in registers, and each plane of the tile is staged in LDS with the cells of
// the five-point x and y stencils of its interior and ring cells (a halo three
// deep along the axes, 4TX + 4TY + 12 cells). Per plane k:
//   A  columns convert plane k+2 (loaded a plane earlier) and stage plane k;
//      halo threads stage their cell of plane k;
//   B  interior and ring columns: the parabola edges of the 15 primitives
//      (x and y stencils from LDS, z from registers), the Hancock predictor,
//      and the face states W* + (a_L - W) below and W* + (a_R - W) above,
//      floored; x and y states to LDS (a ring column only the state its face
//      with the tile needs), z states in registers;
//   C  the plane's x and y faces as in the PLM tile, then the z face below
//      the plane, which completes plane k-1 (and its CFL signal);
//   D  the x-y flux divergence of plane k.
// The pre plane z0-1 only produces the state below face z0-1/2's right side,
// the post plane z1 only the state that completes plane z1-1.
template <typename T, int TX, int TY>
struct PpmTileSmem {
    T w[5][TY + 6][TX + 6];                    // plane k, offset 3
    T fl[5][TileGeom<TX, TY>::NF];
    T fr[5][TileGeom<TX, TY>::NF];
};

template <int TX, int TY>
constexpr int ppm_halo_cells() { return 4 * TX + 4 * TY + 12; }

template <typename T, int MODE, bool CT, int RS, int TX, int TY, bool GHOSTED>
__device__ void ppm_tile(const PatchDesc &P, const T *__restrict__ u_in_base,
                         T *__restrict__ u_out_base, T *__restrict__ bflux_base, T dtdx, T lam,
                         const Phys<T> &ph, int x0, int y0, int z0, int z1,
                         PpmTileSmem<T, TX, TY> &sm, int &hits, bool want_cfl, double &smax)
{
    using Geo = TileGeom<TX, TY>;
    constexpr int NF = Geo::NF, NSLOT = Geo::NSLOT;
    static_assert(ppm_halo_cells<TX, TY>() <= Geo::NT, "one halo cell per thread at most");
    const int tid = threadIdx.x;
    const int ax = min(TX, P.nx - x0);
    const int ay = min(TY, P.ny - y0);
    const InputView view = make_view(P);
    const T *__restrict__ uin = u_in_base + P.in_off;

    // ---- role: an interior column, a ring column, or none
    int ci = 0, cj = 0, role = ROLE_NONE;
    if (tid < Geo::NINT) {
        ci = tid % TX;
        cj = tid / TX;
        if (ci < ax && cj < ay) role = ROLE_INT;
    } else {
        const int r = tid - Geo::NINT;
        if (r < ax) { ci = r; cj = -1; role = ROLE_BOTTOM; }
        else if (r < 2 * ax) { ci = r - ax; cj = ay; role = ROLE_TOP; }
        else if (r < 2 * ax + ay) { ci = -1; cj = r - 2 * ax; role = ROLE_LEFT; }
        else if (r < 2 * ax + 2 * ay) { ci = ax; cj = r - 2 * ax - ay; role = ROLE_RIGHT; }
    }
    const bool owner = role != ROLE_NONE;
    const bool interior = role == ROLE_INT;
    const int gi = x0 + ci, gj = y0 + cj;
    const int64_t col = view.column(gi, gj);

    // ---- the halo cell of this thread: the cells two deep beside the
    // interior rows and columns, then those three deep, then the twelve cells
    // around the ring's ends. In the pre and post planes only the interior's
    // stencils are evaluated, which reach the first group only; in a ghosted
    // patch the others are neither read nor staged there (so its corner
    // ghosts, and its edge ghosts three deep, are never read).
    int hi = 0, hj = 0;
    const int nhalo = 4 * ax + 4 * ay + 12;
    const bool halo = tid < nhalo;
    if (halo) {
        const int h = tid;
        if (h < 4 * ay + 4 * ax) {
            const int deep = h >= 2 * ay + 2 * ax;               // three deep
            const int g = h - (deep ? 2 * ay + 2 * ax : 0);
            const int far = g & 1;                               // right or top side
            if (g < 2 * ay) {
                hj = g >> 1;
                hi = far ? ax + 1 + deep : -2 - deep;
            } else {
                hi = (g - 2 * ay) >> 1;
                hj = far ? ay + 1 + deep : -2 - deep;
            }
        } else {
            const int c = h - 4 * ay - 4 * ax;          // 0 .. 11
            if (c < 8) {
                // rows -1 and ay: x = -2, -1, ax, ax+1
                const int w = c & 3;
                hj = c < 4 ? -1 : ay;
                hi = w < 2 ? w - 2 : ax + w - 2;
            } else {
                // columns -1 and ax, rows -2 and ay+1
                const int w = c - 8;
                hi = (w & 1) ? ax : -1;
                hj = (w & 2) ? ay + 1 : -2;
            }
        }
    }
    const int64_t hcol = view.column(x0 + hi, y0 + hj);

    // the faces this thread evaluates in phase C1, and whether each lies in
    // the clipped tile
    unsigned fact = 0;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        const int t = tid + s * Geo::NT;
        int i, j;
        const bool isx = Geo::face_ij(t, i, j);
        if (t < NF && (isx ? (i <= ax && j < ay) : (i < ax && j <= ay))) fact |= 1u << s;
    }

    const bool want_flux = bflux_base != nullptr && P.flux_off >= 0;
    T *__restrict__ bf = want_flux ? bflux_base + P.flux_off : nullptr;
    const int64_t sxs = (int64_t)P.nz * P.ny, sys = (int64_t)P.nz * P.nx, szs = (int64_t)P.ny * P.nx;
    T *__restrict__ out = u_out_base + P.out_off;
    const int64_t ostride = (int64_t)P.nx * P.ny * P.nz;
    const double inv_dx = 1.0 / P.dx;
    const int64_t ocol = (int64_t)gj * P.nx + gi;

    // ---- registers: the column's planes k-2 .. k+2, face-state carries
    T win[5][5], winv[5], Upf[5], Hpf[5], Uold[5];
    T zprev[5], acc[5], zm[5], zpn[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        winv[q] = T(1);
        Upf[q] = Hpf[q] = Uold[q] = zprev[q] = acc[q] = zm[q] = zpn[q] = T(0);
#pragma unroll
        for (int p = 0; p < 5; ++p) win[p][q] = T(0);
    }
    // Every column stages its cell of planes z0-1 .. z1 (the interior's x and
    // y stencils of the pre and post planes reach the ring), so every
    // column's window starts at plane z0-3; the last plane an interior column
    // reads is z1+2, a ring column z1+1 (it computes planes z0 .. z1-1).
    const int last_plane = interior ? z1 + 2 : z1 + 1;
    if (owner) {
        // planes z0-3 .. z0, and the load of plane z0+1, which the first
        // step converts into the window's top plane
        // (a ring column never uses plane z0-3: it computes from plane z0)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if (GHOSTED && p == 0 && !interior) continue;
            T U[5];
            load5(uin + view.plane(z0 - 3 + p) + col, view.vstride, U);
            prim_from_cons(U, win[p], winv[p], ph, hits);
        }
        load5(uin + view.plane(z0 + 1) + col, view.vstride, Upf);
    }
    if (GHOSTED ? tid < 2 * (ax + ay) : halo) load5(uin + view.plane(z0 - 1) + hcol, view.vstride, Hpf);

    const int lx = ci + 3, ly = cj + 3;
    for (int k = z0 - 1; k <= z1; ++k) {
        const bool pre = k < z0;
        const bool post = k == z1;
        // a ring column computes planes z0 .. z1-1 only
        const bool active = interior || (owner && !pre && !post);

        // ---- A: the column's plane k+2, stage plane k. Every thread has
        // finished reading the previous plane from LDS (phase B, then a
        // barrier) before it is overwritten here.
        if (owner) {
            if (k + 2 <= last_plane) prim_from_cons(Upf, win[4], winv[4], ph, hits);
            if (k + 3 <= last_plane) load5(uin + view.plane(k + 3) + col, view.vstride, Upf);
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.w[q][ly][lx] = win[2][q];
        }
        if (GHOSTED && (pre || post) ? tid < 2 * (ax + ay) : halo) {
            T Wh[5], invh;
            prim_from_cons(Hpf, Wh, invh, ph, hits);
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.w[q][hj + 3][hi + 3] = Wh[q];
        }
        if (k + 1 < z1 || !GHOSTED ? (halo && k + 1 <= z1) : (k + 1 == z1 && tid < 2 * (ax + ay)))
            load5(uin + view.plane(k + 1) + hcol, view.vstride, Hpf);
        __syncthreads();

        // ---- B: parabola edges, predictor, face states
        if (active && CT) {
            // characteristic tracing: per axis both traced face states
            const T *W = win[2];
            T aL[3][5], aR[3][5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                ppm_edges<MODE>(sm.w[q][ly][lx - 2], sm.w[q][ly][lx - 1], W[q], sm.w[q][ly][lx + 1],
                                sm.w[q][ly][lx + 2], aL[0][q], aR[0][q]);
                ppm_edges<MODE>(sm.w[q][ly - 2][lx], sm.w[q][ly - 1][lx], W[q], sm.w[q][ly + 1][lx],
                                sm.w[q][ly + 2][lx], aL[1][q], aR[1][q]);
                ppm_edges<MODE>(win[0][q], win[1][q], W[q], win[3][q], win[4][q], aL[2][q], aR[2][q]);
            }
            const T gp = ph.gamma * W[4];
            const T r = fast_rsqrt(gp * W[0]);
            const T c = gp * r, inv_c = W[0] * r;      // sqrt(gamma p / rho) and its inverse
            T lo[5], hi[5];
            if (interior) {
                // The prologue and epilogue planes run this same code (their
                // x and y states are discarded, with their floor counts): the
                // compiler may contract a * b + c differently in separate
                // inlined copies of the tracing, and one copy for every plane
                // keeps results independent of where z-ranges start.
                const bool inner = !pre && !post;
                int xyhits = 0;
                ppm_traced_faces<0, 1, 2>(W, winv[2], aL, aR, c, inv_c, lam, ph, lo, hi, xyhits);
                if (inner) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        sm.fl[q][Geo::xface(ci + 1, cj)] = hi[q];
                        sm.fr[q][Geo::xface(ci, cj)] = lo[q];
                    }
                }
                ppm_traced_faces<1, 0, 2>(W, winv[2], aL, aR, c, inv_c, lam, ph, lo, hi, xyhits);
                if (inner) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        sm.fl[yslot(q)][Geo::yface(ci, cj + 1)] = hi[q];
                        sm.fr[yslot(q)][Geo::yface(ci, cj)] = lo[q];
                    }
                    hits += xyhits;
                }
                ppm_traced_faces<2, 0, 1>(W, winv[2], aL, aR, c, inv_c, lam, ph, zm, zpn, hits);
                if (pre) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) zprev[q] = zpn[q];
                }
            } else {
                // a ring column: the traced states of its axis, the one on the
                // tile side stored (left and bottom columns: the upper state)
                const bool ring_x = role == ROLE_LEFT || role == ROLE_RIGHT;
                const bool ring_lo = role == ROLE_LEFT || role == ROLE_BOTTOM;
                const int ring_face =
                    ring_x ? Geo::xface(ci + ring_lo, cj) : Geo::yface(ci, cj + ring_lo);
                if (ring_x) ppm_traced_faces<0, 1, 2>(W, winv[2], aL, aR, c, inv_c, lam, ph, lo, hi, hits);
                else ppm_traced_faces<1, 0, 2>(W, winv[2], aL, aR, c, inv_c, lam, ph, lo, hi, hits);
                T *dst = ring_lo ? &sm.fl[0][ring_face] : &sm.fr[0][ring_face];
#pragma unroll
                for (int q = 0; q < 5; ++q) dst[(ring_x ? q : yslot(q)) * NF] = ring_lo ? hi[q] : lo[q];
            }
        } else if (active) {
            const T *W = win[2];
            T aL[3][5], aR[3][5], S[3][5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                ppm_edges<MODE>(sm.w[q][ly][lx - 2], sm.w[q][ly][lx - 1], W[q], sm.w[q][ly][lx + 1],
                                sm.w[q][ly][lx + 2], aL[0][q], aR[0][q]);
                ppm_edges<MODE>(sm.w[q][ly - 2][lx], sm.w[q][ly - 1][lx], W[q], sm.w[q][ly + 1][lx],
                                sm.w[q][ly + 2][lx], aL[1][q], aR[1][q]);
                ppm_edges<MODE>(win[0][q], win[1][q], W[q], win[3][q], win[4][q], aL[2][q], aR[2][q]);
#pragma unroll
                for (int d = 0; d < 3; ++d) S[d][q] = aR[d][q] - aL[d][q];
            }
            T Ws[5];
            predictor(W, winv[2], S[0], S[1], S[2], lam, ph.gamma, Ws);
            // the face state of axis d on the lower (a_L) or upper (a_R) side
            auto state = [&](const T a[5], T st[5]) {
#pragma unroll
                for (int q = 0; q < 5; ++q) st[q] = Ws[q] + (a[q] - W[q]);
                st[0] = floored(st[0], ph.rho_floor, hits);
                st[4] = floored(st[4], ph.p_floor, hits);
            };
            if (pre) {
                state(aR[2], zprev);
            } else if (post) {
                state(aL[2], zm);
            } else if (interior) {
                T st[5];
                state(aR[0], st);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fl[q][Geo::xface(ci + 1, cj)] = st[q];
                state(aL[0], st);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fr[q][Geo::xface(ci, cj)] = st[q];
                state(aR[1], st);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fl[yslot(q)][Geo::yface(ci, cj + 1)] = st[q];
                state(aL[1], st);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fr[yslot(q)][Geo::yface(ci, cj)] = st[q];
                state(aL[2], zm);
                state(aR[2], zpn);
            } else {
                // a ring column: the state on the tile side of its face with
                // the tile; left and bottom columns hold the face's left state
                const bool ring_x = role == ROLE_LEFT || role == ROLE_RIGHT;
                const bool ring_lo = role == ROLE_LEFT || role == ROLE_BOTTOM;
                const int ring_face =
                    ring_x ? Geo::xface(ci + ring_lo, cj) : Geo::yface(ci, cj + ring_lo);
                T a[5], st[5];
#pragma unroll
                for (int q = 0; q < 5; ++q)
                    a[q] = ring_x ? (ring_lo ? aR[0][q] : aL[0][q]) : (ring_lo ? aR[1][q] : aL[1][q]);
                state(a, st);
                T *dst = ring_lo ? &sm.fl[0][ring_face] : &sm.fr[0][ring_face];
#pragma unroll
                for (int q = 0; q < 5; ++q) dst[(ring_x ? q : yslot(q)) * NF] = st[q];
            }
        }
        if (!post) __syncthreads();
        // the window moves up one plane
        if (owner) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                winv[p] = winv[p + 1];
#pragma unroll
                for (int q = 0; q < 5; ++q) win[p][q] = win[p + 1][q];
            }
        }
        if (pre) continue;

        // ---- C1: the x and y faces of the plane (as in the PLM tile)
        if (!post) {
#pragma unroll 1
            for (int s = 0; s < NSLOT; ++s) {
                if (!((fact >> s) & 1u)) continue;
                const int t = tid + s * Geo::NT;
                T L[5], R[5], G[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    L[q] = sm.fl[q][t];
                    R[q] = sm.fr[q][t];
                }
                riemann<RS>(L, R, ph, G);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fl[q][t] = G[q];
                if (want_flux) {
                    int i, j;
                    const bool isx = Geo::face_ij(t, i, j);
                    const int fi = x0 + i, fj = y0 + j;
                    if (isx && (fi == 0 || fi == P.nx)) {
                        T *sheet = bf + (fi == 0 ? 0 : 5 * sxs);
#pragma unroll
                        for (int q = 0; q < 5; ++q) sheet[q * sxs + (int64_t)k * P.ny + fj] = G[q];
                    }
                    if (!isx && (fj == 0 || fj == P.ny)) {
                        T *sheet = bf + 10 * sxs + (fj == 0 ? 0 : 5 * sys);
#pragma unroll
                        for (int q = 0; q < 5; ++q)
                            sheet[q * sys + (int64_t)k * P.nx + fi] = G[yslot(q)];
                    }
                }
            }
        }

        // ---- C2: the z face below the plane; completes plane k-1
        if (interior) {
            T F[5];
            face_flux<RS, 2>(zprev, zm, ph, F);
            if (want_flux && (k == 0 || k == P.nz)) {
                T *sheet = bf + 10 * sxs + 10 * sys + (k == 0 ? 0 : 5 * szs);
#pragma unroll
                for (int q = 0; q < 5; ++q) sheet[q * szs + (int64_t)gj * P.nx + gi] = F[q];
            }
            if (k > z0) {
                load5(uin + view.plane(k - 1) + col, view.vstride, Uold);
                T *o = out + (int64_t)(k - 1) * P.nx * P.ny + ocol;
                T Un[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    Un[q] = Uold[q] - dtdx * (acc[q] + F[q]);
                    o[q * ostride] = Un[q];
                }
                if (want_cfl) {
                    int unused = 0;
                    smax = fmax(smax, cell_signal(Un, ph, unused) * inv_dx);
                }
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                acc[q] = -F[q];
                zprev[q] = zpn[q];
            }
        }
        if (post) break;
        __syncthreads();

        // ---- D: x-y flux divergence of the plane
        if (interior) {
#pragma unroll
            for (int q = 0; q < 5; ++q)
                acc[q] = ((sm.fl[q][Geo::xface(ci + 1, cj)] - sm.fl[q][Geo::xface(ci, cj)]) +
                          (sm.fl[yslot(q)][Geo::yface(ci, cj + 1)] -
                           sm.fl[yslot(q)][Geo::yface(ci, cj)])) + acc[q];
        }
    }
}

// One patch, one launch: tiles in z-segment-major order, remapped per XCD as
// in the PLM step kernel.
template <typename T, int MODE, bool CT, int RS, int TX, int TY, bool GHOSTED>
__global__ __launch_bounds__(tile_threads(TX, TY)) __attribute__((amdgpu_waves_per_eu(2)))
void ppm_tile_kernel(PatchDesc P, const T *__restrict__ u_in, T *__restrict__ u_out,
                     T *__restrict__ bflux, const double *dt_dev, Scalars sc,
                     unsigned long long *hits_ctr, int ntx, int nty, int zlen, CflOut co)
{
    __shared__ PpmTileSmem<T, TX, TY> sm;
    const Phys<T> ph = make_phys<T>(sc);
    const double dt = dt_dev ? *dt_dev : P.dt;
    const T dtdx = T(dt / P.dx), lam = T(dt / (2.0 * P.dx));
    const int nblocks = gridDim.x, b = blockIdx.x;
    const int per_xcd = nblocks / 8;
    const int item = b < 8 * per_xcd ? (b % 8) * per_xcd + b / 8 : b;
    const int ntiles = ntx * nty;
    const int seg = item / ntiles, tile = item % ntiles;
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int z0 = seg * zlen, z1 = min(z0 + zlen, P.nz);
    int hits = 0;
    double smax = 0.0;
    const bool want_cfl = co.dt_next != nullptr;
    ppm_tile<T, MODE, CT, RS, TX, TY, GHOSTED>(P, u_in, u_out, bflux, dtdx, lam, ph, x0, y0, z0, z1,
                                               sm, hits, want_cfl, smax);
    flush_hits(hits, hits_ctr);
    if (want_cfl) cfl_block_max(smax, co.smax_bits);
}

template <typename T, int MODE, bool CT, int RS>
int launch_ppm_tile_t(const PatchDesc &P, const void *u_in, void *u_out, void *bflux,
                      const double *dt_dev, const Scalars &sc, unsigned long long *hits,
                      int min_blocks, const CflOut &co, hipStream_t s)
{
    constexpr int TX = PPM_FUSED_TX, TY = PPM_FUSED_TY;
    // periodic coordinates are wrapped twice, which covers the stencils'
    // reach of three cells only for extents of 2 and more
    if (P.periodic && (P.nx < 2 || P.ny < 2 || P.nz < 2)) return (int)hipErrorInvalidValue;
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    const int64_t ntiles = (int64_t)ntx * nty;
    // z-ranges of 32 planes, shorter (down to one) when that leaves the chip
    // without enough workgroups, as for the PLM step
    int zlen = std::min(32, P.nz);
    if (ntiles * ((P.nz + zlen - 1) / zlen) < min_blocks) {
        const int64_t want = (min_blocks + ntiles - 1) / ntiles;
        zlen = (int)std::min<int64_t>(zlen, std::max<int64_t>(1, (P.nz + want - 1) / want));
    }
    const int64_t nblocks = ntiles * ((P.nz + zlen - 1) / zlen);
    if (nblocks <= 0 || nblocks > 0x7fffffff) return (int)hipErrorInvalidValue;
    if (P.periodic)
        hipLaunchKernelGGL((ppm_tile_kernel<T, MODE, CT, RS, TX, TY, false>), dim3((unsigned)nblocks),
                           dim3(TileGeom<TX, TY>::NT), 0, s, P, (const T *)u_in, (T *)u_out,
                           (T *)bflux, dt_dev, sc, hits, ntx, nty, zlen, co);
    else
        hipLaunchKernelGGL((ppm_tile_kernel<T, MODE, CT, RS, TX, TY, true>), dim3((unsigned)nblocks),
                           dim3(TileGeom<TX, TY>::NT), 0, s, P, (const T *)u_in, (T *)u_out,
                           (T *)bflux, dt_dev, sc, hits, ntx, nty, zlen, co);
    return (int)hipGetLastError();
}

// A batch of ghosted patches, one launch: the persistent work queue of the
// PLM batched step over (patch, tile, z-range) items, each item the march of
// the single-patch kernel. The last workgroup to leave resets the counter.
template <typename T, int MODE, bool CT, int RS, int TX, int TY>
__global__ __launch_bounds__(tile_threads(TX, TY)) __attribute__((amdgpu_waves_per_eu(2)))
void ppm_batched_kernel(const PatchDesc *__restrict__ patches, const WorkItem *__restrict__ items,
                        int nitems, const T *__restrict__ u_in, T *__restrict__ u_out,
                        T *__restrict__ bflux, const double *dt_dev, Scalars sc,
                        unsigned long long *hits_ctr, unsigned *queue, CflOut co)
{
    __shared__ PpmTileSmem<T, TX, TY> sm;
    __shared__ int s_item;
    const Phys<T> ph = make_phys<T>(sc);
    int hits = 0;
    double smax = 0.0;
    const bool want_cfl = co.dt_next != nullptr;
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
        ppm_tile<T, MODE, CT, RS, TX, TY, true>(P, u_in, u_out, bflux, dtdx, lam, ph, w.x0, w.y0,
                                                w.z0, w.z1, sm, hits, want_cfl, smax);
        __syncthreads();
    }
    flush_hits(hits, hits_ctr);
    if (want_cfl) cfl_block_max(smax, co.smax_bits);
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&queue[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
        }
    }
}

template <typename T, int MODE, bool CT, int RS>
int launch_ppm_batched_t(const PatchDesc *d_patches, const WorkItem *d_items, int nitems,
                         const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                         const Scalars &sc, unsigned long long *hits, unsigned *d_queue,
                         int num_cus, const CflOut &co, hipStream_t s)
{
    constexpr int TX = PPM_FUSED_TX, TY = PPM_FUSED_TY;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ppm_batched_kernel<T, MODE, CT, RS, TX, TY>,
                                                     TileGeom<TX, TY>::NT, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int grid = std::max(1, std::min(nitems, per_cu * num_cus));
    hipLaunchKernelGGL((ppm_batched_kernel<T, MODE, CT, RS, TX, TY>), dim3(grid),
                       dim3(TileGeom<TX, TY>::NT), 0, s, d_patches, d_items, nitems,
                       (const T *)u_in, (T *)u_out, (T *)bflux, dt_dev, sc, hits, d_queue, co);
    return (int)hipGetLastError();
}

template <typename T, int MODE, bool CT, int RS>
int launch_ppm_t(const PatchDesc &P, const void *u_in, void *u_out, void *bflux, void *scratch,
                 const double *dt_dev, const Scalars &sc, unsigned long long *hits, hipStream_t s)
{
    const int e = P.periodic ? 0 : 1;
    const int64_t ncell = (int64_t)P.nx * P.ny * P.nz;
    const int64_t ntiles = (int64_t)((P.nx + 2 * e + PT - 1) / PT) * ((P.ny + 2 * e + PT - 1) / PT) *
                           ((P.nz + 2 * e + PZ - 1) / PZ);
    hipLaunchKernelGGL((ppm_predict_kernel<T, MODE, CT>), dim3((unsigned)ntiles), dim3(PT * PT), 0, s,
                       P, (const T *)u_in, (T *)scratch, dt_dev, sc, hits);
    hipLaunchKernelGGL((ppm_update_kernel<T, RS>), dim3((unsigned)((ncell + PPM_BLOCK - 1) / PPM_BLOCK)),
                       dim3(PPM_BLOCK), 0, s, P, (const T *)u_in, (const T *)scratch, (T *)u_out,
                       (T *)bflux, dt_dev, sc);
    return (int)hipGetLastError();
}

template <typename T>
int launch_ppm_d(int limiter, int riemann, const PatchDesc &P, const void *u_in, void *u_out,
                 void *bflux, void *scratch, const double *dt_dev, const Scalars &sc,
                 unsigned long long *hits, hipStream_t s)
{
#define GD_PPM(M, C, R) return launch_ppm_t<T, M, C, R>(P, u_in, u_out, bflux, scratch, dt_dev, sc, hits, s)
    // limiters 3, 4: Hancock half step with the limited / unlimited parabola;
    // 5, 6: characteristic tracing with the limited / unlimited parabola
    const bool central = limiter == 4 || limiter == 6;
    const bool traced = limiter == 5 || limiter == 6;
    if (riemann == RS_HLL) {
        if (traced) {
            if (central) GD_PPM(PPM_CENTRAL, true, RS_HLL);
            GD_PPM(PPM_LIMITED, true, RS_HLL);
        }
        if (central) GD_PPM(PPM_CENTRAL, false, RS_HLL);
        GD_PPM(PPM_LIMITED, false, RS_HLL);
    }
    if (traced) {
        if (central) GD_PPM(PPM_CENTRAL, true, RS_HLLC);
        GD_PPM(PPM_LIMITED, true, RS_HLLC);
    }
    if (central) GD_PPM(PPM_CENTRAL, false, RS_HLLC);
    GD_PPM(PPM_LIMITED, false, RS_HLLC);
#undef GD_PPM
}

}  // namespace

int launch_ppm_tile(int dtype, int limiter, int riemann, const PatchDesc &P, const void *u_in,
                    void *u_out, void *bflux, const double *dt_dev, const Scalars &sc,
                    unsigned long long *hits, int min_blocks, const CflOut &co, hipStream_t s)
{
#define GD_PPMT(T, M, C, R) return launch_ppm_tile_t<T, M, C, R>(P, u_in, u_out, bflux, dt_dev, sc, \
                                                                 hits, min_blocks, co, s)
#define GD_PPMT_LIM(T, C, R)                                                    \
    do {                                                                        \
        if (central) GD_PPMT(T, PPM_CENTRAL, C, R);                             \
        GD_PPMT(T, PPM_LIMITED, C, R);                                          \
    } while (0)
#define GD_PPMT_CT(T, R)                                                        \
    do {                                                                        \
        if (traced) GD_PPMT_LIM(T, true, R);                                    \
        GD_PPMT_LIM(T, false, R);                                               \
    } while (0)
    const bool central = limiter == 4 || limiter == 6;
    const bool traced = limiter == 5 || limiter == 6;
    if (dtype == 1) {
        if (riemann == RS_HLL) GD_PPMT_CT(float, RS_HLL);
        GD_PPMT_CT(float, RS_HLLC);
    }
    if (riemann == RS_HLL) GD_PPMT_CT(double, RS_HLL);
    GD_PPMT_CT(double, RS_HLLC);
#undef GD_PPMT_CT
#undef GD_PPMT_LIM
#undef GD_PPMT
}

int launch_ppm_batched(int dtype, int limiter, int riemann, const PatchDesc *d_patches,
                       const WorkItem *d_items, int nitems, const void *u_in, void *u_out,
                       void *bflux, const double *dt_dev, const Scalars &sc,
                       unsigned long long *hits, unsigned *d_queue, int num_cus, const CflOut &co,
                       hipStream_t s)
{
    if (nitems <= 0) return 0;
#define GD_PPMB(T, M, C, R) return launch_ppm_batched_t<T, M, C, R>(d_patches, d_items, nitems, u_in, \
                                                                    u_out, bflux, dt_dev, sc, hits,   \
                                                                    d_queue, num_cus, co, s)
#define GD_PPMB_LIM(T, C, R)                                                    \
    do {                                                                        \
        if (central) GD_PPMB(T, PPM_CENTRAL, C, R);                             \
        GD_PPMB(T, PPM_LIMITED, C, R);                                          \
    } while (0)
#define GD_PPMB_CT(T, R)                                                        \
    do {                                                                        \
        if (traced) GD_PPMB_LIM(T, true, R);                                    \
        GD_PPMB_LIM(T, false, R);                                               \
    } while (0)
    const bool central = limiter == 4 || limiter == 6;
    const bool traced = limiter == 5 || limiter == 6;
    if (dtype == 1) {
        if (riemann == RS_HLL) GD_PPMB_CT(float, RS_HLL);
        GD_PPMB_CT(float, RS_HLLC);
    }
    if (riemann == RS_HLL) GD_PPMB_CT(double, RS_HLL);
    GD_PPMB_CT(double, RS_HLLC);
#undef GD_PPMB_CT
#undef GD_PPMB_LIM
#undef GD_PPMB
}

int64_t ppm_box_cells(const PatchDesc &P)
{
    const int e = P.periodic ? 0 : 1;
    return (int64_t)(P.nx + 2 * e) * (P.ny + 2 * e) * (P.nz + 2 * e);
}

int launch_ppm(int dtype, int limiter, int riemann, const PatchDesc &P, const void *u_in,
               void *u_out, void *bflux, void *scratch, const double *dt_dev, const Scalars &sc,
               unsigned long long *hits, hipStream_t s)
{
    if (dtype == 1)
        return launch_ppm_d<float>(limiter, riemann, P, u_in, u_out, bflux, scratch, dt_dev, sc, hits, s);
    return launch_ppm_d<double>(limiter, riemann, P, u_in, u_out, bflux, scratch, dt_dev, sc, hits, s);
}

}  // namespace gd
