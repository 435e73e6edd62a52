// The tile march of the Euler step on gfx950: the device routine that one
// workgroup runs over a TX x TY column tile of a patch and a z-range of its
// planes, with the addressing and CFL-reduction helpers it uses. Included by
// every translation unit that instantiates a step kernel.
#pragma once

#include "godunov_cell.h"
#include "godunov_internal.h"
#include "godunov_math.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

// Threads of a tile: TX*TY interior columns, then the 2(TX+TY) ring
// columns, rounded up to whole waves (24x8: 192 + 64 = 256 threads, 4 waves).
constexpr int tile_threads(int tx, int ty) { return ((tx * ty + 2 * (tx + ty) + 63) / 64) * 64; }

// NT, the workgroup size, may exceed tile_threads(TX, TY) (a kernel that runs
// tiles of several shapes in one workgroup size); the surplus threads own no
// column and only share the staging and face work.
template <int TX, int TY, int NT_ = tile_threads(TX, TY)>
struct TileGeom {
    static_assert(NT_ >= tile_threads(TX, TY), "workgroup too small for the tile");
    static constexpr int NINT = TX * TY;
    static constexpr int NT = NT_;
    // faces of a plane: the x faces i-1/2 (i = 0..TX) of each row, then the y
    // faces j-1/2 (j = 0..TY) of each column
    static constexpr int NXF = TY * (TX + 1);
    static constexpr int NF = NXF + (TY + 1) * TX;
    static constexpr int NSLOT = (NF + NT - 1) / NT;    // faces per thread
    __device__ static constexpr int xface(int i, int j) { return j * (TX + 1) + i; }
    __device__ static constexpr int yface(int i, int j) { return NXF + j * TX + i; }
    // (i, j) of face t; true for an x face
    __device__ static bool face_ij(int t, int &i, int &j)
    {
        const bool isx = t < NXF;
        const int u = isx ? t : t - NXF;
        i = isx ? u % (TX + 1) : u % TX;
        j = isx ? u / (TX + 1) : u / TX;
        return isx;
    }
};

// Storage slot of primitive component q in a y-face state: y faces are kept in
// their rotated order (rho, v, w, u, p), x faces in the natural one, so a face
// reads and writes slots 0..4 whatever its orientation.
__device__ constexpr int yslot(int q) { return q == 1 ? 3 : (q == 2 ? 1 : (q == 3 ? 2 : q)); }

// ------------------------------------------------------------ addressing

__device__ __forceinline__ int wrap_once(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct InputView {
    int64_t vstride;          // elements between variables
    int32_t sy, sz;           // row and plane strides
    int32_t nx, ny, nz, ng, periodic;

    // offset of column (i, j) within a plane
    __device__ __forceinline__ int64_t column(int i, int j) const
    {
        if (periodic) {
            i = wrap_once(wrap_once(i, nx), nx);
            j = wrap_once(wrap_once(j, ny), ny);
            return (int64_t)j * sy + i;
        }
        return (int64_t)(j + ng) * sy + (i + ng);
    }
    __device__ __forceinline__ int64_t plane(int k) const
    {
        if (periodic) return (int64_t)wrap_once(wrap_once(k, nz), nz) * sz;
        return (int64_t)(k + ng) * sz;
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
__device__ __forceinline__ void load5(const T *__restrict__ p, int64_t vstride, T U[5])
{
#pragma unroll
    for (int q = 0; q < 5; ++q) U[q] = p[q * vstride];
}

// ------------------------------------------------------------ CFL reduction

// |u| + |v| + |w| + 3c of a conserved state, c = sqrt(g p / rho) evaluated as
// g p / sqrt(g p rho). The CFL kernels and the fused CFL of the step kernels
// share this function, so both give the same dt bit for bit.
template <typename T>
__device__ __forceinline__ double cell_signal(const T U[5], const Phys<T> &ph, int &hits)
{
    T W[5], inv;
    prim_from_cons(U, W, inv, ph, hits);
    T gp = ph.gamma * W[4];
    T c = gp * fast_rsqrt(gp * W[0]);
    return (double)(fabs(W[1]) + fabs(W[2]) + fabs(W[3]) + T(3) * c);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide max of v (>= 0) folded into *smax_bits, the bit pattern of a
// non-negative double (which orders like the value). Thread 0 reads the
// running value first and issues the device-wide atomic only when the
// block's maximum exceeds it, so a grid of thousands of workgroups performs
// few same-address atomics. A one-thread launch (cfl_finalize_kernel) then
// turns the maximum into dt and clears it for the next use.
__device__ void cfl_block_max(double v, unsigned long long *smax_bits)
{
    __shared__ double part[16];
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) m = fmax(m, part[i]);
        const unsigned long long b = (unsigned long long)__double_as_longlong(m);
        if (b > __atomic_load_n(smax_bits, __ATOMIC_RELAXED)) atomicMax(smax_bits, b);
    }
}


// ------------------------------------------------------------ the tile march

template <typename T, int TX, int TY>
struct TileSmem {
    // primitives of plane k with its two-deep x-y halo (the column's own
    // planes k-1 and k+1 live in registers)
    T w[5][TY + 4][TX + 4];
    // face states of the plane, indexed as TileGeom::xface / yface, left
    // (lower) state in fl and right (upper) state in fr, y faces in rotated
    // slots (yslot). The flux through a face overwrites its left state (the
    // thread that evaluates a face is the only one touching it).
    T fl[5][TileGeom<TX, TY>::NF];
    T fr[5][TileGeom<TX, TY>::NF];
};

enum { ROLE_NONE = -1, ROLE_INT = 0, ROLE_BOTTOM = 1, ROLE_TOP = 2, ROLE_LEFT = 3, ROLE_RIGHT = 4 };

// One tile: interior columns [x0, x0+TX) x [y0, y0+TY) (clipped to the
// patch), planes [z0, z1). Per plane k (after a prologue plane z0-1 that only
// produces the z+ face states, and before an epilogue plane z1 that only
// produces the z- face states):
//   A  each column owner reads plane k+1 of its column, stages plane k in
//      LDS; halo threads stage the depth-2 halo and the corner cells;
//   B  owners: slopes, predictor, face states (x and y into LDS; the z
//      states of interior columns stay in registers);
//   C  all threads: the x and y faces of the plane as uniform tasks, each
//      face once; then interior columns: the z face below the plane, which
//      completes plane k-1;
//   D  interior: x-y flux divergence accumulated for plane k.
// STREAM_OUT: write the new state with streaming (non-temporal) stores. The
// batched launches do: there the outputs of many small patches would
// otherwise evict from the L2 the inputs that neighbouring tiles still read
// (7% fewer bytes fetched on the 4096-patch batch, 1.5% faster). A single
// patch keeps ordinary stores: streaming ones raised its write traffic by 8%
// (rows that two tiles share are no longer merged in the L2) at no gain.
template <typename T, int LIM, int RS, int TX, int TY, int NT = tile_threads(TX, TY),
          bool STREAM_OUT = false>
__device__ void godunov_tile(const PatchDesc &P, const T *__restrict__ u_in_base,
                             T *__restrict__ u_out_base, T *__restrict__ bflux_base, T dtdx, T lam,
                             const Phys<T> &ph, int x0, int y0, int z0, int z1,
                             TileSmem<T, TX, TY> &sm, int &hits, bool want_cfl, double &smax)
{
    using Geo = TileGeom<TX, TY, NT>;
    constexpr int NF = Geo::NF;
    const int tid = threadIdx.x;
    const int ax = min(TX, P.nx - x0);
    const int ay = min(TY, P.ny - y0);
    const InputView view = make_view(P);
    const T *__restrict__ uin = u_in_base + P.in_off;

    // ---- role of this thread: an interior column, a ring column, or none
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
    const int64_t col = view.column(gi, gj);

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
    const int64_t hcol = view.column(x0 + hi, y0 + hj);

    // boundary-flux sheets of this patch
    const bool want_flux = bflux_base != nullptr && P.flux_off >= 0;
    T *__restrict__ bf = want_flux ? bflux_base + P.flux_off : nullptr;
    const int64_t sxs = (int64_t)P.nz * P.ny, sys = (int64_t)P.nz * P.nx, szs = (int64_t)P.ny * P.nx;

    T *__restrict__ out = u_out_base + P.out_off;
    const int64_t ostride = (int64_t)P.nx * P.ny * P.nz;
    const double inv_dx = 1.0 / P.dx;
    const int64_t ocol = (int64_t)gj * P.nx + gi;

    // ---- registers of the owned column
    T Wm[5], W0[5], Wp[5], inv0 = T(1), invp = T(1);
    T zprev[5], acc[5], zm[5], zpn[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        Wm[q] = W0[q] = Wp[q] = T(0);
        zprev[q] = acc[q] = zm[q] = zpn[q] = T(0);
    }

    // Column loads run one plane ahead of their use: the raw conserved state
    // of plane k+1 (Upf) and of the halo of plane k (Hpf) are in flight while
    // plane k-1 is computed. The last plane a column reads is z1+1 for an
    // interior column and z1 for a ring column.
    const int last_plane = interior ? z1 + 1 : z1;
    T Upf[5], Hpf[5], Uold[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) Upf[q] = Hpf[q] = Uold[q] = T(0);

    // prologue: plane z0-2 (interior only, into W0, which the first step
    // moves to Wm), plane z0-1 (into Wp) and the loads of plane z0
    if (owner) {
        T U[5], inv;
        if (interior) {
            load5(uin + view.plane(z0 - 2) + col, view.vstride, U);
            prim_from_cons(U, W0, inv, ph, hits);
        }
        load5(uin + view.plane(z0 - 1) + col, view.vstride, U);
        prim_from_cons(U, Wp, invp, ph, hits);
        load5(uin + view.plane(z0) + col, view.vstride, Upf);
    }
    if (halo) load5(uin + view.plane(z0) + hcol, view.vstride, Hpf);

    // the faces this thread evaluates in phase C1, and whether each lies in
    // the clipped tile
    unsigned fact = 0;
#pragma unroll
    for (int s = 0; s < Geo::NSLOT; ++s) {
        const int t = tid + s * Geo::NT;
        int i, j;
        const bool isx = Geo::face_ij(t, i, j);
        if (t < NF && (isx ? (i <= ax && j < ay) : (i < ax && j <= ay))) fact |= 1u << s;
    }

    const int lx = ci + 2, ly = cj + 2;
    const T half = T(0.5);
    for (int k = z0 - 1; k <= z1; ++k) {
        const bool pre = k < z0;
        const bool post = k == z1;

        // ---- A: advance the column, stage plane k. Every thread has
        // finished reading plane k-1 from LDS (phase B, then a barrier)
        // before it is overwritten here.
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Wm[q] = W0[q];
            W0[q] = Wp[q];
        }
        inv0 = invp;
        if (owner && k + 1 <= last_plane) {
            prim_from_cons(Upf, Wp, invp, ph, hits);
            if (k + 2 <= last_plane) load5(uin + view.plane(k + 2) + col, view.vstride, Upf);
        }
        if (owner) {
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.w[q][ly][lx] = W0[q];
        }
        if (!pre && !post && halo) {
            T Wh[5], invh;
            prim_from_cons(Hpf, Wh, invh, ph, hits);
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.w[q][hj + 2][hi + 2] = Wh[q];
            if (k + 1 < z1) load5(uin + view.plane(k + 1) + hcol, view.vstride, Hpf);
        }
        __syncthreads();

        // ---- B: slopes, predictor, face states
        const bool work = pre || post ? interior : owner;
        if (work) {
            T Sx[5], Sy[5], Sz[5], Ws[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                T c = W0[q];
                Sx[q] = limited_slope<LIM>(c - sm.w[q][ly][lx - 1], sm.w[q][ly][lx + 1] - c);
                Sy[q] = limited_slope<LIM>(c - sm.w[q][ly - 1][lx], sm.w[q][ly + 1][lx] - c);
                Sz[q] = limited_slope<LIM>(c - Wm[q], Wp[q] - c);
            }
            predictor(W0, inv0, Sx, Sy, Sz, lam, ph.gamma, Ws);
            if (pre) {
                face_state(Ws, Sz, half, zprev, ph, hits);
            } else if (post) {
                face_state(Ws, Sz, -half, zm, ph, hits);
            } else if (interior) {
                T st[5];
                face_state(Ws, Sx, half, st, ph, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fl[q][Geo::xface(ci + 1, cj)] = st[q];
                face_state(Ws, Sx, -half, st, ph, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fr[q][Geo::xface(ci, cj)] = st[q];
                face_state(Ws, Sy, half, st, ph, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fl[yslot(q)][Geo::yface(ci, cj + 1)] = st[q];
                face_state(Ws, Sy, -half, st, ph, hits);
#pragma unroll
                for (int q = 0; q < 5; ++q) sm.fr[yslot(q)][Geo::yface(ci, cj)] = st[q];
                face_state(Ws, Sz, -half, zm, ph, hits);
                face_state(Ws, Sz, half, zpn, ph, hits);
            } else {
                // a ring column: the one state its face with the tile needs,
                // direction and side selected per lane, so that a wave holding
                // ring columns of all four sides evaluates a single face state.
                // The face is an x face for the left and right columns, a y
                // face for the bottom and top rows; the left and bottom
                // columns hold the face's left (lower) state.
                const bool ring_x = role == ROLE_LEFT || role == ROLE_RIGHT;
                const bool ring_lo = role == ROLE_LEFT || role == ROLE_BOTTOM;
                const int ring_face =
                    ring_x ? Geo::xface(ci + ring_lo, cj) : Geo::yface(ci, cj + ring_lo);
                T S[5], st[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) S[q] = ring_x ? Sx[q] : Sy[q];
                face_state(Ws, S, ring_lo ? half : -half, st, ph, hits);
                T *dst = ring_lo ? &sm.fl[0][ring_face] : &sm.fr[0][ring_face];
#pragma unroll
                for (int q = 0; q < 5; ++q) dst[(ring_x ? q : yslot(q)) * NF] = st[q];
            }
        }
        if (!post) __syncthreads();
        if (pre) continue;

        // ---- C1: the x and y faces of the plane, NSLOT per thread (face t =
        // tid + s NT). Both orientations read their states from and write their
        // flux to slots 0..4 of face t, so the task needs no per-face address
        // arithmetic; only the boundary-flux sheets need the face's (i, j).
        if (!post) {
            // not unrolled: two faces in flight at once would double the
            // registers the Riemann solver holds
#pragma unroll 1
            for (int s = 0; s < Geo::NSLOT; ++s) {
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
                // loaded here rather than ahead: the registers a prefetch would
                // hold keep the kernel within three waves per SIMD without spills
                load5(uin + view.plane(k - 1) + col, view.vstride, Uold);
                // U' = U - dt/dx (acc + F_z(k-1/2)), acc = div_xy(k-1) - F_z(k-3/2)
                T *o = out + (int64_t)(k - 1) * P.nx * P.ny + ocol;
                T Un[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    Un[q] = Uold[q] - dtdx * (acc[q] + F[q]);
                    if constexpr (STREAM_OUT)
                        __builtin_nontemporal_store(Un[q], &o[q * ostride]);
                    else
                        o[q * ostride] = Un[q];
                }
                if (want_cfl) {
                    // signal speed of the new state, exactly as cfl_dt computes it
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

__device__ __forceinline__ void flush_hits(int hits, unsigned long long *counter)
{
    if (hits) atomicAdd(counter, (unsigned long long)hits);
}

// One patch. Workgroups are dispatched round-robin over the 8 XCDs (each
// with its own L2); the block index is remapped so that each XCD works
// through a contiguous range of items, ordered z-segment-major then tile
// row-major, so that tiles sharing halo columns run on the same L2.
// Occupancy target: three waves per SIMD in FP64 (168 VGPRs), four in FP32.
template <typename T>
constexpr int waves_per_eu() { return sizeof(T) == 8 ? 3 : 4; }

}  // namespace gd
