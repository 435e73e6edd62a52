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
#include "godunov_cell.h"
#include "godunov_internal.h"
#include "godunov_math.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

int tile_tx(int shape)
{
    switch (shape) {
    case TILE_8x8: return 8;
    case TILE_32x8: return 32;
    case TILE_16x8: return 16;
    case TILE_24x8: return 24;
    default: return 16;
    }
}
int tile_ty(int shape)
{
    switch (shape) {
    case TILE_8x8: case TILE_32x8: case TILE_16x8: case TILE_24x8: return 8;
    default: return 16;
    }
}

// Threads of a tile: TX*TY interior columns, then the 2(TX+TY) ring
// columns, rounded up to whole waves (24x8: 192 + 64 = 256 threads, 4 waves).
constexpr int tile_threads(int tx, int ty) { return ((tx * ty + 2 * (tx + ty) + 63) / 64) * 64; }

template <int TX, int TY>
struct TileGeom {
    static constexpr int NINT = TX * TY;
    static constexpr int NT = tile_threads(TX, TY);
};

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

__global__ __launch_bounds__(64) void cfl_finalize_kernel(double cfl, double *dt_out,
                                                          unsigned long long *smax_bits)
{
    if (threadIdx.x == 0) {
        const unsigned long long b = atomicExch(smax_bits, 0ull);
        *dt_out = cfl / __longlong_as_double((long long)b);
    }
}

// ------------------------------------------------------------ the tile march

template <typename T, int TX, int TY>
struct TileSmem {
    // primitives of plane k with its two-deep x-y halo (the column's own
    // planes k-1 and k+1 live in registers)
    T w[5][TY + 4][TX + 4];
    // face states of the plane: x face i-1/2 of row j has its left state in
    // xl[.][j][i] and its right state in xr[.][j][i]; likewise y face j-1/2 of
    // column i in yl/yr[.][j][i]. The flux through a face overwrites its left
    // state (the thread that evaluates a face is the only one touching it).
    T xl[5][TY][TX + 1];
    T xr[5][TY][TX + 1];
    T yl[5][TY + 1][TX];
    T yr[5][TY + 1][TX];
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
template <typename T, int LIM, int RS, int TX, int TY>
__device__ void godunov_tile(const PatchDesc &P, const T *__restrict__ u_in_base,
                             T *__restrict__ u_out_base, T *__restrict__ bflux_base, T dtdx, T lam,
                             const Phys<T> &ph, int x0, int y0, int z0, int z1,
                             TileSmem<T, TX, TY> &sm, int &hits, bool want_cfl, double &smax)
{
    using Geo = TileGeom<TX, TY>;
    constexpr int NXF = TY * (TX + 1), NYF = (TY + 1) * TX;
    constexpr int XVS = TY * (TX + 1), YVS = (TY + 1) * TX;    // LDS variable strides
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
            } else {
                T st[5];
                if (interior || role == ROLE_LEFT) {
                    face_state(Ws, Sx, half, st, ph, hits);
#pragma unroll
                    for (int q = 0; q < 5; ++q) sm.xl[q][cj][ci + 1] = st[q];
                }
                if (interior || role == ROLE_RIGHT) {
                    face_state(Ws, Sx, -half, st, ph, hits);
#pragma unroll
                    for (int q = 0; q < 5; ++q) sm.xr[q][cj][ci] = st[q];
                }
                if (interior || role == ROLE_BOTTOM) {
                    face_state(Ws, Sy, half, st, ph, hits);
#pragma unroll
                    for (int q = 0; q < 5; ++q) sm.yl[q][cj + 1][ci] = st[q];
                }
                if (interior || role == ROLE_TOP) {
                    face_state(Ws, Sy, -half, st, ph, hits);
#pragma unroll
                    for (int q = 0; q < 5; ++q) sm.yr[q][cj][ci] = st[q];
                }
                if (interior) {
                    face_state(Ws, Sz, -half, zm, ph, hits);
                    face_state(Ws, Sz, half, zpn, ph, hits);
                }
            }
        }
        if (!post) __syncthreads();
        if (pre) continue;

        // ---- C1: x and y faces as tasks over all threads. Task t < NXF is
        // x face (i, j) = (t % (TX+1), t / (TX+1)); the rest are y faces
        // (i, j) = (u % TX, u / TX) with u = t - NXF. States are read and
        // fluxes written through per-lane LDS addresses in rotated order
        // (normal velocity first), so one code path serves both directions.
        if (!post) {
            for (int t = tid; t < NXF + NYF; t += Geo::NT) {
                const bool isx = t < NXF;
                const int u = isx ? t : t - NXF;
                const int i = isx ? u % (TX + 1) : u % TX;
                const int j = isx ? u / (TX + 1) : u / TX;
                const bool active = isx ? (i <= ax && j < ay) : (i < ax && j <= ay);
                if (!active) continue;
                T *lb = isx ? &sm.xl[0][j][i] : &sm.yl[0][j][i];
                const T *rb = isx ? &sm.xr[0][j][i] : &sm.yr[0][j][i];
                const int vs = isx ? XVS : YVS;
                // rotated component offsets: x (u, v, w), y (v, w, u)
                const int on = (isx ? 1 : 2) * vs, o1 = (isx ? 2 : 3) * vs, o2 = (isx ? 3 : 1) * vs;
                T L[5] = { lb[0], lb[on], lb[o1], lb[o2], lb[4 * vs] };
                T R[5] = { rb[0], rb[on], rb[o1], rb[o2], rb[4 * vs] };
                T G[5];
                riemann<RS>(L, R, ph, G);
                lb[0] = G[0]; lb[on] = G[1]; lb[o1] = G[2]; lb[o2] = G[3]; lb[4 * vs] = G[4];
                if (want_flux) {
                    const int fi = x0 + i, fj = y0 + j;
                    T F[5];
                    F[0] = G[0]; F[4] = G[4];
                    F[1] = isx ? G[1] : G[3];
                    F[2] = isx ? G[2] : G[1];
                    F[3] = isx ? G[3] : G[2];
                    if (isx && (fi == 0 || fi == P.nx)) {
                        T *sheet = bf + (fi == 0 ? 0 : 5 * sxs);
#pragma unroll
                        for (int q = 0; q < 5; ++q) sheet[q * sxs + (int64_t)k * P.ny + fj] = F[q];
                    }
                    if (!isx && (fj == 0 || fj == P.ny)) {
                        T *sheet = bf + 10 * sxs + (fj == 0 ? 0 : 5 * sys);
#pragma unroll
                        for (int q = 0; q < 5; ++q) sheet[q * sys + (int64_t)k * P.nx + fi] = F[q];
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
                acc[q] = ((sm.xl[q][cj][ci + 1] - sm.xl[q][cj][ci]) +
                          (sm.yl[q][cj + 1][ci] - sm.yl[q][cj][ci])) + acc[q];
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

template <typename T, int LIM, int RS, int TX, int TY>
__global__ __launch_bounds__(tile_threads(TX, TY))
__attribute__((amdgpu_waves_per_eu(waves_per_eu<T>()))) void step_kernel(
    PatchDesc P, const T *__restrict__ u_in, T *__restrict__ u_out, T *__restrict__ bflux,
    const double *dt_dev, Scalars sc, unsigned long long *hits_ctr, int ntx, int nty, int zlen,
    CflOut co)
{
    __shared__ TileSmem<T, TX, TY> sm;
    const Phys<T> ph = make_phys<T>(sc);
    const double dt = dt_dev ? *dt_dev : P.dt;
    const T dtdx = T(dt / P.dx), lam = T(dt / (2.0 * P.dx));
    const int nblocks = gridDim.x, b = blockIdx.x;
    const int per_xcd = nblocks / 8;
    const int item = b < 8 * per_xcd ? (b % 8) * per_xcd + b / 8 : b;
    const int ntiles = ntx * nty;
    const int seg = item / ntiles;
    const int tile = item % ntiles;
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int z0 = seg * zlen, z1 = min(z0 + zlen, P.nz);
    int hits = 0;
    double smax = 0.0;
    const bool want_cfl = co.dt_next != nullptr;
    godunov_tile<T, LIM, RS, TX, TY>(P, u_in, u_out, bflux, dtdx, lam, ph, x0, y0, z0, z1, sm, hits,
                                     want_cfl, smax);
    flush_hits(hits, hits_ctr);
    if (want_cfl) cfl_block_max(smax, co.smax_bits);
}

// A batch: a persistent grid; each workgroup pulls (patch, tile, z-range)
// items from an atomic counter until the table is exhausted. The last
// workgroup to leave resets the counter, so the next launch (or graph replay)
// starts from zero without a separate reset.
template <typename T, int LIM, int RS, int TX, int TY>
__global__ __launch_bounds__(tile_threads(TX, TY))
__attribute__((amdgpu_waves_per_eu(waves_per_eu<T>()))) void step_batched_kernel(
    const PatchDesc *__restrict__ patches, const WorkItem *__restrict__ items, int nitems,
    const T *__restrict__ u_in, T *__restrict__ u_out, T *__restrict__ bflux,
    const double *dt_dev, Scalars sc, unsigned long long *hits_ctr, unsigned *queue, CflOut co)
{
    __shared__ TileSmem<T, TX, TY> sm;
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
        godunov_tile<T, LIM, RS, TX, TY>(P, u_in, u_out, bflux, dtdx, lam, ph, w.x0, w.y0, w.z0,
                                         w.z1, sm, hits, want_cfl, smax);
        __syncthreads();
    }
    flush_hits(hits, hits_ctr);
    if (want_cfl) cfl_block_max(smax, co.smax_bits);
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned done = atomicAdd(&queue[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
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
            load5(base + view.plane(c.k) + view.column(i, j), view.vstride, U);
            vmax = fmax(vmax, cell_signal(U, ph, hits) * inv_dx);
        }
    }
    (void)hits_ctr;
    (void)cfl;
    (void)dt_out;
    (void)done;
    cfl_block_max(vmax, smax_bits);
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
        load5(base + view.plane(k) + view.column(i, j), view.vstride, U);
        vmax = fmax(vmax, cell_signal(U, ph, hits) * inv_dx);
    }
    (void)cfl;
    (void)dt_out;
    (void)done;
    cfl_block_max(vmax, smax_bits);
}

// ------------------------------------------------------------ launchers

template <typename T, int LIM, int RS, int TX, int TY>
static int launch_step_t(const PatchDesc &P, const void *u_in, void *u_out, void *bflux,
                         const double *dt_dev, const Scalars &sc, unsigned long long *hits,
                         int zlen, int min_blocks, const CflOut &co, hipStream_t s)
{
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    const int64_t ntiles = (int64_t)ntx * nty;
    if (ntiles * ((P.nz + zlen - 1) / zlen) < min_blocks) {
        // too few workgroups to fill the chip: shorter z-ranges, down to one
        // plane (a range recomputes the two planes below it, which an
        // otherwise idle chip absorbs)
        const int64_t want = (min_blocks + ntiles - 1) / ntiles;
        zlen = std::min<int64_t>(zlen, std::max<int64_t>(1, (P.nz + want - 1) / want));
    }
    const int nseg = (P.nz + zlen - 1) / zlen;
    const int64_t nblocks = (int64_t)ntx * nty * nseg;
    if (nblocks <= 0 || nblocks > 0x7fffffff) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((step_kernel<T, LIM, RS, TX, TY>), dim3((unsigned)nblocks),
                       dim3(TileGeom<TX, TY>::NT), 0, s, P, (const T *)u_in, (T *)u_out, (T *)bflux,
                       dt_dev, sc, hits, ntx, nty, zlen, co);
    if (co.dt_next)
        hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(64), 0, s, co.cfl, co.dt_next,
                           co.smax_bits);
    return (int)hipGetLastError();
}

template <typename T, int LIM, int RS, int TX, int TY>
static int launch_batched_t(const PatchDesc *d_patches, const WorkItem *d_items, int nitems,
                            const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                            const Scalars &sc, unsigned long long *hits, unsigned *d_queue,
                            int grid, const CflOut &co, hipStream_t s)
{
    hipLaunchKernelGGL((step_batched_kernel<T, LIM, RS, TX, TY>), dim3(grid),
                       dim3(TileGeom<TX, TY>::NT), 0, s, d_patches, d_items, nitems,
                       (const T *)u_in, (T *)u_out, (T *)bflux, dt_dev, sc, hits, d_queue, co);
    if (co.dt_next)
        hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(64), 0, s, co.cfl, co.dt_next,
                           co.smax_bits);
    return (int)hipGetLastError();
}

template <typename T, int LIM, int RS>
static int dispatch_shape_step(int shape, const PatchDesc &P, const void *u_in, void *u_out,
                               void *bflux, const double *dt_dev, const Scalars &sc,
                               unsigned long long *hits, int zlen, int min_blocks,
                               const CflOut &co, hipStream_t s)
{
    switch (shape) {
    case TILE_8x8: return launch_step_t<T, LIM, RS, 8, 8>(P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, min_blocks, co, s);
    case TILE_32x8: return launch_step_t<T, LIM, RS, 32, 8>(P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, min_blocks, co, s);
    case TILE_16x8: return launch_step_t<T, LIM, RS, 16, 8>(P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, min_blocks, co, s);
    case TILE_24x8: return launch_step_t<T, LIM, RS, 24, 8>(P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, min_blocks, co, s);
    default: return launch_step_t<T, LIM, RS, 16, 16>(P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, min_blocks, co, s);
    }
}

template <typename T, int LIM, int RS>
static int dispatch_shape_batched(int shape, const PatchDesc *d_patches, const WorkItem *d_items,
                                  int nitems, const void *u_in, void *u_out, void *bflux,
                                  const double *dt_dev, const Scalars &sc,
                                  unsigned long long *hits, unsigned *d_queue, int grid,
                                  const CflOut &co, hipStream_t s)
{
    switch (shape) {
    case TILE_8x8: return launch_batched_t<T, LIM, RS, 8, 8>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, co, s);
    case TILE_32x8: return launch_batched_t<T, LIM, RS, 32, 8>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, co, s);
    case TILE_16x8: return launch_batched_t<T, LIM, RS, 16, 8>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, co, s);
    case TILE_24x8: return launch_batched_t<T, LIM, RS, 24, 8>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, co, s);
    default: return launch_batched_t<T, LIM, RS, 16, 16>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, co, s);
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
                const Scalars &sc, unsigned long long *hits, int zlen, int min_blocks,
                const CflOut &co, hipStream_t s)
{
    if (dtype == 1)
        GD_DISPATCH_SCHEME(dispatch_shape_step, float, shape, P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, min_blocks, co, s);
    GD_DISPATCH_SCHEME(dispatch_shape_step, double, shape, P, u_in, u_out, bflux, dt_dev, sc, hits, zlen, min_blocks, co, s);
}

int launch_step_batched(int dtype, int limiter, int riemann, int shape,
                        const PatchDesc *d_patches, const WorkItem *d_items, int nitems,
                        const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                        const Scalars &sc, unsigned long long *hits, unsigned *d_queue, int grid,
                        const CflOut &co, hipStream_t s)
{
    if (dtype == 1)
        GD_DISPATCH_SCHEME(dispatch_shape_batched, float, shape, d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, co, s);
    GD_DISPATCH_SCHEME(dispatch_shape_batched, double, shape, d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, co, s);
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
    hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(64), 0, s, cfl, dt_out, smax_bits);
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
    hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(64), 0, s, cfl, dt_out, smax_bits);
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
    case TILE_16x8:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_batched_kernel<T, LIM, RS, 16, 8>, TileGeom<16, 8>::NT, 0);
        break;
    case TILE_24x8:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_batched_kernel<T, LIM, RS, 24, 8>, TileGeom<24, 8>::NT, 0);
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
