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
#include "godunov_tile.h"

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
int patch_tile_shape(int shape, int nx, int ny)
{
    if (shape != TILE_PAIR_24x8) return shape;
    const int other = TILE_24x8;
    auto padded = [&](int sh) {
        const int tx = tile_tx(sh), ty = tile_ty(sh);
        return (int64_t)((nx + tx - 1) / tx * tx) * ((ny + ty - 1) / ty * ty);
    };
    return padded(other) < padded(TILE_16x8) ? other : TILE_16x8;
}

// workgroup size of a pair kernel: the larger of the two tiles'
constexpr int pair_threads(int txb, int tyb)
{
    return tile_threads(txb, tyb) > tile_threads(16, 8) ? tile_threads(txb, tyb) : tile_threads(16, 8);
}


__global__ __launch_bounds__(64) void cfl_finalize_kernel(double cfl, double *dt_out,
                                                          unsigned long long *smax_bits)
{
    if (threadIdx.x == 0) {
        const unsigned long long b = atomicExch(smax_bits, 0ull);
        *dt_out = cfl / __longlong_as_double((long long)b);
    }
}


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
        godunov_tile<T, LIM, RS, TX, TY, tile_threads(TX, TY), true>(
            P, u_in, u_out, bflux, dtdx, lam, ph, w.x0, w.y0, w.z0, w.z1, sm, hits, want_cfl, smax);
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

// A batch in two tile shapes: the same work queue, each item naming its
// shape (A = 16x8 or B). Workgroups are sized for the larger tile; a thread
// that owns no column of a smaller tile only shares the staging and the face
// solves. The two shapes' LDS buffers overlap.
template <typename T, int LIM, int RS, int TXB, int TYB>
__global__ __launch_bounds__(pair_threads(TXB, TYB))
__attribute__((amdgpu_waves_per_eu(waves_per_eu<T>()))) void step_batched_pair_kernel(
    const PatchDesc *__restrict__ patches, const WorkItem *__restrict__ items, int nitems,
    const T *__restrict__ u_in, T *__restrict__ u_out, T *__restrict__ bflux,
    const double *dt_dev, Scalars sc, unsigned long long *hits_ctr, unsigned *queue, CflOut co)
{
    constexpr int NT = pair_threads(TXB, TYB);
    __shared__ union {
        TileSmem<T, 16, 8> a;
        TileSmem<T, TXB, TYB> b;
    } sm;
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
        if (w.shape == TILE_16x8)
            godunov_tile<T, LIM, RS, 16, 8, NT, true>(P, u_in, u_out, bflux, dtdx, lam, ph, w.x0, w.y0,
                                                w.z0, w.z1, sm.a, hits, want_cfl, smax);
        else
            godunov_tile<T, LIM, RS, TXB, TYB, NT, true>(P, u_in, u_out, bflux, dtdx, lam, ph, w.x0,
                                                   w.y0, w.z0, w.z1, sm.b, hits, want_cfl, smax);
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

template <typename T, int LIM, int RS, int TXB, int TYB>
static int launch_batched_pair_t(const PatchDesc *d_patches, const WorkItem *d_items, int nitems,
                                 const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                                 const Scalars &sc, unsigned long long *hits, unsigned *d_queue,
                                 int grid, const CflOut &co, hipStream_t s)
{
    hipLaunchKernelGGL((step_batched_pair_kernel<T, LIM, RS, TXB, TYB>), dim3(grid),
                       dim3(pair_threads(TXB, TYB)), 0, s, d_patches, d_items, nitems,
                       (const T *)u_in, (T *)u_out, (T *)bflux, dt_dev, sc, hits, d_queue, co);
    if (co.dt_next)
        hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(64), 0, s, co.cfl, co.dt_next,
                           co.smax_bits);
    return (int)hipGetLastError();
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
    case TILE_PAIR_24x8: return launch_batched_pair_t<T, LIM, RS, 24, 8>(d_patches, d_items, nitems, u_in, u_out, bflux, dt_dev, sc, hits, d_queue, grid, co, s);
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
    case TILE_PAIR_24x8:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_batched_pair_kernel<T, LIM, RS, 24, 8>, pair_threads(24, 8), 0);
        break;
    default:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_batched_kernel<T, LIM, RS, 16, 16>, TileGeom<16, 16>::NT, 0);
    }
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

int launch_cfl_finalize(double cfl, double *dt_out, unsigned long long *smax_bits, hipStream_t s)
{
    hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(64), 0, s, cfl, dt_out, smax_bits);
    return (int)hipGetLastError();
}

int max_resident_blocks(int dtype, int limiter, int riemann, int shape, int device)
{
    if (dtype == 1) GD_DISPATCH_SCHEME(occupancy_t, float, shape, device);
    GD_DISPATCH_SCHEME(occupancy_t, double, shape, device);
}

}  // namespace gd
