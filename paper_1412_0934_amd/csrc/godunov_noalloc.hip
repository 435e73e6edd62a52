// The batched Euler step for callers that cannot allocate device memory:
// godunov_step_batched_noalloc. Its work queue, counters and work
// decomposition live in `scratch`, a file-scope device array of fixed size
// that the code object carries, instead of library allocations; the patch
// descriptors are read from the caller's device memory at every launch, so
// the call needs no host-to-device copy either and can be captured into a
// HIP graph as it is.
//
// Two launches per call, stream-ordered:
//   na_plan_kernel  one workgroup: validates every descriptor, counts the
//                   (tile, z-range) work items of each patch, and writes the
//                   queue order -- patches grouped by z-range length, longest
//                   first, then in descriptor order -- with each patch's first
//                   item number; clears the queue counter;
//   na_step_kernel  the persistent step grid: workgroups take item numbers
//                   from the queue counter, find their patch by binary search
//                   in the plan and run the same tile march as every other
//                   step kernel.
#include "godunov.h"
#include "godunov_tile.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

namespace gd {

namespace {

constexpr int NA_MAX_PATCHES = 65536;
constexpr int NA_ZMAX = 32;          // longest z-range of an item
constexpr int NA_BUCKETS = 6;        // z-range lengths 32, 16..31, 8..15, 4..7, 2..3, 1
constexpr int NA_THREADS = 1024;     // threads of the plan kernel
// scratch words (64-bit): [0] queue counter, [1] number of items, [2] planned
// patches, [3] floor hits, [4] rejected descriptors, [5..7] unused; then the
// first item number of each planned patch and the total (NA_MAX_PATCHES + 1
// words); then the patch index of each queue position (NA_MAX_PATCHES int32,
// two per word)
constexpr int NA_HEAD = 8;
constexpr int NA_START = NA_HEAD;
constexpr int NA_ORDER = NA_START + NA_MAX_PATCHES + 1;
constexpr int NA_WORDS = NA_ORDER + NA_MAX_PATCHES / 2;

}  // namespace

}  // namespace gd

// 786,504 bytes per device, shared by every call on that device.
static __device__ __align__(256) unsigned long long scratch[gd::NA_WORDS];

namespace gd {

namespace {

struct NaItem {
    int32_t patch, x0, y0, z0, z1;
};

// Tile shape and z-range of a planned patch; items = 0 for a descriptor the
// step cannot take (it is skipped and counted).
template <int TX, int TY>
__device__ __forceinline__ int64_t na_items(const gd_patch &p, bool host_dt, int &zlen)
{
    const bool ok = p.nx >= 1 && p.ny >= 1 && p.nz >= 1 && p.nx <= 16384 && p.ny <= 16384 &&
                    p.nz <= 16384 && p.ng >= 2 && p.ng <= 64 && p.dx > 0.0 &&
                    (!host_dt || p.dt >= 0.0) && p.u_in_off >= 0 && p.u_out_off >= 0 &&
                    (int64_t)(p.nx + 2 * p.ng) * (p.ny + 2 * p.ng) <= 0x7fffffffLL;
    if (!ok) return 0;
    zlen = min(p.nz, NA_ZMAX);
    const int64_t ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    return ntx * nty * ((p.nz + zlen - 1) / zlen);
}

__device__ __forceinline__ int na_bucket(int zlen)
{
    // 32 -> 0, 16..31 -> 1, ..., 1 -> 5
    return 5 - (31 - __clz(zlen));
}

// Exclusive prefix sum over the NA_THREADS threads of the workgroup.
__device__ unsigned long long block_exclusive_scan(unsigned long long v, unsigned long long *part,
                                                   unsigned long long &total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned long long x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) part[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        for (int w = 0; w < NA_THREADS / 64; ++w) {
            unsigned long long t = part[w];
            part[w] = run;
            run += t;
        }
        part[NA_THREADS / 64] = run;
    }
    __syncthreads();
    const unsigned long long r = part[wv] + x - v;
    total = part[NA_THREADS / 64];
    __syncthreads();
    return r;
}

template <int TX, int TY>
__global__ __launch_bounds__(NA_THREADS) void na_plan_kernel(const gd_patch *__restrict__ patches,
                                                            int npatch, int host_dt,
                                                            unsigned long long *__restrict__ scr)
{
    __shared__ unsigned long long part[NA_THREADS / 64 + 1];
    // thread t plans the contiguous descriptors [lo, hi)
    const int per = (npatch + NA_THREADS - 1) / NA_THREADS;
    const int lo = min(npatch, (int)threadIdx.x * per), hi = min(npatch, lo + per);
    unsigned long long items[NA_BUCKETS], count[NA_BUCKETS];
#pragma unroll
    for (int b = 0; b < NA_BUCKETS; ++b) items[b] = count[b] = 0;
    unsigned long long bad = 0;
    for (int i = lo; i < hi; ++i) {
        const gd_patch p = patches[i];
        int zlen = 1;
        const int64_t n = na_items<TX, TY>(p, host_dt != 0, zlen);
        if (n == 0) { ++bad; continue; }
        const int b = na_bucket(zlen);
#pragma unroll
        for (int c = 0; c < NA_BUCKETS; ++c)
            if (c == b) { items[c] += (unsigned long long)n; count[c] += 1; }
    }
    // bases of this thread's patches in each bucket, buckets in queue order
    unsigned long long ibase[NA_BUCKETS], cbase[NA_BUCKETS];
    unsigned long long irun = 0, crun = 0;
#pragma unroll
    for (int b = 0; b < NA_BUCKETS; ++b) {
        unsigned long long itot, ctot;
        ibase[b] = irun + block_exclusive_scan(items[b], part, itot);
        cbase[b] = crun + block_exclusive_scan(count[b], part, ctot);
        irun += itot;
        crun += ctot;
    }
    unsigned long long badtot;
    (void)block_exclusive_scan(bad, part, badtot);
    int32_t *order = (int32_t *)(scr + NA_ORDER);
    for (int i = lo; i < hi; ++i) {
        const gd_patch p = patches[i];
        int zlen = 1;
        const int64_t n = na_items<TX, TY>(p, host_dt != 0, zlen);
        if (n == 0) continue;
        const int b = na_bucket(zlen);
        unsigned long long pos = 0, first = 0;
#pragma unroll
        for (int c = 0; c < NA_BUCKETS; ++c)
            if (c == b) {
                pos = cbase[c]++;
                first = ibase[c];
                ibase[c] += (unsigned long long)n;
            }
        scr[NA_START + pos] = first;
        order[pos] = i;
    }
    if (threadIdx.x == 0) {
        scr[NA_START + crun] = irun;    // the end of the last planned patch
        scr[0] = 0;                     // queue counter
        scr[1] = irun;                  // items
        scr[2] = crun;                  // planned patches
        scr[3] = 0;
        scr[4] = badtot;
    }
}

// The planned patch holding item `it`: the last position whose first item is
// at or below it.
__device__ __forceinline__ int na_find(const unsigned long long *__restrict__ scr, int nplanned,
                                       unsigned long long it)
{
    int lo = 0, hi = nplanned - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (scr[NA_START + mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T, int LIM, int RS, int TX, int TY>
__global__ __launch_bounds__(tile_threads(TX, TY))
__attribute__((amdgpu_waves_per_eu(waves_per_eu<T>()))) void na_step_kernel(
    const gd_patch *__restrict__ patches, const T *__restrict__ u_in, T *__restrict__ u_out,
    T *__restrict__ bflux, const double *dt_dev, Scalars sc, unsigned long long *scr)
{
    __shared__ TileSmem<T, TX, TY> sm;
    __shared__ NaItem s_item;
    const Phys<T> ph = make_phys<T>(sc);
    const unsigned long long nitems = scr[1];
    const int nplanned = (int)scr[2];
    const int32_t *order = (const int32_t *)(scr + NA_ORDER);
    int hits = 0;
    double smax = 0.0;
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned long long it = atomicAdd(&scr[0], 1ull);
            NaItem w{ -1, 0, 0, 0, 0 };
            if (it < nitems) {
                const int pos = na_find(scr, nplanned, it);
                const int p = order[pos];
                const gd_patch g = patches[p];
                const int zlen = min(g.nz, NA_ZMAX);
                const int64_t local = (int64_t)(it - scr[NA_START + pos]);
                const int64_t ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY;
                const int64_t tile = local % (ntx * nty), seg = local / (ntx * nty);
                w.patch = p;
                w.x0 = (int)(tile % ntx) * TX;
                w.y0 = (int)(tile / ntx) * TY;
                w.z0 = (int)seg * zlen;
                w.z1 = min(w.z0 + zlen, g.nz);
            }
            s_item = w;
        }
        __syncthreads();
        const NaItem w = s_item;
        __syncthreads();
        if (w.patch < 0) break;
        const gd_patch g = patches[w.patch];
        PatchDesc P{};
        P.nx = g.nx; P.ny = g.ny; P.nz = g.nz; P.ng = g.ng; P.periodic = 0;
        P.in_off = g.u_in_off; P.out_off = g.u_out_off; P.flux_off = g.flux_off;
        P.dx = g.dx; P.dt = g.dt;
        const double dt = dt_dev ? *dt_dev : P.dt;
        const T dtdx = T(dt / P.dx), lam = T(dt / (2.0 * P.dx));
        godunov_tile<T, LIM, RS, TX, TY, tile_threads(TX, TY), true>(
            P, u_in, u_out, bflux, dtdx, lam, ph, w.x0, w.y0, w.z0, w.z1, sm, hits, false, smax);
        __syncthreads();
    }
    flush_hits(hits, &scr[3]);
}

// Per-device state: the device address of `scratch` (each GPU holds its own
// copy of the array at its own address), the CU count, and the resident
// workgroups per CU of each step-kernel variant.
constexpr int NA_MAX_DEVICES = 64;
struct NaDevice {
    bool ready = false;
    unsigned long long *scr = nullptr;
    int num_cus = 0;
};
NaDevice g_na[NA_MAX_DEVICES];
std::mutex g_na_lock;

template <typename T, int LIM, int RS, int TX, int TY>
int na_launch_t(const gd_patch *patches, int npatch, const void *u_in, void *u_out, void *bflux,
                const double *dt_dev, const Scalars &sc, const NaDevice &d, hipStream_t s)
{
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, na_step_kernel<T, LIM, RS, TX, TY>, tile_threads(TX, TY), 0);
    if (e != hipSuccess) return (int)e;
    if (per_cu < 1) per_cu = 1;
    hipLaunchKernelGGL((na_plan_kernel<TX, TY>), dim3(1), dim3(NA_THREADS), 0, s, patches, npatch,
                       dt_dev ? 0 : 1, d.scr);
    hipLaunchKernelGGL((na_step_kernel<T, LIM, RS, TX, TY>), dim3(per_cu * d.num_cus),
                       dim3(tile_threads(TX, TY)), 0, s, patches, (const T *)u_in, (T *)u_out,
                       (T *)bflux, dt_dev, sc, d.scr);
    return (int)hipGetLastError();
}

// FP64 on 16x8 tiles (the shape the autotuner picks for batches of
// 8^3..32^3 patches), FP32 on 24x8 tiles (within about 5% of the 16x8 + 24x8
// pair it picks there). Results do not depend on the shape.
template <typename T, int LIM, int RS>
int na_launch_shape(const gd_patch *patches, int npatch, const void *u_in, void *u_out, void *bflux,
                    const double *dt_dev, const Scalars &sc, const NaDevice &d, hipStream_t s)
{
    if constexpr (sizeof(T) == 8)
        return na_launch_t<T, LIM, RS, 16, 8>(patches, npatch, u_in, u_out, bflux, dt_dev, sc, d, s);
    else
        return na_launch_t<T, LIM, RS, 24, 8>(patches, npatch, u_in, u_out, bflux, dt_dev, sc, d, s);
}

#define GD_NA_DISPATCH(T, ...)                                                                  \
    do {                                                                                        \
        if (riemann == RS_HLL) {                                                                \
            if (limiter == LIM_MC) return na_launch_shape<T, LIM_MC, RS_HLL>(__VA_ARGS__);      \
            if (limiter == LIM_NONE) return na_launch_shape<T, LIM_NONE, RS_HLL>(__VA_ARGS__);  \
            return na_launch_shape<T, LIM_MINMOD, RS_HLL>(__VA_ARGS__);                         \
        }                                                                                       \
        if (limiter == LIM_MC) return na_launch_shape<T, LIM_MC, RS_HLLC>(__VA_ARGS__);         \
        if (limiter == LIM_NONE) return na_launch_shape<T, LIM_NONE, RS_HLLC>(__VA_ARGS__);     \
        return na_launch_shape<T, LIM_MINMOD, RS_HLLC>(__VA_ARGS__);                            \
    } while (0)

int na_launch(int dtype, int limiter, int riemann, const gd_patch *patches, int npatch,
              const void *u_in, void *u_out, void *bflux, const double *dt_dev, const Scalars &sc,
              const NaDevice &d, hipStream_t s)
{
    if (dtype == GD_F32)
        GD_NA_DISPATCH(float, patches, npatch, u_in, u_out, bflux, dt_dev, sc, d, s);
    GD_NA_DISPATCH(double, patches, npatch, u_in, u_out, bflux, dt_dev, sc, d, s);
}

// Set-up of the current device, once: the device address of `scratch`.
int na_device(int dev, NaDevice **out)
{
    if (dev < 0 || dev >= NA_MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_na_lock);
    NaDevice &d = g_na[dev];
    if (!d.ready) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return (int)e;
        d.scr = (unsigned long long *)p;
        d.num_cus = cus > 0 ? cus : 256;
        d.ready = true;
    }
    *out = &d;
    return 0;
}

}  // namespace

}  // namespace gd

extern "C" int godunov_step_batched_noalloc(const gd_opts *opts, int npatch,
                                            const gd_patch *patches_dev, const void *u_in_base,
                                            void *u_out_base, void *bflux_base,
                                            const double *dt_dev, double gamma, void *hip_stream)
{
    using namespace gd;
    if (!opts) return set_call_error(GD_E_ARG, "opts is NULL");
    if (opts->dtype != GD_F64 && opts->dtype != GD_F32)
        return set_call_error(GD_E_ARG, "bad dtype %d", opts->dtype);
    if (opts->bc != GD_GHOSTED)
        return set_call_error(GD_E_UNSUPPORTED, "the batched step takes ghosted patches only");
    if (opts->limiter < GD_MINMOD || opts->limiter > GD_UNLIMITED)
        return set_call_error(opts->limiter <= GD_PPM_CT_UNLIMITED ? GD_E_UNSUPPORTED : GD_E_ARG,
                              "limiter %d is not available without allocation", opts->limiter);
    if (opts->riemann != GD_HLLC && opts->riemann != GD_HLL)
        return set_call_error(GD_E_ARG, "bad riemann solver %d", opts->riemann);
    if (!(opts->rho_floor >= 0.0) || !(opts->p_floor >= 0.0))
        return set_call_error(GD_E_ARG, "floors must be >= 0");
    if (npatch < 1 || npatch > NA_MAX_PATCHES)
        return set_call_error(GD_E_ARG, "npatch %d outside [1, %d], the static scratch's limit",
                              npatch, NA_MAX_PATCHES);
    if (!patches_dev || !u_in_base || !u_out_base)
        return set_call_error(GD_E_ARG, "patches_dev, u_in_base and u_out_base must not be NULL");
    if (!(gamma > 1.0)) return set_call_error(GD_E_ARG, "gamma must be > 1");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_call_error(GD_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    NaDevice *d = nullptr;
    int r = na_device(dev, &d);
    if (r) return set_call_error(GD_E_HIP, "scratch set-up on device %d: %s", dev,
                                 hipGetErrorString((hipError_t)r));
    Scalars sc{ gamma, opts->rho_floor, opts->p_floor };
    r = na_launch(opts->dtype, opts->limiter, opts->riemann, patches_dev, npatch, u_in_base,
                  u_out_base, bflux_base, dt_dev, sc, *d, (hipStream_t)hip_stream);
    if (r) return set_call_error(GD_E_HIP, "godunov_step_batched_noalloc launch: %s",
                                 hipGetErrorString((hipError_t)r));
    return GD_OK;
}
