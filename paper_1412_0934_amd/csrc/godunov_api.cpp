// C-ABI host layer of libgodunov.so: argument validation, the context (device
// counters, cached batch tables, tuning choices) and dispatch to the kernels.
#include "godunov.h"
#include "godunov_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace {

// Message of the last failure that had no context to hold it (gd_create, or
// an argument check of a call made with a NULL context).
thread_local std::string g_create_error;

struct BatchCache {
    std::vector<gd_patch> host;       // descriptors the tables were built from
    int dtype = -1, shape = -1;
    gd::PatchDesc *d_patches = nullptr;
    gd::WorkItem *d_items = nullptr;
    gd::CflItem *d_cfl_items = nullptr;
    int nitems = 0, ncfl = 0;
    size_t cap_patches = 0, cap_items = 0, cap_cfl = 0;
    bool captured = false;            // a stream capture used these tables
};

// Scratch memory grown on demand. A buffer that a stream capture used is
// never freed before gd_destroy: a graph made from that capture still reads it.
struct Scratch {
    void *p = nullptr;
    size_t bytes = 0;
    bool captured = false;
};

// Device counters of one stream: the batched work queue and the CFL and MHD
// speed accumulators. Streams get slots of their own (up to NSLOT streams),
// so launches in flight together on different streams do not share them.
constexpr int NSLOT = 64;
constexpr int SLOT_U64 = 8, SLOT_U32 = 4;
struct Slot {
    unsigned long long *u64;   // [1] cfl max bits, [2] fused cfl max bits,
                               // [4..5] MHD speed maxima, [6..7] fused MHD maxima
    unsigned *u32;             // [0..1] work queue, [2] cfl done, [3] fused cfl done
};

}  // namespace

namespace gd {

int set_call_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_create_error = buf;
    return code;
}

}  // namespace gd

struct gd_stream_state;                  // the streamed-batch pipeline (below)
static void free_stream_state(gd_stream_state *st);

struct gd_ctx {
    int device = 0;
    int num_cus = 0;
    std::string err;
    // device counters: d_u64[0] floor hits (summed by every stream), then
    // NSLOT per-stream slots of SLOT_U64 words; d_u32: NSLOT slots of SLOT_U32
    unsigned long long *d_u64 = nullptr;
    unsigned *d_u32 = nullptr;
    std::vector<hipStream_t> slot_stream;   // stream of each assigned slot
    unsigned slot_shared = 0;               // round robin beyond NSLOT streams
    BatchCache batch;
    BatchCache ppm_batch;                // work items of the fused PPM batched step
    BatchCache cfl;                      // descriptor cache used by cfl_dt
    Scratch adj;                         // adjoint scratch (grown on demand)
    Scratch mhd;                         // MHD step scratch (grown on demand)
    Scratch ppm_s;                       // PPM face-state scratch (grown on demand)
    std::vector<void *> retired;         // captured buffers replaced since; freed at destroy
    gd_stream_state *stream = nullptr;   // streamed batches (created on first use)
    // tuned configuration per dtype (index 0: FP64, 1: FP32)
    int zlen_single[2] = { 32, 32 };
    int shape_single[2] = { gd::TILE_16x16, gd::TILE_16x16 };
    int shape_batched[2] = { gd::TILE_16x16, gd::TILE_16x16 };
    int zpolicy_batched[2] = { 1, 1 };
};

namespace {

int fail(gd_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_error = buf;
    return code;
}

int hip_fail(gd_ctx *ctx, int e, const char *where)
{
    return fail(ctx, GD_E_HIP, "%s: HIP error %d (%s)", where, e,
                hipGetErrorString((hipError_t)e));
}

int check_opts(gd_ctx *ctx, const gd_opts *o)
{
    if (!o) return fail(ctx, GD_E_ARG, "opts is NULL");
    if (o->dtype != GD_F64 && o->dtype != GD_F32) return fail(ctx, GD_E_ARG, "bad dtype %d", o->dtype);
    if (o->bc != GD_GHOSTED && o->bc != GD_PERIODIC) return fail(ctx, GD_E_ARG, "bad bc %d", o->bc);
    if (o->limiter < GD_MINMOD || o->limiter > GD_PPM_CT_UNLIMITED)
        return fail(ctx, GD_E_ARG, "bad limiter %d", o->limiter);
    if (o->riemann != GD_HLLC && o->riemann != GD_HLL)
        return fail(ctx, GD_E_ARG, "bad riemann solver %d", o->riemann);
    if (!(o->rho_floor >= 0.0) || !(o->p_floor >= 0.0))
        return fail(ctx, GD_E_ARG, "floors must be >= 0");
    return GD_OK;
}

size_t elem_size(const gd_opts *o) { return o->dtype == GD_F32 ? 4 : 8; }

bool is_ppm(const gd_opts *o) { return o->limiter >= GD_PPM && o->limiter <= GD_PPM_CT_UNLIMITED; }

int reject_ppm(gd_ctx *ctx, const gd_opts *o, const char *what)
{
    if (is_ppm(o)) return fail(ctx, GD_E_UNSUPPORTED, "%s does not take the PPM reconstruction", what);
    return GD_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    auto pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

int64_t in_elems(int nx, int ny, int nz, int ng, bool periodic)
{
    if (periodic) return 5LL * nx * ny * nz;
    return 5LL * (nx + 2LL * ng) * (ny + 2LL * ng) * (nz + 2LL * ng);
}

int64_t flux_elems(int nx, int ny, int nz)
{
    return 10LL * ((int64_t)nz * ny + (int64_t)nz * nx + (int64_t)ny * nx);
}

int check_extents(gd_ctx *ctx, int nx, int ny, int nz, int ng, bool periodic)
{
    if (nx < 1 || ny < 1 || nz < 1) return fail(ctx, GD_E_ARG, "extents must be >= 1 (%d,%d,%d)", nx, ny, nz);
    // the kernels use 16-bit tile coordinates and 32-bit plane offsets
    if (nx > 16384 || ny > 16384 || nz > 16384) return fail(ctx, GD_E_ARG, "extent above 16384");
    if (!periodic && ng < 2) return fail(ctx, GD_E_ARG, "ng must be >= 2 in ghosted mode (got %d)", ng);
    if (!periodic && ng > 64) return fail(ctx, GD_E_ARG, "ng above 64");
    int64_t gx = periodic ? nx : nx + 2LL * ng, gy = periodic ? ny : ny + 2LL * ng;
    if (gx * gy > 0x7fffffffLL) return fail(ctx, GD_E_ARG, "plane too large");
    return GD_OK;
}

int check_scalars(gd_ctx *ctx, double gamma, double dx, double dt)
{
    if (!(gamma > 1.0)) return fail(ctx, GD_E_ARG, "gamma must be > 1");
    if (!(dx > 0.0)) return fail(ctx, GD_E_ARG, "dx must be > 0");
    if (!(dt >= 0.0)) return fail(ctx, GD_E_ARG, "dt must be >= 0");
    return GD_OK;
}

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

// The counter slot of stream s (assigned on the stream's first call; host
// bookkeeping only, so a first call under capture is fine).
Slot slot_for(gd_ctx *ctx, hipStream_t s)
{
    int i = -1;
    for (size_t k = 0; k < ctx->slot_stream.size(); ++k)
        if (ctx->slot_stream[k] == s) { i = (int)k; break; }
    if (i < 0) {
        if ((int)ctx->slot_stream.size() < NSLOT) {
            ctx->slot_stream.push_back(s);
            i = (int)ctx->slot_stream.size() - 1;
        } else {
            i = (int)(ctx->slot_shared++ % NSLOT);
        }
    }
    return Slot{ ctx->d_u64 + SLOT_U64 * (i + 1), ctx->d_u32 + SLOT_U32 * i };
}

// Free a device buffer that is being replaced, unless a capture used it.
void release(gd_ctx *ctx, void *p, bool captured)
{
    if (!p) return;
    if (captured) ctx->retired.push_back(p);
    else (void)hipFree(p);
}

// Grow a scratch buffer to `need` bytes. The growth waits for the device
// (work already queued may use the old buffer) and is refused under stream
// capture; a call under capture marks the buffer as captured.
int ensure_scratch(gd_ctx *ctx, Scratch &sc, size_t need, hipStream_t s, const char *what)
{
    const bool cap = capturing(s);
    if (need > sc.bytes || !sc.p) {
        if (cap)
            return fail(ctx, GD_E_UNSUPPORTED,
                        "%s scratch must grow (to %zu bytes), which a stream capture cannot do: "
                        "make one call of this size outside the capture first", what, need);
        hipError_t he = hipDeviceSynchronize();
        if (he != hipSuccess) return hip_fail(ctx, he, what);
        release(ctx, sc.p, sc.captured);
        sc = Scratch{};
        if (hipMalloc(&sc.p, need) != hipSuccess) {
            sc.p = nullptr;
            return fail(ctx, GD_E_NOMEM, "%s scratch of %zu bytes", what, need);
        }
        sc.bytes = need;
    }
    if (cap) sc.captured = true;
    return GD_OK;
}

// A table cache that must be rebuilt: refused under capture; otherwise the
// device waits (other streams may read the tables) and captured tables are
// set aside rather than overwritten.
int prepare_rebuild(gd_ctx *ctx, hipStream_t s, bool &captured, std::initializer_list<void **> ptrs,
                    std::initializer_list<size_t *> caps, const char *what)
{
    if (capturing(s))
        return fail(ctx, GD_E_UNSUPPORTED,
                    "the %s for these descriptors are not built, which a stream capture cannot do: "
                    "make one call with them outside the capture first", what);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    if (captured) {
        for (void **p : ptrs) {
            release(ctx, *p, true);
            *p = nullptr;
        }
        for (size_t *c : caps) *c = 0;
        captured = false;
    }
    return GD_OK;
}

template <typename X>
int ensure_capacity(gd_ctx *ctx, X **ptr, size_t *cap, size_t n)
{
    if (n <= *cap && *ptr) return GD_OK;
    if (*ptr) (void)hipFree(*ptr);
    *ptr = nullptr;
    *cap = 0;
    size_t want = std::max<size_t>(n, 16);
    hipError_t e = hipMalloc((void **)ptr, want * sizeof(X));
    if (e != hipSuccess) return fail(ctx, GD_E_NOMEM, "hipMalloc of %zu bytes failed", want * sizeof(X));
    *cap = want;
    return GD_OK;
}

bool same_patches(const BatchCache &c, int npatch, const gd_patch *p)
{
    return (int)c.host.size() == npatch && std::memcmp(c.host.data(), p, npatch * sizeof(gd_patch)) == 0;
}

int validate_patches(gd_ctx *ctx, int npatch, const gd_patch *patches, bool periodic)
{
    if (npatch < 1) return fail(ctx, GD_E_ARG, "npatch must be >= 1");
    if (!patches) return fail(ctx, GD_E_ARG, "patches is NULL");
    for (int i = 0; i < npatch; ++i) {
        const gd_patch &p = patches[i];
        int r = check_extents(ctx, p.nx, p.ny, p.nz, p.ng, periodic);
        if (r) {
            std::string why = gd_last_error(ctx);
            return fail(ctx, r, "patch %d: %s", i, why.c_str());
        }
        if (!(p.dx > 0.0)) return fail(ctx, GD_E_ARG, "patch %d: dx must be > 0", i);
        if (!(p.dt >= 0.0)) return fail(ctx, GD_E_ARG, "patch %d: dt must be >= 0", i);
        if (p.u_in_off < 0 || p.u_out_off < 0) return fail(ctx, GD_E_ARG, "patch %d: negative offset", i);
    }
    return GD_OK;
}

gd::PatchDesc to_desc(const gd_patch &p, bool periodic)
{
    gd::PatchDesc d{};
    d.nx = p.nx; d.ny = p.ny; d.nz = p.nz; d.ng = periodic ? 0 : p.ng;
    d.periodic = periodic ? 1 : 0;
    d.in_off = p.u_in_off; d.out_off = p.u_out_off; d.flux_off = p.flux_off;
    d.dx = p.dx; d.dt = p.dt;
    return d;
}

// z-range length of batched items by patch size: long enough to amortise the
// two extra planes a march reads, short enough to spread a patch over
// several workgroups.
// Policies: 0 = ranges of 8 planes, 1 = ranges of 16 planes (a patch of up
// to 32 planes is split in two), 2 = the whole patch in one range, 3 (the
// PPM march, whose window reaches three planes past a range) = ranges of up
// to 32 planes.
int batched_zlen(int nz, int policy)
{
    if (policy == 0) return std::min(nz, 8);
    if (policy == 2) return nz;
    if (policy == 3) return std::min(nz, 32);
    return nz <= 16 ? nz : (nz <= 32 ? (nz + 1) / 2 : 16);
}

int build_step_tables(gd_ctx *ctx, int dtype, int shape, int zpolicy, int npatch,
                      const gd_patch *patches, hipStream_t s, BatchCache *cache = nullptr)
{
    BatchCache &c = cache ? *cache : ctx->batch;
    const int tag = dtype * 16 + zpolicy;
    if (c.dtype == tag && c.shape == shape && same_patches(c, npatch, patches)) {
        if (capturing(s)) c.captured = true;
        return GD_OK;
    }
    int r;
    if ((r = prepare_rebuild(ctx, s, c.captured, { (void **)&c.d_patches, (void **)&c.d_items },
                             { &c.cap_patches, &c.cap_items }, "batch tables")))
        return r;
    std::vector<gd::PatchDesc> desc(npatch);
    std::vector<gd::WorkItem> items;
    std::vector<std::pair<int64_t, int>> order;     // (cells, patch): largest first
    for (int i = 0; i < npatch; ++i) {
        desc[i] = to_desc(patches[i], false);
        order.push_back({-(int64_t)patches[i].nx * patches[i].ny * patches[i].nz, i});
    }
    std::stable_sort(order.begin(), order.end());
    for (auto &o : order) {
        const gd_patch &p = patches[o.second];
        const int zl = batched_zlen(p.nz, zpolicy);
        const int pshape = gd::patch_tile_shape(shape, p.nx, p.ny);
        const int TX = gd::tile_tx(pshape), TY = gd::tile_ty(pshape);
        for (int z0 = 0; z0 < p.nz; z0 += zl)
            for (int y0 = 0; y0 < p.ny; y0 += TY)
                for (int x0 = 0; x0 < p.nx; x0 += TX) {
                    gd::WorkItem w{};
                    w.patch = o.second;
                    w.x0 = (int16_t)x0; w.y0 = (int16_t)y0;
                    w.z0 = (int16_t)z0; w.z1 = (int16_t)std::min(z0 + zl, p.nz);
                    w.shape = (int16_t)pshape;
                    items.push_back(w);
                }
    }
    if (items.size() > 0x7fffffff) return fail(ctx, GD_E_ARG, "too many work items");
    if ((r = ensure_capacity(ctx, &c.d_patches, &c.cap_patches, desc.size()))) return r;
    if ((r = ensure_capacity(ctx, &c.d_items, &c.cap_items, items.size()))) return r;
    // The tables are written before any kernel that reads them (the device
    // waited above): a synchronous copy keeps the host vectors' lifetime out
    // of the stream.
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(c.d_patches, desc.data(), desc.size() * sizeof(gd::PatchDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c.d_items, items.data(), items.size() * sizeof(gd::WorkItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "upload of batch tables");
    c.host.assign(patches, patches + npatch);
    c.nitems = (int)items.size();
    c.dtype = tag;
    c.shape = shape;
    return GD_OK;
}

int build_cfl_tables(gd_ctx *ctx, bool periodic, int npatch, const gd_patch *patches, hipStream_t s,
                     BatchCache *cache = nullptr)
{
    BatchCache &c = cache ? *cache : ctx->cfl;
    int tag = periodic ? 1 : 0;
    if (c.dtype == tag && same_patches(c, npatch, patches)) {
        if (capturing(s)) c.captured = true;
        return GD_OK;
    }
    int r;
    if ((r = prepare_rebuild(ctx, s, c.captured, { (void **)&c.d_patches, (void **)&c.d_cfl_items },
                             { &c.cap_patches, &c.cap_cfl }, "CFL tables")))
        return r;
    std::vector<gd::PatchDesc> desc(npatch);
    std::vector<gd::CflItem> items;
    for (int i = 0; i < npatch; ++i) {
        const gd_patch &p = patches[i];
        desc[i] = to_desc(p, periodic);
        // about 2048 cells per item
        int rows = std::max(1, std::min(p.ny, 2048 / std::max(1, p.nx)));
        for (int k = 0; k < p.nz; ++k)
            for (int j0 = 0; j0 < p.ny; j0 += rows)
                items.push_back(gd::CflItem{ i, k, j0, std::min(rows, p.ny - j0) });
    }
    if (items.size() > 0x7fffffff) return fail(ctx, GD_E_ARG, "too many cfl items");
    if ((r = ensure_capacity(ctx, &c.d_patches, &c.cap_patches, desc.size()))) return r;
    if ((r = ensure_capacity(ctx, &c.d_cfl_items, &c.cap_cfl, items.size()))) return r;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(c.d_patches, desc.data(), desc.size() * sizeof(gd::PatchDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c.d_cfl_items, items.data(), items.size() * sizeof(gd::CflItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "upload of cfl tables");
    c.host.assign(patches, patches + npatch);
    c.ncfl = (int)items.size();
    c.dtype = tag;
    return GD_OK;
}

int set_device(gd_ctx *ctx)
{
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    return GD_OK;
}

}  // namespace

extern "C" {

int gd_create(gd_ctx **out, int device)
{
    if (!out) return fail(nullptr, GD_E_ARG, "ctx pointer is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1) return fail(nullptr, GD_E_HIP, "no HIP device available");
    if (device < 0 || device >= n) return fail(nullptr, GD_E_ARG, "device %d out of range [0,%d)", device, n);
    if ((e = hipSetDevice(device)) != hipSuccess) return fail(nullptr, GD_E_HIP, "hipSetDevice(%d) failed", device);
    gd_ctx *ctx = new gd_ctx();
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    if (ctx->num_cus < 1) ctx->num_cus = 256;
    const size_t n64 = SLOT_U64 * (NSLOT + 1), n32 = SLOT_U32 * NSLOT;
    e = hipMalloc((void **)&ctx->d_u64, n64 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->d_u32, n32 * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(ctx->d_u64, 0, n64 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(ctx->d_u32, 0, n32 * sizeof(unsigned));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        gd_destroy(ctx);
        return fail(nullptr, GD_E_NOMEM, "device scratch allocation failed");
    }
    *out = ctx;
    return GD_OK;
}

int gd_destroy(gd_ctx *ctx)
{
    if (!ctx) return GD_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (BatchCache *c : { &ctx->batch, &ctx->ppm_batch, &ctx->cfl }) {
        if (c->d_patches) (void)hipFree(c->d_patches);
        if (c->d_items) (void)hipFree(c->d_items);
        if (c->d_cfl_items) (void)hipFree(c->d_cfl_items);
    }
    for (Scratch *sc : { &ctx->adj, &ctx->mhd, &ctx->ppm_s })
        if (sc->p) (void)hipFree(sc->p);
    for (void *p : ctx->retired) (void)hipFree(p);
    free_stream_state(ctx->stream);
    if (ctx->d_u64) (void)hipFree(ctx->d_u64);
    if (ctx->d_u32) (void)hipFree(ctx->d_u32);
    delete ctx;
    return GD_OK;
}

const char *gd_last_error(const gd_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int gd_get_stats(gd_ctx *ctx, uint64_t *floor_hits)
{
    if (!ctx || !floor_hits) return fail(ctx, GD_E_ARG, "NULL argument");
    int r = set_device(ctx);
    if (r) return r;
    unsigned long long h = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&h, ctx->d_u64, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "gd_get_stats");
    *floor_hits = h;
    return GD_OK;
}

int gd_reset_stats(gd_ctx *ctx)
{
    if (!ctx) return fail(ctx, GD_E_ARG, "NULL ctx");
    int r = set_device(ctx);
    if (r) return r;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemset(ctx->d_u64, 0, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "gd_reset_stats");
    return GD_OK;
}

}  // extern "C"

namespace {

int ensure_ppm_scratch(gd_ctx *ctx, size_t need, hipStream_t s)
{
    return ensure_scratch(ctx, ctx->ppm_s, need, s, "PPM");
}

int step_impl(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
              const void *u_in, void *u_out, void *bflux, double gamma, double dx, double dt,
              const double *dt_dev, double cfl, double *dt_next, void *hip_stream)
{
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    const bool periodic = opts->bc == GD_PERIODIC;
    if ((r = check_extents(ctx, nx, ny, nz, ng, periodic))) return r;
    if ((r = check_scalars(ctx, gamma, dx, dt_dev ? 0.0 : dt))) return r;
    if (!u_in || !u_out) return fail(ctx, GD_E_ARG, "u_in and u_out must not be NULL");
    const size_t es = elem_size(opts);
    const size_t nin = (size_t)in_elems(nx, ny, nz, ng, periodic) * es;
    const size_t nout = 5ull * nx * ny * nz * es;
    const size_t nfl = (size_t)flux_elems(nx, ny, nz) * es;
    if (overlap(u_in, nin, u_out, nout)) return fail(ctx, GD_E_ARG, "u_out overlaps u_in");
    if (bflux && (overlap(bflux, nfl, u_in, nin) || overlap(bflux, nfl, u_out, nout)))
        return fail(ctx, GD_E_ARG, "bflux overlaps u_in or u_out");
    if (dt_next && !(cfl > 0.0)) return fail(ctx, GD_E_ARG, "cfl must be > 0");
    if (dt_next && (overlap(dt_next, 8, u_in, nin) || overlap(dt_next, 8, u_out, nout)))
        return fail(ctx, GD_E_ARG, "dt_next overlaps a state array");
    if (is_ppm(opts) && !periodic && ng < 3)
        return fail(ctx, GD_E_ARG, "the PPM step needs ng >= 3 in ghosted mode (got %d)", ng);
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if ((r = set_device(ctx))) return r;

    gd::PatchDesc P{};
    P.nx = nx; P.ny = ny; P.nz = nz; P.ng = periodic ? 0 : ng; P.periodic = periodic;
    P.in_off = 0; P.out_off = 0; P.flux_off = bflux ? 0 : -1;
    P.dx = dx; P.dt = dt;
    gd::Scalars sc{ gamma, opts->rho_floor, opts->p_floor };
    hipStream_t s = (hipStream_t)hip_stream;
    const Slot slot = slot_for(ctx, s);
    if (is_ppm(opts) && (!periodic || std::min(nx, std::min(ny, nz)) >= 2)) {
        // the PPM step of one patch: one fused launch, no scratch (its
        // stencils reach three cells past a tile, which two wraps of a
        // periodic coordinate cover only for extents of 2 and more)
        gd::CflOut co{ cfl, dt_next, slot.u64 + 2, slot.u32 + 3 };
        int e = gd::launch_ppm_tile(opts->dtype, opts->limiter, opts->riemann, P, u_in, u_out, bflux,
                                    dt_dev, sc, ctx->d_u64, 2 * ctx->num_cus, co, s);
        if (!e && dt_next) e = gd::launch_cfl_finalize(cfl, dt_next, co.smax_bits, s);
        if (e) return hip_fail(ctx, e, "PPM step launch");
        return GD_OK;
    }
    if (is_ppm(opts)) {
        if ((r = ensure_ppm_scratch(ctx, (size_t)gd::ppm_box_cells(P) * 30 * es, s))) return r;
        int e = gd::launch_ppm(opts->dtype, opts->limiter, opts->riemann, P, u_in, u_out, bflux,
                               ctx->ppm_s.p, dt_dev, sc, ctx->d_u64, s);
        if (e) return hip_fail(ctx, e, "PPM step launch");
        if (dt_next) {
            // the CFL step of the new state, reduced over u_out
            gd::PatchDesc Po = P;
            Po.periodic = 1; Po.ng = 0;
            e = gd::launch_cfl_single(opts->dtype, Po, u_out, sc, cfl, dt_next, slot.u64 + 2,
                                      slot.u32 + 3, s);
            if (e) return hip_fail(ctx, e, "PPM step CFL launch");
        }
        return GD_OK;
    }
    gd::CflOut co{ cfl, dt_next, slot.u64 + 2, slot.u32 + 3 };
    // the workgroups the chip holds at once: fewer leave CUs idle
    const int shape = ctx->shape_single[opts->dtype];
    const int per_cu = gd::max_resident_blocks(opts->dtype, opts->limiter, opts->riemann, shape,
                                               ctx->device);
    int e = gd::launch_step(opts->dtype, opts->limiter, opts->riemann, shape, P, u_in, u_out,
                            bflux, dt_dev, sc, ctx->d_u64, ctx->zlen_single[opts->dtype],
                            per_cu * ctx->num_cus, co, s);
    if (e) return hip_fail(ctx, e, "godunov_step launch");
    return GD_OK;
}

int step_batched_impl(gd_ctx *ctx, const gd_opts *opts, int npatch, const gd_patch *patches,
                      const void *u_in_base, void *u_out_base, void *bflux_base,
                      const double *dt_dev, double gamma, double cfl, double *dt_next,
                      void *hip_stream)
{
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    if (opts->bc != GD_GHOSTED) return fail(ctx, GD_E_UNSUPPORTED, "batched calls take ghosted patches only");
    if ((r = validate_patches(ctx, npatch, patches, false))) return r;
    if (!(gamma > 1.0)) return fail(ctx, GD_E_ARG, "gamma must be > 1");
    if (!u_in_base || !u_out_base) return fail(ctx, GD_E_ARG, "u_in_base and u_out_base must not be NULL");
    // extents of the three buffers, for the overlap check
    int64_t in_end = 0, out_end = 0, fl_end = 0;
    for (int i = 0; i < npatch; ++i) {
        const gd_patch &p = patches[i];
        in_end = std::max<int64_t>(in_end, p.u_in_off + in_elems(p.nx, p.ny, p.nz, p.ng, false));
        out_end = std::max<int64_t>(out_end, p.u_out_off + (int64_t)5 * p.nx * p.ny * p.nz);
        if (bflux_base && p.flux_off >= 0) fl_end = std::max<int64_t>(fl_end, p.flux_off + flux_elems(p.nx, p.ny, p.nz));
    }
    const size_t es = elem_size(opts);
    if (overlap(u_in_base, in_end * es, u_out_base, out_end * es))
        return fail(ctx, GD_E_ARG, "u_out_base range overlaps u_in_base range");
    if (bflux_base && fl_end > 0 && (overlap(bflux_base, fl_end * es, u_in_base, in_end * es) ||
                                     overlap(bflux_base, fl_end * es, u_out_base, out_end * es)))
        return fail(ctx, GD_E_ARG, "bflux range overlaps u_in or u_out");
    if (dt_next && !(cfl > 0.0)) return fail(ctx, GD_E_ARG, "cfl must be > 0");
    if (dt_next && (overlap(dt_next, 8, u_in_base, in_end * es) ||
                    overlap(dt_next, 8, u_out_base, out_end * es)))
        return fail(ctx, GD_E_ARG, "dt_next overlaps a state array");
    if (is_ppm(opts))
        for (int i = 0; i < npatch; ++i)
            if (patches[i].ng < 3)
                return fail(ctx, GD_E_ARG, "patch %d: the PPM step needs ng >= 3 (got %d)", i,
                            patches[i].ng);
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if ((r = set_device(ctx))) return r;
    hipStream_t s = (hipStream_t)hip_stream;
    const Slot slot = slot_for(ctx, s);
    if (is_ppm(opts)) {
        // the PPM step of a batch: one persistent launch of the single-patch
        // march over 24x8 tiles, with the fused CFL reduction
        if ((r = build_step_tables(ctx, opts->dtype, gd::TILE_24x8, 3, npatch, patches, s,
                                   &ctx->ppm_batch)))
            return r;
        const BatchCache &c = ctx->ppm_batch;
        gd::Scalars sc{ gamma, opts->rho_floor, opts->p_floor };
        gd::CflOut co{ cfl, dt_next, slot.u64 + 2, slot.u32 + 3 };
        int e = gd::launch_ppm_batched(opts->dtype, opts->limiter, opts->riemann, c.d_patches,
                                       c.d_items, c.nitems, u_in_base, u_out_base, bflux_base, dt_dev,
                                       sc, ctx->d_u64, slot.u32, ctx->num_cus, co, s);
        if (!e && dt_next) e = gd::launch_cfl_finalize(cfl, dt_next, co.smax_bits, s);
        if (e) return hip_fail(ctx, e, "PPM batched step launch");
        return GD_OK;
    }
    if ((r = build_step_tables(ctx, opts->dtype, ctx->shape_batched[opts->dtype],
                               ctx->zpolicy_batched[opts->dtype], npatch, patches, s)))
        return r;
    const BatchCache &c = ctx->batch;
    int per_cu = gd::max_resident_blocks(opts->dtype, opts->limiter, opts->riemann, c.shape, ctx->device);
    int grid = std::min(c.nitems, per_cu * ctx->num_cus);
    gd::Scalars sc{ gamma, opts->rho_floor, opts->p_floor };
    gd::CflOut co{ cfl, dt_next, slot.u64 + 2, slot.u32 + 3 };
    int e = gd::launch_step_batched(opts->dtype, opts->limiter, opts->riemann, c.shape, c.d_patches,
                                    c.d_items, c.nitems, u_in_base, u_out_base, bflux_base, dt_dev,
                                    sc, ctx->d_u64, slot.u32, std::max(grid, 1), co, s);
    if (e) return hip_fail(ctx, e, "godunov_step_batched launch");
    return GD_OK;
}

}  // namespace

extern "C" {

int godunov_step(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
                 const void *u_in, void *u_out, void *bflux, double gamma, double dx, double dt,
                 const double *dt_dev, void *hip_stream)
{
    return step_impl(ctx, opts, nx, ny, nz, ng, u_in, u_out, bflux, gamma, dx, dt, dt_dev, 0.0,
                     nullptr, hip_stream);
}

int godunov_step_cfl(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
                     const void *u_in, void *u_out, void *bflux, double gamma, double dx,
                     double dt, const double *dt_dev, double cfl, double *dt_next_dev,
                     void *hip_stream)
{
    if (!dt_next_dev) return fail(ctx, GD_E_ARG, "dt_next_dev must not be NULL");
    return step_impl(ctx, opts, nx, ny, nz, ng, u_in, u_out, bflux, gamma, dx, dt, dt_dev, cfl,
                     dt_next_dev, hip_stream);
}

int godunov_step_batched(gd_ctx *ctx, const gd_opts *opts, int npatch, const gd_patch *patches,
                         const void *u_in_base, void *u_out_base, void *bflux_base,
                         const double *dt_dev, double gamma, void *hip_stream)
{
    return step_batched_impl(ctx, opts, npatch, patches, u_in_base, u_out_base, bflux_base, dt_dev,
                             gamma, 0.0, nullptr, hip_stream);
}

int godunov_step_batched_cfl(gd_ctx *ctx, const gd_opts *opts, int npatch,
                             const gd_patch *patches, const void *u_in_base, void *u_out_base,
                             void *bflux_base, const double *dt_dev, double gamma, double cfl,
                             double *dt_next_dev, void *hip_stream)
{
    if (!dt_next_dev) return fail(ctx, GD_E_ARG, "dt_next_dev must not be NULL");
    return step_batched_impl(ctx, opts, npatch, patches, u_in_base, u_out_base, bflux_base, dt_dev,
                             gamma, cfl, dt_next_dev, hip_stream);
}

int cfl_dt(gd_ctx *ctx, const gd_opts *opts, int npatch, const gd_patch *patches,
           const void *u_base, double gamma, double cfl, double *dt_dev, void *hip_stream)
{
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    const bool periodic = opts->bc == GD_PERIODIC;
    if ((r = validate_patches(ctx, npatch, patches, periodic))) return r;
    if (!(gamma > 1.0)) return fail(ctx, GD_E_ARG, "gamma must be > 1");
    if (!(cfl > 0.0)) return fail(ctx, GD_E_ARG, "cfl must be > 0");
    if (!u_base || !dt_dev) return fail(ctx, GD_E_ARG, "u_base and dt_dev must not be NULL");
    if (periodic && npatch != 1) return fail(ctx, GD_E_ARG, "periodic mode takes exactly one patch");
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if ((r = set_device(ctx))) return r;
    hipStream_t s = (hipStream_t)hip_stream;
    const Slot slot = slot_for(ctx, s);
    gd::Scalars sc{ gamma, opts->rho_floor, opts->p_floor };
    int e;
    if (npatch == 1) {
        gd::PatchDesc P = to_desc(patches[0], periodic);
        e = gd::launch_cfl_single(opts->dtype, P, u_base, sc, cfl, dt_dev, slot.u64 + 1,
                                  slot.u32 + 2, s);
    } else {
        if ((r = build_cfl_tables(ctx, periodic, npatch, patches, s))) return r;
        const BatchCache &c = ctx->cfl;
        int grid = std::min(c.ncfl, 8 * ctx->num_cus);
        e = gd::launch_cfl(opts->dtype, c.d_patches, c.d_cfl_items, c.ncfl, u_base, sc, cfl, dt_dev,
                           slot.u64 + 1, slot.u32 + 2, std::max(grid, 1), s);
    }
    if (e) return hip_fail(ctx, e, "cfl_dt launch");
    return GD_OK;
}

int godunov_step_adjoint(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
                         const void *u_in, const void *lam_out, const void *lam_bflux,
                         void *lam_in, double gamma, double dx, double dt, void *hip_stream)
{
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    if ((r = reject_ppm(ctx, opts, "the adjoint"))) return r;
    if (opts->dtype != GD_F64) return fail(ctx, GD_E_UNSUPPORTED, "the adjoint is FP64 only");
    const bool periodic = opts->bc == GD_PERIODIC;
    if ((r = check_extents(ctx, nx, ny, nz, ng, periodic))) return r;
    if ((r = check_scalars(ctx, gamma, dx, dt))) return r;
    if (!u_in || !lam_out || !lam_in) return fail(ctx, GD_E_ARG, "u_in, lam_out and lam_in must not be NULL");
    const size_t nin = (size_t)in_elems(nx, ny, nz, ng, periodic) * 8;
    const size_t nout = 5ull * nx * ny * nz * 8;
    const size_t nfl = (size_t)flux_elems(nx, ny, nz) * 8;
    if (overlap(lam_in, nin, u_in, nin) || overlap(lam_in, nin, lam_out, nout) ||
        (lam_bflux && overlap(lam_in, nin, lam_bflux, nfl)))
        return fail(ctx, GD_E_ARG, "lam_in overlaps an input");
    gd::PatchDesc P{};
    P.nx = nx; P.ny = ny; P.nz = nz; P.ng = periodic ? 0 : ng; P.periodic = periodic;
    P.flux_off = lam_bflux ? 0 : -1;
    P.dx = dx; P.dt = dt;
    if (!gd::adjoint_fits_32bit(P))
        return fail(ctx, GD_E_UNSUPPORTED, "the adjoint supports boxes of up to 2^31/15 extended cells");
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if ((r = set_device(ctx))) return r;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t need = gd::adjoint_scratch_bytes(P);
    if ((r = ensure_scratch(ctx, ctx->adj, need, s, "adjoint"))) return r;
    gd::Scalars sc{ gamma, opts->rho_floor, opts->p_floor };
    int e = gd::launch_adjoint(opts->limiter, opts->riemann, P, (const double *)u_in,
                               (const double *)lam_out, (const double *)lam_bflux, (double *)lam_in,
                               sc, dt, (double *)ctx->adj.p, s);
    if (e) return hip_fail(ctx, e, "godunov_step_adjoint launch");
    return GD_OK;
}

}  // extern "C"

// ------------------------------------------------------------ autotuning

namespace {

// Mean time in ms of `reps` calls of fn() on stream s after one warm-up.
template <typename Fn>
int time_calls(gd_ctx *ctx, hipStream_t s, int reps, Fn fn, float *ms)
{
    int r = fn();
    if (r) return r;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return fail(ctx, GD_E_HIP, "hipEventCreate");
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(ctx, GD_E_HIP, "hipEventCreate");
    }
    hipError_t e = hipEventRecord(a, s);
    for (int i = 0; i < reps && e == hipSuccess && r == GD_OK; ++i) r = fn();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (r) return r;
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune timing");
    *ms = t / reps;
    return GD_OK;
}

}  // namespace

extern "C" {

int gd_autotune_step(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
                     const void *u_in, void *u_out, double gamma, double dx, double dt,
                     void *hip_stream, int *choice)
{
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    if ((r = reject_ppm(ctx, opts, "the autotuner"))) return r;
    if (capturing((hipStream_t)hip_stream))
        return fail(ctx, GD_E_UNSUPPORTED, "the autotuner waits on the host and cannot be captured");
    const int dt_i = opts->dtype;
    const int shapes[5] = { gd::TILE_16x16, gd::TILE_32x8, gd::TILE_8x8, gd::TILE_16x8,
                            gd::TILE_24x8 };
    const int zlens[3] = { 16, 32, 64 };
    const int keep_shape = ctx->shape_single[dt_i], keep_zlen = ctx->zlen_single[dt_i];
    // the first pass runs every candidate once (clocks and caches settle);
    // the next two time each candidate over 4 calls; a candidate's time is its
    // best pass, so a transient slowdown does not decide the choice
    float best_ms[15];
    for (float &m : best_ms) m = 1e30f;
    for (int round = 0; round < 3; ++round)
        for (int c = 0; c < 15; ++c) {
            ctx->shape_single[dt_i] = shapes[c / 3];
            ctx->zlen_single[dt_i] = zlens[c % 3];
            float ms = 0.f;
            r = time_calls(ctx, (hipStream_t)hip_stream, round == 0 ? 1 : 4, [&] {
                return godunov_step(ctx, opts, nx, ny, nz, ng, u_in, u_out, nullptr, gamma, dx,
                                    dt, nullptr, hip_stream);
            }, &ms);
            if (r) {
                ctx->shape_single[dt_i] = keep_shape;
                ctx->zlen_single[dt_i] = keep_zlen;
                return r;
            }
            if (round > 0) best_ms[c] = std::min(best_ms[c], ms);
        }
    int best_i = 0;
    for (int c = 1; c < 15; ++c)
        if (best_ms[c] < best_ms[best_i]) best_i = c;
    ctx->shape_single[dt_i] = shapes[best_i / 3];
    ctx->zlen_single[dt_i] = zlens[best_i % 3];
    if (choice) *choice = best_i;
    return GD_OK;
}

int gd_autotune_batched(gd_ctx *ctx, const gd_opts *opts, int npatch, const gd_patch *patches,
                        const void *u_in_base, void *u_out_base, void *bflux_base, double gamma,
                        void *hip_stream, int *choice)
{
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    if ((r = reject_ppm(ctx, opts, "the autotuner"))) return r;
    if (capturing((hipStream_t)hip_stream))
        return fail(ctx, GD_E_UNSUPPORTED, "the autotuner waits on the host and cannot be captured");
    const int dt_i = opts->dtype;
    const int shapes[6] = { gd::TILE_16x16, gd::TILE_32x8, gd::TILE_8x8, gd::TILE_16x8,
                            gd::TILE_24x8, gd::TILE_PAIR_24x8 };
    const int keep_shape = ctx->shape_batched[dt_i], keep_pol = ctx->zpolicy_batched[dt_i];
    // the same protocol as gd_autotune_step: a warm-up round, then the best
    // of two timed rounds per candidate
    float best_ms[18];
    for (float &m : best_ms) m = 1e30f;
    for (int round = 0; round < 3; ++round)
        for (int c = 0; c < 18; ++c) {
            ctx->shape_batched[dt_i] = shapes[c / 3];
            ctx->zpolicy_batched[dt_i] = c % 3;
            float ms = 0.f;
            r = time_calls(ctx, (hipStream_t)hip_stream, round == 0 ? 1 : 3, [&] {
                return godunov_step_batched(ctx, opts, npatch, patches, u_in_base, u_out_base,
                                            bflux_base, nullptr, gamma, hip_stream);
            }, &ms);
            if (r) {
                ctx->shape_batched[dt_i] = keep_shape;
                ctx->zpolicy_batched[dt_i] = keep_pol;
                return r;
            }
            if (round > 0) best_ms[c] = std::min(best_ms[c], ms);
        }
    int best_i = 0;
    for (int c = 1; c < 18; ++c)
        if (best_ms[c] < best_ms[best_i]) best_i = c;
    ctx->shape_batched[dt_i] = shapes[best_i / 3];
    ctx->zpolicy_batched[dt_i] = best_i % 3;
    if (choice) *choice = best_i;
    return GD_OK;
}

int gd_get_config(gd_ctx *ctx, int dtype, int *shape_single, int *zlen_single, int *shape_batched,
                  int *zpolicy_batched)
{
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if (dtype != GD_F64 && dtype != GD_F32) return fail(ctx, GD_E_ARG, "bad dtype %d", dtype);
    if (shape_single) *shape_single = ctx->shape_single[dtype];
    if (zlen_single) *zlen_single = ctx->zlen_single[dtype];
    if (shape_batched) *shape_batched = ctx->shape_batched[dtype];
    if (zpolicy_batched) *zpolicy_batched = ctx->zpolicy_batched[dtype];
    return GD_OK;
}

int gd_set_config(gd_ctx *ctx, int dtype, int shape_single, int zlen_single, int shape_batched,
                  int zpolicy_batched)
{
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if (dtype != GD_F64 && dtype != GD_F32) return fail(ctx, GD_E_ARG, "bad dtype %d", dtype);
    if (shape_single < 0 || shape_single >= gd::NUM_TILE_SHAPES || shape_batched < 0 ||
        shape_batched >= gd::NUM_BATCHED_SHAPES)
        return fail(ctx, GD_E_ARG, "bad tile shape");
    if (zlen_single < 1 || zlen_single > 4096) return fail(ctx, GD_E_ARG, "bad z-range length");
    if (zpolicy_batched < 0 || zpolicy_batched > 2) return fail(ctx, GD_E_ARG, "bad z-range policy");
    ctx->shape_single[dtype] = shape_single;
    ctx->zlen_single[dtype] = zlen_single;
    ctx->shape_batched[dtype] = shape_batched;
    ctx->zpolicy_batched[dtype] = zpolicy_batched;
    return GD_OK;
}

}  // extern "C"

namespace {

int check_mhd(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, double gamma, double dx)
{
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    if ((r = reject_ppm(ctx, opts, "the MHD step"))) return r;
    if (opts->bc != GD_PERIODIC)
        return fail(ctx, GD_E_UNSUPPORTED, "the MHD step supports periodic boxes only");
    if (nx < 1 || ny < 1 || nz < 1) return fail(ctx, GD_E_ARG, "extents must be >= 1 (%d,%d,%d)", nx, ny, nz);
    if (nx > 65535 * 64 || ny > 65535 * 4 || nz > 65535) return fail(ctx, GD_E_ARG, "extent too large");
    // 54 face-state values per cell are addressed with 64-bit offsets, the
    // cells of the box with 32-bit ones
    if ((int64_t)nx * ny * nz * 9 > 0x7fffffffLL) return fail(ctx, GD_E_UNSUPPORTED, "box too large");
    if (!(gamma > 1.0)) return fail(ctx, GD_E_ARG, "gamma must be > 1");
    if (!(dx > 0.0)) return fail(ctx, GD_E_ARG, "dx must be > 0");
    return GD_OK;
}

}  // namespace

namespace {

int step_mhd_impl(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, const void *u_in,
                  void *u_out, double gamma, double dx, double dt, const double *dt_dev, double ch,
                  const double *ch_dev, double alpha, double cfl, double *dt_next,
                  double *ch_next, void *hip_stream)
{
    int r;
    if ((r = check_mhd(ctx, opts, nx, ny, nz, gamma, dx))) return r;
    if (!dt_dev && !(dt >= 0.0)) return fail(ctx, GD_E_ARG, "dt must be >= 0");
    if (!ch_dev && !(ch > 0.0)) return fail(ctx, GD_E_ARG, "ch must be > 0");
    if (!(alpha >= 0.0)) return fail(ctx, GD_E_ARG, "alpha must be >= 0");
    if ((dt_next || ch_next) && !(cfl > 0.0)) return fail(ctx, GD_E_ARG, "cfl must be > 0");
    if (!u_in || !u_out) return fail(ctx, GD_E_ARG, "u_in and u_out must not be NULL");
    const size_t bytes = 9ull * nx * ny * nz * elem_size(opts);
    if (overlap(u_in, bytes, u_out, bytes)) return fail(ctx, GD_E_ARG, "u_out overlaps u_in");
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if ((r = set_device(ctx))) return r;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t need = gd::mhd_scratch_bytes(opts->dtype, nx, ny, nz);
    if ((r = ensure_scratch(ctx, ctx->mhd, need, s, "MHD"))) return r;
    gd::MhdScalars sc{ gamma, opts->rho_floor, opts->p_floor, dx, dt, ch, alpha };
    int e = gd::launch_mhd_step(opts->dtype, opts->limiter, nx, ny, nz, u_in, u_out, sc, dt_dev,
                                ch_dev, ctx->mhd.p, cfl, dt_next, ch_next,
                                slot_for(ctx, s).u64 + 6, s);
    if (e) return hip_fail(ctx, e, "godunov_step_mhd launch");
    return GD_OK;
}

}  // namespace

extern "C" {

int godunov_step_mhd(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, const void *u_in,
                     void *u_out, double gamma, double dx, double dt, const double *dt_dev,
                     double ch, const double *ch_dev, double alpha, void *hip_stream)
{
    return step_mhd_impl(ctx, opts, nx, ny, nz, u_in, u_out, gamma, dx, dt, dt_dev, ch, ch_dev,
                         alpha, 0.0, nullptr, nullptr, hip_stream);
}

int godunov_step_mhd_cfl(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz,
                         const void *u_in, void *u_out, double gamma, double dx, double dt,
                         const double *dt_dev, double ch, const double *ch_dev, double alpha,
                         double cfl, double *dt_next_dev, double *ch_next_dev, void *hip_stream)
{
    if (!dt_next_dev && !ch_next_dev)
        return fail(ctx, GD_E_ARG, "dt_next_dev and ch_next_dev are both NULL");
    return step_mhd_impl(ctx, opts, nx, ny, nz, u_in, u_out, gamma, dx, dt, dt_dev, ch, ch_dev,
                         alpha, cfl, dt_next_dev, ch_next_dev, hip_stream);
}

int cfl_dt_mhd(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, const void *u,
               double gamma, double dx, double cfl, double *dt_dev, double *ch_dev,
               void *hip_stream)
{
    int r;
    if ((r = check_mhd(ctx, opts, nx, ny, nz, gamma, dx))) return r;
    if (!(cfl > 0.0)) return fail(ctx, GD_E_ARG, "cfl must be > 0");
    if (!u) return fail(ctx, GD_E_ARG, "u must not be NULL");
    if (!dt_dev && !ch_dev) return fail(ctx, GD_E_ARG, "dt_dev and ch_dev are both NULL");
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if ((r = set_device(ctx))) return r;
    gd::MhdScalars sc{ gamma, opts->rho_floor, opts->p_floor, dx, 0.0, 0.0, 0.0 };
    int e = gd::launch_mhd_speeds(opts->dtype, nx, ny, nz, u, sc, cfl, dt_dev, ch_dev,
                                  slot_for(ctx, (hipStream_t)hip_stream).u64 + 4,
                                  (hipStream_t)hip_stream);
    if (e) return hip_fail(ctx, e, "cfl_dt_mhd launch");
    return GD_OK;
}

}  // extern "C"

// ------------------------------------------------------------ two-level AMR

struct gd_amr {
    int device = 0;
    int nc[3] = { 0, 0, 0 };
    double dx = 0.0;
    std::vector<gd_patch> fine;     // descriptors of the fine batch (ng 2, dx / 2)
    int64_t in_end = 0, out_end = 0, fl_end = 0;   // fine buffer extents, elements
    void *mem = nullptr;            // one device block holding every table
    double *d_dt = nullptr;         // dt of gd_amr_step when given on the host
                                    // (the tables also hold the reflux scratch)
    gd::AmrTables t{};
};

namespace {

int64_t coarse_elems(const gd_amr *a) { return 5LL * a->nc[0] * a->nc[1] * a->nc[2]; }

int check_plan(gd_ctx *ctx, const gd_amr *plan)
{
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if (!plan) return fail(ctx, GD_E_ARG, "plan is NULL");
    if (plan->device != ctx->device)
        return fail(ctx, GD_E_ARG, "plan was built on device %d, ctx is on device %d", plan->device,
                    ctx->device);
    return GD_OK;
}

int amr_fill_impl(gd_ctx *ctx, const gd_amr *plan, int dtype, const void *coarse_u,
                  void *fine_in_base, hipStream_t s)
{
    int r;
    if ((r = check_plan(ctx, plan))) return r;
    if (dtype != GD_F64 && dtype != GD_F32) return fail(ctx, GD_E_ARG, "bad dtype %d", dtype);
    if (!coarse_u || (!fine_in_base && plan->t.nfill)) return fail(ctx, GD_E_ARG, "NULL state pointer");
    const size_t es = dtype == GD_F32 ? 4 : 8;
    if (fine_in_base && overlap(coarse_u, coarse_elems(plan) * es, fine_in_base, plan->in_end * es))
        return fail(ctx, GD_E_ARG, "fine_in_base range overlaps coarse_u");
    if ((r = set_device(ctx))) return r;
    int e = gd::launch_amr_fill(dtype, plan->t, coarse_u, fine_in_base, s);
    if (e) return hip_fail(ctx, e, "gd_amr_fill_ghosts launch");
    return GD_OK;
}

int amr_seam_impl(gd_ctx *ctx, const gd_amr *plan, const gd_opts *opts, const void *coarse_old,
                  void *coarse_new, const void *fine_out, const void *fine_flux, double gamma,
                  double dt, const double *dt_dev, hipStream_t s)
{
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    if ((r = reject_ppm(ctx, opts, "the AMR seams"))) return r;
    if ((r = check_plan(ctx, plan))) return r;
    if ((r = check_scalars(ctx, gamma, plan->dx, dt_dev ? 0.0 : dt))) return r;
    const bool fine = !plan->fine.empty();
    if (!coarse_old || !coarse_new || (fine && (!fine_out || !fine_flux)))
        return fail(ctx, GD_E_ARG, "NULL state pointer");
    const size_t es = elem_size(opts), nc = coarse_elems(plan) * es;
    if (overlap(coarse_old, nc, coarse_new, nc)) return fail(ctx, GD_E_ARG, "coarse_new overlaps coarse_old");
    if (fine && (overlap(coarse_new, nc, fine_out, plan->out_end * es) ||
                 overlap(coarse_new, nc, fine_flux, plan->fl_end * es)))
        return fail(ctx, GD_E_ARG, "coarse_new overlaps a fine buffer");
    if ((r = set_device(ctx))) return r;
    gd::Scalars sc{ gamma, opts->rho_floor, opts->p_floor };
    int e = gd::launch_amr_seam(opts->dtype, opts->limiter, opts->riemann, plan->t, coarse_old,
                                coarse_new, fine_out, fine_flux, sc, plan->dx, dt, dt_dev, s);
    if (e) return hip_fail(ctx, e, "gd_amr_reflux launch");
    return GD_OK;
}

// Device block layout: each table at a 256-byte aligned offset.
struct Block {
    size_t size = 0;
    size_t add(size_t bytes)
    {
        size_t at = size;
        size += (bytes + 255) / 256 * 256;
        return at;
    }
};

}  // namespace

extern "C" {

int gd_amr_create(gd_ctx *ctx, int ncx, int ncy, int ncz, double dx_coarse, int npatch,
                  const gd_amr_patch *patches, gd_amr **plan)
{
    if (!plan) return fail(ctx, GD_E_ARG, "plan pointer is NULL");
    *plan = nullptr;
    const int nc[3] = { ncx, ncy, ncz };
    for (int a = 0; a < 3; ++a)
        if (nc[a] < 1 || nc[a] > 8192) return fail(ctx, GD_E_ARG, "coarse extents must be in [1, 8192]");
    const int64_t ncell = (int64_t)ncx * ncy * ncz;
    if (ncell >= 0x7fffffffLL) return fail(ctx, GD_E_ARG, "coarse box has 2^31 cells or more");
    if (!(dx_coarse > 0.0)) return fail(ctx, GD_E_ARG, "dx_coarse must be > 0");
    if (npatch < 0 || (npatch > 0 && !patches)) return fail(ctx, GD_E_ARG, "bad patch list");

    std::vector<int32_t> owner(ncell, -1);
    auto cidx = [&](int x, int y, int z) { return ((int64_t)z * ncy + y) * ncx + x; };
    std::vector<gd::AmrPatch> dp(npatch);
    std::vector<gd_patch> fine(npatch);
    int64_t in_end = 0, out_end = 0, fl_end = 0;
    for (int p = 0; p < npatch; ++p) {
        const gd_amr_patch &P = patches[p];
        for (int a = 0; a < 3; ++a) {
            if (P.n[a] < 2 || P.n[a] % 2) return fail(ctx, GD_E_ARG, "patch %d: extents must be even and >= 2", p);
            if (P.lo[a] < 0 || P.lo[a] + P.n[a] / 2 > nc[a])
                return fail(ctx, GD_E_ARG, "patch %d: not inside the coarse box", p);
        }
        if (P.u_in_off < 0 || P.u_out_off < 0 || P.flux_off < 0)
            return fail(ctx, GD_E_ARG, "patch %d: negative offset", p);
        if ((int64_t)(P.n[0] + 4) * (P.n[1] + 4) * (P.n[2] + 4) >= 0x7fffffffLL)
            return fail(ctx, GD_E_ARG, "patch %d: too large", p);
        for (int z = P.lo[2]; z < P.lo[2] + P.n[2] / 2; ++z)
            for (int y = P.lo[1]; y < P.lo[1] + P.n[1] / 2; ++y)
                for (int x = P.lo[0]; x < P.lo[0] + P.n[0] / 2; ++x) {
                    int32_t &o = owner[cidx(x, y, z)];
                    if (o >= 0) return fail(ctx, GD_E_ARG, "patches %d and %d overlap", o, p);
                    o = p;
                }
        gd::AmrPatch &d = dp[p];
        for (int a = 0; a < 3; ++a) { d.lo[a] = P.lo[a]; d.n[a] = P.n[a]; }
        d.in_off = P.u_in_off; d.out_off = P.u_out_off; d.flux_off = P.flux_off;
        gd_patch &f = fine[p];
        f.nx = P.n[0]; f.ny = P.n[1]; f.nz = P.n[2]; f.ng = 2;
        f.u_in_off = P.u_in_off; f.u_out_off = P.u_out_off; f.flux_off = P.flux_off;
        f.dx = dx_coarse / 2; f.dt = 0.0;
        in_end = std::max<int64_t>(in_end, P.u_in_off + in_elems(P.n[0], P.n[1], P.n[2], 2, false));
        out_end = std::max<int64_t>(out_end, P.u_out_off + 5LL * P.n[0] * P.n[1] * P.n[2]);
        fl_end = std::max<int64_t>(fl_end, P.flux_off + flux_elems(P.n[0], P.n[1], P.n[2]));
    }

    // ghost fill: 256-cell pieces of each patch's one-coarse-cell shell box
    std::vector<gd::AmrFillItem> fill;
    for (int p = 0; p < npatch; ++p) {
        const int box = (dp[p].n[0] / 2 + 2) * (dp[p].n[1] / 2 + 2) * (dp[p].n[2] / 2 + 2);
        for (int s0 = 0; s0 < box; s0 += 256) fill.push_back(gd::AmrFillItem{ p, s0 });
    }
    // interface faces, per patch, axis, side and footprint cell; grouped by
    // the uncovered cell they correct, in that order
    std::vector<int32_t> cells;
    std::vector<std::vector<gd::AmrFace>> per_cell;
    std::vector<int32_t> slot(ncell, -1);
    for (int p = 0; p < npatch; ++p) {
        const gd::AmrPatch &P = dp[p];
        const int size[3] = { P.n[0] / 2, P.n[1] / 2, P.n[2] / 2 };
        const int64_t sx = 5LL * P.n[2] * P.n[1], sy = 5LL * P.n[2] * P.n[0], sz = 5LL * P.n[1] * P.n[0];
        const int64_t sheet0[6] = { 0, sx, 2 * sx, 2 * sx + sy, 2 * sx + 2 * sy, 2 * sx + 2 * sy + sz };
        for (int d = 0; d < 3; ++d) {
            const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
            for (int side = 0; side < 2; ++side)
                for (int b = 0; b < size[t2]; ++b)
                    for (int a = 0; a < size[t1]; ++a) {
                        int c[3] = { P.lo[0], P.lo[1], P.lo[2] };
                        c[t1] += a;
                        c[t2] += b;
                        c[d] = P.lo[d] + (side ? size[d] - 1 : 0);
                        int o[3] = { c[0], c[1], c[2] };
                        o[d] = (c[d] + (side ? 1 : -1) + nc[d]) % nc[d];
                        const int64_t oi = cidx(o[0], o[1], o[2]);
                        if (owner[oi] >= 0) continue;
                        gd::AmrFace f{};
                        const int *rc = side ? o : c;
                        f.right = (int32_t)cidx(rc[0], rc[1], rc[2]);
                        f.dside = 2 * d + side;
                        // sheet axes (slow, fast): x (z, y), y (z, x), z (y, x)
                        const int slow = d == 2 ? 1 : 2, fast = d == 0 ? 1 : 0;
                        const int ls = 2 * (c[slow] - P.lo[slow]), lf = 2 * (c[fast] - P.lo[fast]);
                        f.row = P.n[fast];
                        f.vstride = (int32_t)((d == 0 ? sx : (d == 1 ? sy : sz)) / 5);
                        f.fine = P.flux_off + sheet0[2 * d + side] + (int64_t)ls * f.row + lf;
                        if (slot[oi] < 0) {
                            slot[oi] = (int32_t)cells.size();
                            cells.push_back((int32_t)oi);
                            per_cell.emplace_back();
                        }
                        per_cell[slot[oi]].push_back(f);
                    }
        }
    }
    std::vector<int32_t> start(1, 0);
    std::vector<gd::AmrFace> faces;
    for (auto &v : per_cell) {
        faces.insert(faces.end(), v.begin(), v.end());
        start.push_back((int32_t)faces.size());
    }
    std::vector<gd::AmrCover> cover;
    for (int p = 0; p < npatch; ++p) {
        const gd::AmrPatch &P = dp[p];
        for (int k = 0; k < P.n[2] / 2; ++k)
            for (int j = 0; j < P.n[1] / 2; ++j)
                for (int i = 0; i < P.n[0] / 2; ++i) {
                    gd::AmrCover c{};
                    c.coarse = (int32_t)cidx(P.lo[0] + i, P.lo[1] + j, P.lo[2] + k);
                    c.patch = p;
                    c.child = P.out_off + ((int64_t)2 * k * P.n[1] + 2 * j) * P.n[0] + 2 * i;
                    cover.push_back(c);
                }
    }
    if (fill.size() > 0x7fffffff / 2 || cells.size() + cover.size() > 0x7fffffff / 2 ||
        faces.size() > 0x7fffffff / 4)
        return fail(ctx, GD_E_ARG, "hierarchy too large");

    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    int r;
    if ((r = set_device(ctx))) return r;
    Block blk;
    const size_t o_owner = blk.add(owner.size() * 4), o_patch = blk.add(dp.size() * sizeof(gd::AmrPatch));
    const size_t o_fill = blk.add(fill.size() * sizeof(gd::AmrFillItem));
    const size_t o_cells = blk.add(cells.size() * 4), o_start = blk.add(start.size() * 4);
    const size_t o_faces = blk.add(faces.size() * sizeof(gd::AmrFace));
    const size_t o_cover = blk.add(cover.size() * sizeof(gd::AmrCover));
    const size_t o_dt = blk.add(sizeof(double));
    const size_t o_fs = blk.add(faces.size() * 10 * sizeof(double));
    gd_amr *a = new gd_amr();
    a->device = ctx->device;
    for (int k = 0; k < 3; ++k) a->nc[k] = nc[k];
    a->dx = dx_coarse;
    a->fine = fine;
    a->in_end = in_end; a->out_end = out_end; a->fl_end = fl_end;
    hipError_t e = hipMalloc(&a->mem, blk.size);
    if (e != hipSuccess) {
        delete a;
        return fail(ctx, GD_E_NOMEM, "hipMalloc of %zu bytes for the AMR tables failed", blk.size);
    }
    char *base = (char *)a->mem;
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(base + off, src, bytes, hipMemcpyHostToDevice);
    };
    put(o_owner, owner.data(), owner.size() * 4);
    put(o_patch, dp.data(), dp.size() * sizeof(gd::AmrPatch));
    put(o_fill, fill.data(), fill.size() * sizeof(gd::AmrFillItem));
    put(o_cells, cells.data(), cells.size() * 4);
    put(o_start, start.data(), start.size() * 4);
    put(o_faces, faces.data(), faces.size() * sizeof(gd::AmrFace));
    put(o_cover, cover.data(), cover.size() * sizeof(gd::AmrCover));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(a->mem);
        delete a;
        return hip_fail(ctx, e, "upload of the AMR tables");
    }
    gd::AmrTables &t = a->t;
    for (int k = 0; k < 3; ++k) t.nc[k] = nc[k];
    t.nfill = (int32_t)fill.size();
    t.ncells = (int32_t)cells.size();
    t.ncover = (int32_t)cover.size();
    t.nfaces = (int32_t)faces.size();
    t.owner = (const int32_t *)(base + o_owner);
    t.patches = (const gd::AmrPatch *)(base + o_patch);
    t.fill = (const gd::AmrFillItem *)(base + o_fill);
    t.cells = (const int32_t *)(base + o_cells);
    t.cell_start = (const int32_t *)(base + o_start);
    t.faces = (const gd::AmrFace *)(base + o_faces);
    t.cover = (const gd::AmrCover *)(base + o_cover);
    a->d_dt = (double *)(base + o_dt);
    t.fstate = base + o_fs;
    *plan = a;
    return GD_OK;
}

int gd_amr_destroy(gd_amr *plan)
{
    if (!plan) return GD_OK;
    (void)hipSetDevice(plan->device);
    if (plan->mem) (void)hipFree(plan->mem);
    delete plan;
    return GD_OK;
}

int gd_amr_fill_ghosts(gd_ctx *ctx, const gd_amr *plan, int dtype, const void *coarse_u,
                       void *fine_in_base, void *hip_stream)
{
    return amr_fill_impl(ctx, plan, dtype, coarse_u, fine_in_base, (hipStream_t)hip_stream);
}

int gd_amr_reflux(gd_ctx *ctx, const gd_amr *plan, const gd_opts *opts, const void *coarse_old,
                  void *coarse_new, const void *fine_out_base, const void *fine_flux_base,
                  double gamma, double dt, const double *dt_dev, void *hip_stream)
{
    return amr_seam_impl(ctx, plan, opts, coarse_old, coarse_new, fine_out_base, fine_flux_base,
                         gamma, dt, dt_dev, (hipStream_t)hip_stream);
}

int gd_amr_step(gd_ctx *ctx, const gd_amr *plan, const gd_opts *opts, const void *coarse_in,
                void *coarse_out, void *fine_in_base, void *fine_out_base, void *fine_flux_base,
                double gamma, double dt, const double *dt_dev, void *hip_stream)
{
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    if ((r = reject_ppm(ctx, opts, "the AMR seams"))) return r;
    if ((r = check_plan(ctx, plan))) return r;
    if ((r = check_scalars(ctx, gamma, plan->dx, dt_dev ? 0.0 : dt))) return r;
    const bool fine = !plan->fine.empty();
    if (!coarse_in || !coarse_out || (fine && (!fine_in_base || !fine_out_base || !fine_flux_base)))
        return fail(ctx, GD_E_ARG, "NULL state pointer");
    const size_t es = elem_size(opts), nc = coarse_elems(plan) * es;
    if (fine && (overlap(coarse_in, nc, fine_in_base, plan->in_end * es) ||
                 overlap(coarse_out, nc, fine_in_base, plan->in_end * es)))
        return fail(ctx, GD_E_ARG, "fine_in_base overlaps a coarse buffer");
    if ((r = set_device(ctx))) return r;
    hipStream_t s = (hipStream_t)hip_stream;
    const double *dtp = dt_dev;
    if (!dtp) {
        int e = gd::launch_set_scalar(plan->d_dt, dt, s);
        if (e) return hip_fail(ctx, e, "gd_amr_step dt store");
        dtp = plan->d_dt;
    }
    gd_opts o = *opts;
    if (fine && (r = amr_fill_impl(ctx, plan, o.dtype, coarse_in, fine_in_base, s))) return r;
    o.bc = GD_PERIODIC;
    if ((r = step_impl(ctx, &o, plan->nc[0], plan->nc[1], plan->nc[2], 0, coarse_in, coarse_out,
                       nullptr, gamma, plan->dx, 0.0, dtp, 0.0, nullptr, s)))
        return r;
    o.bc = GD_GHOSTED;
    if (fine && (r = step_batched_impl(ctx, &o, (int)plan->fine.size(), plan->fine.data(),
                                       fine_in_base, fine_out_base, fine_flux_base, dtp, gamma,
                                       0.0, nullptr, s)))
        return r;
    return amr_seam_impl(ctx, plan, &o, coarse_in, coarse_out, fine_out_base, fine_flux_base,
                         gamma, 0.0, dtp, s);
}

}  // extern "C"


// ------------------------------------------------------------ streamed batches

namespace {

// One contiguous host <-> staging copy, in elements.
struct CopyRun {
    int64_t host, staging, elems;
};

struct StreamChunk {
    int patch0, npatch;                 // range in the plan's descriptor table
    int item0, nitems;                  // range in the plan's work items
    int64_t in_elems, out_elems, fl_elems;
    std::vector<CopyRun> in, out, flux;
};

}  // namespace

// Staging slots of the streamed pipeline: chunk c uses slot c mod NSTAGE, so
// the copy in of a chunk waits only for the step NSTAGE chunks back, and the
// step for that chunk's copy out.
constexpr int NSTAGE = 3;

// The plan of a streamed batch: chunks of patches that fit one staging slot,
// the device descriptors and work items of every chunk (offsets relative to
// the slot), and the pipeline's streams, events and staging memory.
struct gd_stream_state {
    std::vector<gd_patch> host;         // descriptors the plan was built from
    int dtype = -1, shape = -1, zpolicy = -1, has_flux = -1;
    size_t chunk_bytes = 0;
    std::vector<StreamChunk> chunks;
    int64_t in_max = 0, out_max = 0, fl_max = 0;        // slot regions, elements
    gd::PatchDesc *d_patches = nullptr;
    gd::WorkItem *d_items = nullptr;
    size_t cap_patches = 0, cap_items = 0;
    void *staging = nullptr;            // NSTAGE slots of in_max + out_max + fl_max elements
    size_t staging_bytes = 0;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    hipEvent_t ev_in[NSTAGE] = {}, ev_comp[NSTAGE] = {}, ev_out[NSTAGE] = {};
    hipEvent_t ev_start = nullptr;       // the caller's stream at the call
    bool streams = false;
};

static void free_stream_state(gd_stream_state *st)
{
    if (!st) return;
    if (st->d_patches) (void)hipFree(st->d_patches);
    if (st->d_items) (void)hipFree(st->d_items);
    if (st->staging) (void)hipFree(st->staging);
    if (st->streams) {
        for (int b = 0; b < NSTAGE; ++b) {
            (void)hipEventDestroy(st->ev_in[b]);
            (void)hipEventDestroy(st->ev_comp[b]);
            (void)hipEventDestroy(st->ev_out[b]);
        }
        (void)hipEventDestroy(st->ev_start);
        (void)hipStreamDestroy(st->s_in);
        (void)hipStreamDestroy(st->s_comp);
        (void)hipStreamDestroy(st->s_out);
    }
    delete st;
}

namespace {

// Maximal runs of consecutive blocks (in chunk order) that are contiguous in
// host memory; staging blocks are packed in chunk order.
void add_block(std::vector<CopyRun> &runs, int64_t host, int64_t staging, int64_t elems)
{
    if (!runs.empty() && runs.back().host + runs.back().elems == host &&
        runs.back().staging + runs.back().elems == staging) {
        runs.back().elems += elems;
        return;
    }
    runs.push_back(CopyRun{ host, staging, elems });
}

int build_stream_plan(gd_ctx *ctx, gd_stream_state &st, const gd_opts *opts, int npatch,
                      const gd_patch *patches, bool has_flux, size_t chunk_bytes, hipStream_t s)
{
    const int dtype = opts->dtype, shape = ctx->shape_batched[dtype], zp = ctx->zpolicy_batched[dtype];
    if (st.dtype == dtype && st.shape == shape && st.zpolicy == zp && st.has_flux == (int)has_flux &&
        st.chunk_bytes == chunk_bytes && (int)st.host.size() == npatch &&
        std::memcmp(st.host.data(), patches, npatch * sizeof(gd_patch)) == 0)
        return GD_OK;
    const size_t es = elem_size(opts);
    // patches in host-memory order of their inputs, so that packed batches
    // copy in one run per chunk and buffer
    std::vector<int> order(npatch);
    for (int i = 0; i < npatch; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return patches[a].u_in_off < patches[b].u_in_off; });
    std::vector<gd::PatchDesc> desc;
    std::vector<gd::WorkItem> items;
    std::vector<StreamChunk> chunks;
    int64_t in_max = 0, out_max = 0, fl_max = 0;
    size_t i = 0;
    while (i < order.size()) {
        StreamChunk c{};
        c.patch0 = (int)desc.size();
        c.item0 = (int)items.size();
        while (i < order.size()) {
            const gd_patch &p = patches[order[i]];
            const int64_t ni = in_elems(p.nx, p.ny, p.nz, p.ng, false);
            const int64_t no = 5LL * p.nx * p.ny * p.nz;
            const int64_t nf = has_flux && p.flux_off >= 0 ? flux_elems(p.nx, p.ny, p.nz) : 0;
            const size_t bytes = (size_t)(c.in_elems + ni + c.out_elems + no + c.fl_elems + nf) * es;
            if (bytes > chunk_bytes) {
                if (c.npatch == 0)
                    return fail(ctx, GD_E_ARG, "patch %d needs %zu bytes, more than chunk_bytes %zu",
                                order[i], (size_t)(ni + no + nf) * es, chunk_bytes);
                break;
            }
            gd::PatchDesc d = to_desc(p, false);
            d.in_off = c.in_elems;
            d.out_off = c.out_elems;
            d.flux_off = nf ? c.fl_elems : -1;
            add_block(c.in, p.u_in_off, c.in_elems, ni);
            add_block(c.out, p.u_out_off, c.out_elems, no);
            if (nf) add_block(c.flux, p.flux_off, c.fl_elems, nf);
            c.in_elems += ni;
            c.out_elems += no;
            c.fl_elems += nf;
            const int pidx = (int)desc.size();
            desc.push_back(d);
            const int zl = batched_zlen(p.nz, zp);
            const int pshape = gd::patch_tile_shape(shape, p.nx, p.ny);
            const int TX = gd::tile_tx(pshape), TY = gd::tile_ty(pshape);
            for (int z0 = 0; z0 < p.nz; z0 += zl)
                for (int y0 = 0; y0 < p.ny; y0 += TY)
                    for (int x0 = 0; x0 < p.nx; x0 += TX) {
                        gd::WorkItem w{};
                        w.patch = pidx;
                        w.x0 = (int16_t)x0; w.y0 = (int16_t)y0;
                        w.z0 = (int16_t)z0; w.z1 = (int16_t)std::min(z0 + zl, p.nz);
                        w.shape = (int16_t)pshape;
                        items.push_back(w);
                    }
            ++c.npatch;
            ++i;
        }
        c.nitems = (int)items.size() - c.item0;
        in_max = std::max(in_max, c.in_elems);
        out_max = std::max(out_max, c.out_elems);
        fl_max = std::max(fl_max, c.fl_elems);
        chunks.push_back(std::move(c));
    }
    if (items.size() > 0x7fffffff) return fail(ctx, GD_E_ARG, "too many work items");
    int r;
    if ((r = ensure_capacity(ctx, &st.d_patches, &st.cap_patches, desc.size()))) return r;
    if ((r = ensure_capacity(ctx, &st.d_items, &st.cap_items, items.size()))) return r;
    const size_t need = NSTAGE * (size_t)(in_max + out_max + fl_max) * es;
    hipError_t e = hipDeviceSynchronize();         // tables and staging may be in use
    if (e == hipSuccess && need > st.staging_bytes) {
        if (st.staging) (void)hipFree(st.staging);
        st.staging = nullptr;
        st.staging_bytes = 0;
        if (hipMalloc(&st.staging, need) != hipSuccess)
            return fail(ctx, GD_E_NOMEM, "staging of %zu bytes", need);
        st.staging_bytes = need;
    }
    if (e == hipSuccess) e = hipMemcpy(st.d_patches, desc.data(), desc.size() * sizeof(gd::PatchDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st.d_items, items.data(), items.size() * sizeof(gd::WorkItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "upload of the streaming tables");
    (void)s;
    st.host.assign(patches, patches + npatch);
    st.dtype = dtype; st.shape = shape; st.zpolicy = zp; st.has_flux = (int)has_flux;
    st.chunk_bytes = chunk_bytes;
    st.chunks = std::move(chunks);
    st.in_max = in_max; st.out_max = out_max; st.fl_max = fl_max;
    return GD_OK;
}

int ensure_streams(gd_ctx *ctx, gd_stream_state &st)
{
    if (st.streams) return GD_OK;
    hipError_t e = hipStreamCreateWithFlags(&st.s_in, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st.s_comp, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st.s_out, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st.ev_start, hipEventDisableTiming);
    for (int b = 0; b < NSTAGE && e == hipSuccess; ++b) {
        e = hipEventCreateWithFlags(&st.ev_in[b], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.ev_comp[b], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.ev_out[b], hipEventDisableTiming);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "streaming streams and events");
    // mark every slot free: record each event once on its (idle) stream
    for (int b = 0; b < NSTAGE && e == hipSuccess; ++b) {
        e = hipEventRecord(st.ev_comp[b], st.s_comp);
        if (e == hipSuccess) e = hipEventRecord(st.ev_out[b], st.s_out);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "streaming events");
    st.streams = true;
    return GD_OK;
}

}  // namespace

extern "C" {

int godunov_step_batched_streamed(gd_ctx *ctx, const gd_opts *opts, int npatch,
                                  const gd_patch *patches, const void *u_in_host, void *u_out_host,
                                  void *bflux_host, const double *dt_dev, double gamma,
                                  size_t chunk_bytes, void *hip_stream)
{
    int r;
    if ((r = check_opts(ctx, opts))) return r;
    if (opts->bc != GD_GHOSTED) return fail(ctx, GD_E_UNSUPPORTED, "batched calls take ghosted patches only");
    if ((r = reject_ppm(ctx, opts, "the streamed batch"))) return r;
    if ((r = validate_patches(ctx, npatch, patches, false))) return r;
    if (!(gamma > 1.0)) return fail(ctx, GD_E_ARG, "gamma must be > 1");
    if (!u_in_host || !u_out_host) return fail(ctx, GD_E_ARG, "u_in_host and u_out_host must not be NULL");
    if (chunk_bytes < 4096) return fail(ctx, GD_E_ARG, "chunk_bytes must be >= 4096");
    const size_t es = elem_size(opts);
    int64_t in_end = 0, out_end = 0, fl_end = 0;
    for (int i = 0; i < npatch; ++i) {
        const gd_patch &p = patches[i];
        in_end = std::max<int64_t>(in_end, p.u_in_off + in_elems(p.nx, p.ny, p.nz, p.ng, false));
        out_end = std::max<int64_t>(out_end, p.u_out_off + 5LL * p.nx * p.ny * p.nz);
        if (bflux_host && p.flux_off >= 0)
            fl_end = std::max<int64_t>(fl_end, p.flux_off + flux_elems(p.nx, p.ny, p.nz));
    }
    if (overlap(u_in_host, in_end * es, u_out_host, out_end * es))
        return fail(ctx, GD_E_ARG, "u_out_host range overlaps u_in_host range");
    if (bflux_host && fl_end > 0 && (overlap(bflux_host, fl_end * es, u_in_host, in_end * es) ||
                                     overlap(bflux_host, fl_end * es, u_out_host, out_end * es)))
        return fail(ctx, GD_E_ARG, "bflux_host range overlaps u_in_host or u_out_host");
    if (!ctx) return fail(ctx, GD_E_ARG, "ctx is NULL");
    if ((r = set_device(ctx))) return r;
    if (capturing((hipStream_t)hip_stream))
        return fail(ctx, GD_E_UNSUPPORTED, "a streamed batch cannot be captured into a graph");
    if (!ctx->stream) ctx->stream = new gd_stream_state();
    gd_stream_state &st = *ctx->stream;
    hipStream_t caller = (hipStream_t)hip_stream;
    if ((r = ensure_streams(ctx, st))) return r;
    if ((r = build_stream_plan(ctx, st, opts, npatch, patches, bflux_host != nullptr, chunk_bytes,
                               caller)))
        return r;

    // the pipeline starts after the caller's earlier work (dt_dev may come
    // from it) and the caller's stream waits for its end
    hipError_t e = hipEventRecord(st.ev_start, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(st.s_in, st.ev_start, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(st.s_comp, st.ev_start, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "streamed batch start");
    const int64_t slot = st.in_max + st.out_max + st.fl_max;
    const int per_cu = gd::max_resident_blocks(opts->dtype, opts->limiter, opts->riemann, st.shape,
                                               ctx->device);
    gd::Scalars sc{ gamma, opts->rho_floor, opts->p_floor };
    const Slot cslot = slot_for(ctx, st.s_comp);
    gd::CflOut co{ 0.0, nullptr, cslot.u64 + 2, cslot.u32 + 3 };
    const char *hin = (const char *)u_in_host;
    char *hout = (char *)u_out_host, *hfl = (char *)bflux_host;
    for (size_t c = 0; c < st.chunks.size() && e == hipSuccess; ++c) {
        const StreamChunk &ch = st.chunks[c];
        const int b = (int)(c % NSTAGE);
        char *base = (char *)st.staging + (size_t)b * slot * es;
        char *sin = base, *sout = base + st.in_max * es, *sfl = sout + st.out_max * es;
        // inputs of chunk c overwrite slot b once chunk c-NSTAGE's step has read it
        e = hipStreamWaitEvent(st.s_in, st.ev_comp[b], 0);
        for (const CopyRun &run : ch.in)
            if (e == hipSuccess)
                e = hipMemcpyAsync(sin + run.staging * es, hin + run.host * es, run.elems * es,
                                   hipMemcpyHostToDevice, st.s_in);
        if (e == hipSuccess) e = hipEventRecord(st.ev_in[b], st.s_in);
        // the step writes slot b's outputs once chunk c-NSTAGE's have been copied out
        if (e == hipSuccess) e = hipStreamWaitEvent(st.s_comp, st.ev_in[b], 0);
        if (e == hipSuccess) e = hipStreamWaitEvent(st.s_comp, st.ev_out[b], 0);
        if (e == hipSuccess) {
            int grid = std::max(1, std::min(ch.nitems, per_cu * ctx->num_cus));
            int ke = gd::launch_step_batched(opts->dtype, opts->limiter, opts->riemann, st.shape,
                                             st.d_patches, st.d_items + ch.item0, ch.nitems, sin, sout,
                                             ch.fl_elems ? sfl : nullptr, dt_dev, sc, ctx->d_u64,
                                             cslot.u32, grid, co, st.s_comp);
            if (ke) e = (hipError_t)ke;
        }
        if (e == hipSuccess) e = hipEventRecord(st.ev_comp[b], st.s_comp);
        if (e == hipSuccess) e = hipStreamWaitEvent(st.s_out, st.ev_comp[b], 0);
        for (const CopyRun &run : ch.out)
            if (e == hipSuccess)
                e = hipMemcpyAsync(hout + run.host * es, sout + run.staging * es, run.elems * es,
                                   hipMemcpyDeviceToHost, st.s_out);
        for (const CopyRun &run : ch.flux)
            if (e == hipSuccess)
                e = hipMemcpyAsync(hfl + run.host * es, sfl + run.staging * es, run.elems * es,
                                   hipMemcpyDeviceToHost, st.s_out);
        if (e == hipSuccess) e = hipEventRecord(st.ev_out[b], st.s_out);
    }
    for (int b = 0; b < NSTAGE && e == hipSuccess; ++b) e = hipStreamWaitEvent(caller, st.ev_out[b], 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "streamed batch");
    return GD_OK;
}

}  // extern "C"
