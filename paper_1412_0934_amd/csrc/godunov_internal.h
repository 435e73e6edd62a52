// Internal interface between the C-ABI host layer (godunov_api.cpp) and the
// gfx950 kernels (godunov_kernels.hip). Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

// Device-side description of one patch. Offsets are in elements of the call's
// dtype. For a periodic box ng = 0 and the input has the output's shape.
struct PatchDesc {
    int32_t nx, ny, nz, ng;
    int32_t periodic;
    int32_t pad_;
    int64_t in_off, out_off, flux_off;   // flux_off < 0: no boundary fluxes
    double dx, dt;
};

// One unit of work of the forward step: an x-y tile of a patch and the
// z-range [z0, z1) that the workgroup marches through.
struct WorkItem {
    int32_t patch;
    int16_t x0, y0;
    int16_t z0, z1;
    int16_t shape;       // index of the tile shape (kernel variant) to use
    int16_t pad_;
};

// Tile shapes the forward kernels are instantiated for (interior columns
// TX x TY of one workgroup).
// TILE_PAIR_24x8 is a batched-only choice: one launch that steps each patch
// in 24x8 tiles where they cover its x-y extent with fewer padded columns than
// 16x8 tiles do, and in 16x8 tiles otherwise, in 256-thread workgroups.
enum TileShape : int {
    TILE_16x16 = 0, TILE_8x8 = 1, TILE_32x8 = 2, TILE_16x8 = 3, TILE_24x8 = 4, NUM_TILE_SHAPES = 5,
    TILE_PAIR_24x8 = 5, NUM_BATCHED_SHAPES = 6
};
int tile_tx(int shape);
int tile_ty(int shape);
// the concrete shape that a batched launch of `shape` uses on a patch
int patch_tile_shape(int shape, int nx, int ny);

struct Scalars {
    double gamma, rho_floor, p_floor;
};

// Optional fused CFL output of a step launch: when dt_next is not null the
// launch also reduces the signal speed of the state it writes and its last
// workgroup stores dt_next = cfl / max((|u|+|v|+|w|+3c)/dx).
struct CflOut {
    double cfl;
    double *dt_next;
    unsigned long long *smax_bits;
    unsigned *done;
};

// Launchers. Return 0 or a hipError_t value.
// launch_step: z-ranges of zlen planes, shorter (down to one) where the
// patch would otherwise give fewer than min_blocks workgroups.
int launch_step(int dtype, int limiter, int riemann, int shape, const PatchDesc &P,
                const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                const Scalars &sc, unsigned long long *hits, int zlen, int min_blocks,
                const CflOut &co, hipStream_t s);

int launch_step_batched(int dtype, int limiter, int riemann, int shape,
                        const PatchDesc *d_patches, const WorkItem *d_items, int nitems,
                        const void *u_in, void *u_out, void *bflux, const double *dt_dev,
                        const Scalars &sc, unsigned long long *hits, unsigned *d_queue,
                        int grid, const CflOut &co, hipStream_t s);

// Work item of the CFL reduction: rows [j0, j0+nrow) of plane k of a patch.
struct CflItem {
    int32_t patch;
    int32_t k;
    int32_t j0, nrow;
};

int launch_cfl(int dtype, const PatchDesc *d_patches, const CflItem *d_items, int nitems,
               const void *u, const Scalars &sc, double cfl, double *dt_out,
               unsigned long long *smax_bits, unsigned *done, int grid, hipStream_t s);

int launch_cfl_single(int dtype, const PatchDesc &P, const void *u, const Scalars &sc,
                      double cfl, double *dt_out, unsigned long long *smax_bits,
                      unsigned *done, hipStream_t s);

// Bytes of device scratch the adjoint of one patch needs.
size_t adjoint_scratch_bytes(const PatchDesc &P);

// Whether the adjoint's 32-bit indexing covers the patch.
bool adjoint_fits_32bit(const PatchDesc &P);

int launch_adjoint(int limiter, int riemann, const PatchDesc &P, const double *u_in,
                   const double *lam_out, const double *lam_bflux, double *lam_in,
                   const Scalars &sc, double dt, double *scratch, hipStream_t s);

// Workgroups of the step kernel of a scheme and tile shape that one CU holds
// at once (the batched and single-patch kernels have the same resources).
int max_resident_blocks(int dtype, int limiter, int riemann, int shape, int device);

// Ideal MHD on a periodic box (godunov_mhd.hip).
struct MhdScalars {
    double gamma, rho_floor, p_floor, dx, dt, ch, alpha;
};

// Bytes of device scratch one MHD step of an nx x ny x nz box needs.
size_t mhd_scratch_bytes(int dtype, int nx, int ny, int nz);

// One step; dt_dev / ch_dev, when not null, replace sc.dt / sc.ch. With
// dt_next or ch_next not null the launch also writes the next step's
// cfl dx / max sum_d (|u_d| + cf_d) and max_d (|u_d| + cf_d) of u_out there
// (acc: two zeroed 64-bit accumulators, left zeroed again).
int launch_mhd_step(int dtype, int limiter, int nx, int ny, int nz, const void *u_in, void *u_out,
                    const MhdScalars &sc, const double *dt_dev, const double *ch_dev,
                    void *scratch, double cfl, double *dt_next, double *ch_next,
                    unsigned long long *acc, hipStream_t s);

// dt = cfl dx / max sum_d (|u_d| + cf_d) and ch = max_d (|u_d| + cf_d) into
// device scalars (either may be null); acc: two zeroed 64-bit accumulators,
// left zeroed again.
int launch_mhd_speeds(int dtype, int nx, int ny, int nz, const void *u, const MhdScalars &sc,
                      double cfl, double *dt_dev, double *ch_dev, unsigned long long *acc,
                      hipStream_t s);

// Two-level AMR seams (godunov_amr.hip). Tables are built on the host once
// per hierarchy; coarse cells are indexed (z * ny + y) * nx + x.
struct AmrPatch {
    int32_t lo[3];          // coarse cell (x, y, z) of the lower corner
    int32_t n[3];           // interior extents in fine cells (even)
    int64_t in_off, out_off, flux_off;
};

// 256 consecutive cells of the box of coarse cells around one patch (the
// patch's footprint and a one-cell shell), for the ghost fill.
struct AmrFillItem {
    int32_t patch, start;
};

// One coarse-fine face. right: coarse cell on the + side of the face;
// dside = 2 d + side, side 1 when the uncovered cell is on the + side;
// fine: element offset in the flux buffer of variable 0 of the first of the
// 2x2 fine faces; row: elements between the two rows of the block; vstride:
// elements between variables of the sheet.
struct AmrFace {
    int32_t right, dside;
    int64_t fine;
    int32_t row, vstride;
};

// A covered coarse cell and the offset in the fine output of variable 0 of
// its child at (0, 0, 0).
struct AmrCover {
    int32_t coarse, patch;
    int64_t child;
};

struct AmrTables {
    int32_t nc[3];
    int32_t nfill, ncells, ncover, nfaces;
    const int32_t *owner;           // coarse cell -> covering patch or -1
    const AmrPatch *patches;
    const AmrFillItem *fill;
    const int32_t *cells;           // uncovered coarse cells with interface faces
    const int32_t *cell_start;      // ncells + 1 offsets into faces
    const AmrFace *faces;
    const AmrCover *cover;
    void *fstate;                   // scratch: 10 nfaces values (left, right face states)
};

int launch_amr_fill(int dtype, const AmrTables &t, const void *coarse, void *fine, hipStream_t s);

// Refluxing of the uncovered cells and averaging down of the covered ones
// (two launches: face states, then corrections and averages); dt_dev, when
// not null, replaces dt.
int launch_amr_seam(int dtype, int limiter, int riemann, const AmrTables &t, const void *coarse_old,
                    void *coarse_new, const void *fine_out, const void *fine_flux,
                    const Scalars &sc, double dx_coarse, double dt, const double *dt_dev,
                    hipStream_t s);

// Record the message of a failing call that has no context (the text
// gd_last_error(NULL) returns on this thread); returns code.
int set_call_error(int code, const char *fmt, ...);

// *dst = v, stream-ordered (capturable, unlike a host-to-device copy).
int launch_set_scalar(double *dst, double v, hipStream_t s);

// Piecewise-parabolic reconstruction (godunov_ppm.hip).
// Cells of a patch's PPM scratch box: the interior (periodic) or the interior
// plus one layer (ghosted); the scratch holds 30 values per box cell.
int64_t ppm_box_cells(const PatchDesc &P);

// One PPM step of the patch P in two launches over a face-state scratch of
// 30 values per box cell: the path of periodic boxes with an extent below 2,
// whose wrapped stencils the single-launch march does not cover.
int launch_ppm(int dtype, int limiter, int riemann, const PatchDesc &P, const void *u_in,
               void *u_out, void *bflux, void *scratch, const double *dt_dev, const Scalars &sc,
               unsigned long long *hits, hipStream_t s);

// One PPM step (limiters 3 to 6) of a single patch in one launch: the tile
// march of the PLM step with the parabola, no face-state scratch; with
// co.dt_next the CFL signal of the new state is reduced into co.smax_bits
// (launch_cfl_finalize turns it into dt).
constexpr int PPM_FUSED_TX = 24, PPM_FUSED_TY = 8;
int launch_ppm_tile(int dtype, int limiter, int riemann, const PatchDesc &P, const void *u_in,
                    void *u_out, void *bflux, const double *dt_dev, const Scalars &sc,
                    unsigned long long *hits, int min_blocks, const CflOut &co, hipStream_t s);
// The same for a batch of ghosted patches: one persistent launch over the
// (patch, tile, z-range) items of 24x8 tiles, the queue counters in d_queue
// (reset by the launch's last workgroup), as many workgroups as fit on
// num_cus compute units.
int launch_ppm_batched(int dtype, int limiter, int riemann, const PatchDesc *d_patches,
                       const WorkItem *d_items, int nitems, const void *u_in, void *u_out,
                       void *bflux, const double *dt_dev, const Scalars &sc,
                       unsigned long long *hits, unsigned *d_queue, int num_cus, const CflOut &co,
                       hipStream_t s);
// dt = cfl / (the maximum folded into smax_bits), which is cleared for the next use
int launch_cfl_finalize(double cfl, double *dt_out, unsigned long long *smax_bits, hipStream_t s);

}  // namespace gd
