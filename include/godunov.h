/*
 * godunov.h -- C ABI of the MI355X (gfx950) Godunov step library, libgodunov.so.
 *
 * One call advances the compressible Euler equations of an ideal gas by one
 * time step on one or many ghost-zoned patches, with a second-order unsplit
 * MUSCL-Hancock Godunov scheme (the piecewise-linear method family the paper
 * names in Sec. 2), and hands back the fluxes through each patch boundary
 * that a multilevel, adaptive-time-step caller needs for coarse-fine flux
 * correction (Sec. 4). The patch is the paper's GPU work unit: inner cells
 * plus boundary (ghost) cells already filled by the caller, interpolated
 * where the patch adjoins another refinement level (Sec. 3).
 *
 * Scheme, per step (every array in one call has the same dtype):
 *   1. conserved U = (rho, rho u, rho v, rho w, E) -> primitive
 *      W = (rho, u, v, w, p), p = (gamma-1)(E - |rho u|^2/(2 rho)); rho and p
 *      raised to rho_floor and p_floor (each raise is counted);
 *   2. undivided limited slopes of W along x, y and z (gd_limiter);
 *   3. half-step predictor W* = W - dt/(2dx) sum_d A_d(W) dW_d, with A_d the
 *      primitive-variable Jacobian along d (all three directions, no
 *      transverse Riemann solves);
 *   4. face states W_L = W*_i + dW_i/2, W_R = W*_{i+1} - dW_{i+1}/2, floored;
 *   5. one Riemann flux per face (gd_riemann), Davis wave-speed bounds
 *      S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R);
 *   6. U' = U - dt/dx [((F_x+ - F_x-) + (F_y+ - F_y-)) + (F_z+ - F_z-)].
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller; the
 * library never allocates or frees caller data. Layouts are C order, x
 * fastest, structure of arrays over the five conserved variables:
 *   ghosted input  [5][nz+2ng][ny+2ng][nx+2ng]  (ng >= 2; only the interior,
 *                  face ghosts of depth <= 2 and edge ghosts of depth 1 are
 *                  read -- corner ghosts are never read)
 *   periodic input [5][nz][ny][nx]              (neighbours wrap around)
 *   output         [5][nz][ny][nx]              (interior only)
 *   boundary flux  six sheets in the order x-, x+, y-, y+, z-, z+, each
 *                  [5][slow][fast] with (slow, fast) = (z, y) for x sheets,
 *                  (z, x) for y sheets, (y, x) for z sheets; total
 *                  10 (nz ny + nz nx + ny nx) values. A sheet holds the face
 *                  flux F_d exactly as used in step 6 (positive = transport
 *                  towards +d), per unit area and time; a refluxing caller
 *                  multiplies by dt and the face area.
 *
 * Errors: every entry point returns a gd_status. All argument checks run on
 * the host before anything is launched; on failure nothing is launched and
 * gd_last_error() describes the problem. A HIP error from a launch is
 * returned as GD_E_HIP. Non-physical states are floored and counted, never
 * reported as errors; NaN inputs propagate to the outputs.
 *
 * Ordering: every call is asynchronous and stream-ordered on the HIP stream
 * passed in (NULL = the null stream). The host waits only in gd_get_stats(),
 * the autotuners, context and AMR-plan set-up, and the calls that (re)build
 * device tables or grow the library's scratch: the first batched, PPM or CFL
 * call with a new descriptor list and the first call that needs more
 * scratch (each says so below); later calls with the same descriptors and
 * sizes never wait. One gd_ctx per host thread.
 *
 * Streams: each stream a context sees (the first 64 distinct ones) gets
 * device counters of its own -- the batched work queue and the CFL and MHD
 * speed accumulators -- so steps, batched steps and CFL reductions in flight
 * together on different streams do not interfere (beyond 64 streams the
 * counter slots are shared round robin). The scratch memory of the adjoint,
 * PPM and MHD steps and the cached batch tables are one per context: two
 * calls of those kinds with different sizes or descriptors in flight
 * together on different streams race; give each stream its own gd_ctx.
 *
 * Graph capture: a call made while hip_stream is capturing marks the tables
 * and scratch it uses; the library never overwrites or frees marked memory
 * before gd_destroy (a later call that needs other tables or more scratch
 * allocates new ones), so a captured graph stays valid whatever calls
 * follow. A call under capture that would have to build tables or grow
 * scratch (it would wait on the host) returns GD_E_UNSUPPORTED: make one
 * call with the same descriptors and sizes outside the capture first. The
 * autotuners and the streamed batch cannot be captured (GD_E_UNSUPPORTED).
 * A graph uses the counter slot of the stream it was captured on: replaying
 * it while calls on that stream are in flight elsewhere races.
 */
#ifndef GODUNOV_H
#define GODUNOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gd_ctx gd_ctx;

typedef enum {
    GD_OK = 0,
    GD_E_ARG = -1,          /* invalid argument; nothing was launched */
    GD_E_HIP = -2,          /* the HIP runtime reported an error */
    GD_E_NOMEM = -3,        /* the library could not allocate its own scratch */
    GD_E_UNSUPPORTED = -4   /* valid but not implemented combination */
} gd_status;

typedef enum { GD_F64 = 0, GD_F32 = 1 } gd_dtype;          /* dtype of every array */
typedef enum { GD_GHOSTED = 0, GD_PERIODIC = 1 } gd_bc;      /* layout of the input */
typedef enum {
    GD_MINMOD = 0, GD_MC = 1, GD_UNLIMITED = 2,
    GD_PPM = 3,             /* piecewise-parabolic reconstruction (see below) */
    GD_PPM_UNLIMITED = 4,   /* the same parabola without its limiters */
    GD_PPM_CT = 5,          /* GD_PPM with characteristic tracing (see below) */
    GD_PPM_CT_UNLIMITED = 6 /* GD_PPM_UNLIMITED with characteristic tracing */
} gd_limiter;
typedef enum { GD_HLLC = 0, GD_HLL = 1 } gd_riemann;

/* Scheme options. minmod(a,b) = 0 unless a, b share a sign, else the one of
 * smaller magnitude; MC = sign(a) min(2|a|, 2|b|, |a+b|/2) for a, b of one
 * sign, else 0; unlimited = (a+b)/2. HLLC resolves the contact wave (Toro,
 * Spruce & Speares 1994); HLL does not (Harten, Lax & van Leer 1983). */
typedef struct {
    int32_t dtype;          /* gd_dtype */
    int32_t bc;             /* gd_bc (batched calls: GD_GHOSTED only) */
    int32_t limiter;        /* gd_limiter */
    int32_t riemann;        /* gd_riemann */
    double rho_floor;       /* >= 0 */
    double p_floor;         /* >= 0 */
} gd_opts;

/* One patch of a batched call. Offsets are in ELEMENTS (of the call's dtype)
 * from the base pointers; the input block is [5][nz+2ng][ny+2ng][nx+2ng],
 * the output block [5][nz][ny][nx], the flux block the six sheets above.
 * flux_off < 0 means: no boundary fluxes for this patch. Blocks of different
 * patches must not overlap in the output and flux buffers. */
typedef struct {
    int32_t nx, ny, nz, ng;
    int64_t u_in_off, u_out_off, flux_off;
    double dx, dt;          /* cell width and time step of this patch (levels may differ) */
} gd_patch;

/* Create a context on HIP device `device` (made current). Allocates about
 * 5 KB of device counters (a floor-hit counter and 64 per-stream slots). Returns GD_E_HIP if there is no such
 * device; then *ctx is NULL and gd_last_error(NULL) has the reason. */
int gd_create(gd_ctx **ctx, int device);

/* Release a context and its device memory (synchronises its device). */
int gd_destroy(gd_ctx *ctx);

/* Message of the last failing call on ctx (or of the last failing
 * gd_create on this thread when ctx is NULL). Valid until the next call. */
const char *gd_last_error(const gd_ctx *ctx);

/* Number of floor applications since the last reset (sum over calls).
 * Synchronises the device: for tests and diagnostics only. */
int gd_get_stats(gd_ctx *ctx, uint64_t *floor_hits);
int gd_reset_stats(gd_ctx *ctx);

/* One Godunov step of one patch (steps 1-6 above; Sec. 3 and Sec. 4 of the
 * paper: all face fluxes of the patch computed on the device, boundary
 * fluxes returned). nx, ny, nz >= 1; ng >= 2 for GD_GHOSTED, ng >= 3 with PPM (ignored for
 * GD_PERIODIC). u_out must not overlap u_in. bflux may be NULL. If dt_dev is
 * not NULL the step reads dt (a double) from that device address, e.g. as
 * written by cfl_dt, and the dt argument is ignored. gamma > 1, dx > 0,
 * dt >= 0 (dt is passed as double also for GD_F32 and rounded once). */
int godunov_step(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
                 const void *u_in, void *u_out, void *bflux,
                 double gamma, double dx, double dt, const double *dt_dev, void *hip_stream);

/* One Godunov step of every patch in a batch, in ONE persistent launch: the
 * workgroups pull (patch, tile) items from a device work queue, so thousands
 * of uneven patches (e.g. 8^3 .. 32^3) keep the whole GPU busy (the batch of
 * patches that the paper's GPU ports build per level, Sec. 3 and Sec. 4).
 * patches is a HOST array of npatch descriptors (GD_GHOSTED layout only);
 * the library keeps a device copy and rebuilds it only when the descriptors
 * change (the rebuild synchronises hip_stream and uploads the tables), so
 * repeated calls with the same descriptors allocate nothing, never wait and
 * may be captured into a HIP graph. If dt_dev is not NULL every patch uses
 * the device double *dt_dev instead of patches[i].dt. bflux_base may be
 * NULL (then every flux_off is ignored). Patches must not share output. */
int godunov_step_batched(gd_ctx *ctx, const gd_opts *opts, int npatch, const gd_patch *patches,
                         const void *u_in_base, void *u_out_base, void *bflux_base,
                         const double *dt_dev, double gamma, void *hip_stream);

/* godunov_step / godunov_step_batched that also produce the CFL time step of
 * the state they write: the launch reduces (|u|+|v|+|w|+3c)/dx over every
 * interior cell it writes, and its last workgroup stores
 * *dt_next_dev = cfl / max, the value cfl_dt would return for u_out (Sec. 4:
 * adaptive time steps). A time loop then needs one launch per step and never
 * reads the state a second time. dt_next_dev may be the same address as
 * dt_dev (every workgroup reads dt before the last one writes). cfl > 0. */
int godunov_step_cfl(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
                     const void *u_in, void *u_out, void *bflux, double gamma, double dx,
                     double dt, const double *dt_dev, double cfl, double *dt_next_dev,
                     void *hip_stream);
int godunov_step_batched_cfl(gd_ctx *ctx, const gd_opts *opts, int npatch,
                             const gd_patch *patches, const void *u_in_base, void *u_out_base,
                             void *bflux_base, const double *dt_dev, double gamma, double cfl,
                             double *dt_next_dev, void *hip_stream);

/* Reverse-mode adjoint of godunov_step for a FIXED dt (dt is not
 * differentiated): given lam_out = dL/dU^{n+1} ([5][nz][ny][nx]) and
 * optionally lam_bflux = dL/dbflux (boundary-flux layout, or NULL), writes
 * lam_in = dL/dU^n in the layout of u_in: ghost-cell adjoints included for
 * GD_GHOSTED (zero for ghosts the step does not read), contributions of
 * wrapped neighbours folded onto the interior for GD_PERIODIC. At the kinks
 * of the scheme (limiter switches, wave-speed min/max, HLLC region, floors)
 * the derivative of the branch the forward step takes is used. Every
 * element of lam_in is written exactly once (gather form, deterministic).
 * GD_F64 only (GD_E_UNSUPPORTED otherwise); lam_in must not overlap any
 * input (GD_E_ARG). The library keeps a device scratch of 324 bytes per
 * cell of the scratch box -- the box itself when periodic, the box extended
 * by two layers, (nx+4)(ny+4)(nz+4), when ghosted -- grown on first use
 * (the growth synchronises the device; GD_E_NOMEM if it fails); boxes whose
 * scratch box has 20 times its cell count at or above 2^31 (a periodic box
 * above about 475^3) return GD_E_UNSUPPORTED. */
int godunov_step_adjoint(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
                         const void *u_in, const void *lam_out, const void *lam_bflux,
                         void *lam_in, double gamma, double dx, double dt, void *hip_stream);

/* CFL time step dt = cfl / max over patches p and interior cells of
 * (|u| + |v| + |w| + 3c) / dx_p, c the sound speed of the floored primitive
 * state (the stability bound of the unsplit scheme; the paper's codes take an
 * adaptive time step per level, Sec. 4). Written as one double to the device
 * address dt_dev; nothing returns to the host. patches is a HOST array;
 * for one periodic box pass npatch = 1 and opts->bc = GD_PERIODIC with
 * patches[0].ng = 0 and u_in_off = 0. cfl > 0. */
int cfl_dt(gd_ctx *ctx, const gd_opts *opts, int npatch, const gd_patch *patches,
           const void *u_base, double gamma, double cfl, double *dt_dev, void *hip_stream);

/* Autotuning (the choice of tile shape and z-range length of the step
 * kernels). Each call times every candidate configuration on the given
 * problem with HIP events on hip_stream (one warm-up launch, then the mean
 * of a few launches per candidate), keeps the fastest in ctx for later calls
 * of the same dtype, and returns its index in *choice (may be NULL). The
 * outputs are overwritten; the stream is synchronised. Candidates: tiles of
 * 16x16, 32x8, 8x8, 16x8 and 24x8 interior columns, and for batches also
 * the pair 16x8 + 24x8 in one launch (each patch in the shape that covers its
 * x-y extent with fewer padded columns, 16x8 on a tie); z-ranges of 16, 32
 * and 64 planes (single patch) or of 8 planes, 16 planes and the whole patch
 * (batched). The batched candidate index is 3 * (position of the shape in
 * that list) + z policy, 0..17. */
int gd_autotune_step(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, int ng,
                     const void *u_in, void *u_out, double gamma, double dx, double dt,
                     void *hip_stream, int *choice);
int gd_autotune_batched(gd_ctx *ctx, const gd_opts *opts, int npatch, const gd_patch *patches,
                        const void *u_in_base, void *u_out_base, void *bflux_base, double gamma,
                        void *hip_stream, int *choice);

/* The configuration in use: tile shape index (0: 16x16, 1: 8x8, 2: 32x8,
 * 3: 16x8, 4: 24x8; batched also 5: the pair 16x8 + 24x8, the shape
 * chosen per patch)
 * and z-range length (single patch) or z-range policy (batched: 0 = 8
 * planes, 1 = 16, 2 = whole patch) for dtype. */
int gd_get_config(gd_ctx *ctx, int dtype, int *shape_single, int *zlen_single,
                  int *shape_batched, int *zpolicy_batched);

/* Set the configuration explicitly (e.g. one stored from an earlier
 * autotuning run). shape_single in [0, 4], shape_batched in [0, 5];
 * zlen_single in [1, 4096];
 * zpolicy_batched in {0, 1, 2}. zlen_single is an upper bound: a patch that
 * would give fewer workgroups than the device holds at once is cut into
 * shorter z-ranges (down to one plane). The choice never changes results: every
 * face flux and every update is evaluated by the same arithmetic whatever
 * the tiling, so outputs are bitwise identical across configurations. */
int gd_set_config(gd_ctx *ctx, int dtype, int shape_single, int zlen_single, int shape_batched,
                  int zpolicy_batched);

/* ------------------------------------------------------------ streamed batches
 *
 * godunov_step_batched for a batch held in HOST memory (the paper's GPU ports
 * copy each level's patches to the device and back every step, Sec. 3 and
 * Sec. 4; Ramses could not hide that copy): u_in_host, u_out_host and
 * bflux_host (may be NULL) are host buffers laid out as the device buffers of
 * godunov_step_batched (same gd_patch offsets). The patches, taken in the
 * order of their input offsets, are cut into chunks whose input, output and
 * flux blocks fit chunk_bytes (>= 4096; a patch that alone exceeds it is
 * GD_E_ARG). Each chunk is copied into one of three device staging slots,
 * stepped there by the batched kernel and copied back, on three streams of
 * the library's own, so that the copies of one chunk overlap the step of the
 * next; consecutive blocks contiguous in host memory move in one copy.
 * Results are bitwise those of godunov_step_batched on the same data.
 * The pipeline starts after the work already queued on hip_stream, and
 * hip_stream waits for its end: synchronise hip_stream before reading the
 * host outputs; the host buffers must stay valid until then. Copies overlap
 * only with pinned host memory (hipHostMalloc); pageable memory gives the
 * same results without overlap. The context keeps the staging (three slots of
 * up to chunk_bytes) and the chunk tables, rebuilt (synchronising the device)
 * when the descriptors, dtype, chunk_bytes or batched tile choice change.
 * GD_GHOSTED only; PLM limiters only (GD_E_UNSUPPORTED for PPM). */
int godunov_step_batched_streamed(gd_ctx *ctx, const gd_opts *opts, int npatch,
                                  const gd_patch *patches, const void *u_in_host, void *u_out_host,
                                  void *bflux_host, const double *dt_dev, double gamma,
                                  size_t chunk_bytes, void *hip_stream);

/* ------------------------------------------------------------ PPM
 *
 * opts->limiter = GD_PPM or GD_PPM_UNLIMITED on godunov_step(_cfl) and
 * godunov_step_batched(_cfl) replaces steps 2-4 of the scheme by the
 * piecewise-parabolic reconstruction of Colella & Woodward (1984), the PPM
 * the paper lists beside PLM and TVD (Sec. 2, Sec. 4). Per axis and primitive
 * variable a of cell i:
 *   interface value a_{i+1/2} = (a_i + a_{i+1})/2 - (da_{i+1} - da_i)/6,
 *     da the MC-limited slope (GD_PPM) or the central difference
 *     (a_{i+1} - a_{i-1})/2 (GD_PPM_UNLIMITED, fourth-order interface values);
 *   edges a_L = a_{i-1/2}, a_R = a_{i+1/2}; GD_PPM then sets a_L = a_R = a_i
 *     at a local extremum ((a_R - a_i)(a_i - a_L) <= 0), else with
 *     D = a_R - a_L, m = a_i - (a_L + a_R)/2: a_L = 3a_i - 2a_R if
 *     D m > D^2/6, a_R = 3a_i - 2a_L if D m < -D^2/6;
 *   the Hancock half step of step 3 with slopes a_R - a_L, and the face
 *     states W* + (a_R - W) (upper face) and W* + (a_L - W) (lower face),
 *     floored; steps 5-7 unchanged.
 * GD_PPM_CT and GD_PPM_CT_UNLIMITED replace the last two items by Colella &
 * Woodward's characteristic tracing along each axis d: with the waves of the
 * primitive system along d at the cell's state (speeds u_d - c, u_d (entropy
 * and two shear waves), u_d + c, Courant numbers s = speed dt/dx), the state
 * on the upper face is a_R + sum over the waves with s > 0 of
 * (l . (A(s) - a_R)) r, A(s) - a_R = -(s/2)(a_R - a_L - (1 - 2s/3) a_6),
 * a_6 = 6 (a - (a_L + a_R)/2) -- the parabolas' average over the last s of
 * the cell minus the edge -- and on the lower face a_L + the same over the
 * waves with s < 0 with A(s) - a_L = (|s|/2)(a_R - a_L + (1 - 2|s|/3) a_6);
 * l, r the left and right eigenvectors in (rho, u_n, u_t1, u_t2, p):
 * r = (1, -+c/rho, 0, 0, c^2), l = (0, -+rho/(2c), 0, 0, 1/(2c^2)) for u -+ c;
 * entropy r = (1, 0, 0, 0, 0), l = (1, 0, 0, 0, -1/c^2); shear waves the
 * transverse velocities. Each face state then gains the Hancock terms of the
 * two other axes, -dt/(2dx) sum_{d' != d} A_d'(W) (a_R,d' - a_L,d'), and is
 * floored. For a contact this is the PPM advection scheme (third order on
 * smooth data for the unlimited parabola).
 * A ghosted patch needs ng >= 3 (GD_E_ARG otherwise): the stencil reads face
 * ghosts to depth 3 and edge ghosts at depths (1, <= 2); corners never.
 * godunov_step(_cfl) runs a patch, and godunov_step_batched(_cfl) a batch, in
 * one launch with no scratch (and reduces the new state's CFL step in the
 * same pass), except a periodic box with an extent below 2. That box uses two
 * launches over a device scratch of 30 values per cell of the box, grown on
 * first use (the growth synchronises the device); its _cfl entry point
 * reduces the CFL step in a separate launch after the step. The adjoint, the
 * autotuner, the MHD step and the AMR seams return GD_E_UNSUPPORTED for
 * PPM. */

/* ------------------------------------------------------------ ideal MHD
 *
 * One unsplit MUSCL-Hancock step of ideal magnetohydrodynamics with
 * hyperbolic-parabolic divergence cleaning, the equation set of the paper's
 * Enzo GPU solver (Sec. 2, Sec. 4), on a PERIODIC box (opts->bc must be
 * GD_PERIODIC, else GD_E_UNSUPPORTED; opts->riemann is ignored: the fluxes
 * are HLLD). Units with mu0 = 1.
 *   conserved U = (rho, rho u, rho v, rho w, E, Bx, By, Bz, psi),
 *     E = p/(gamma-1) + rho |u|^2/2 + |B|^2/2; layout [9][nz][ny][nx];
 *   primitive W = (rho, u, v, w, p, Bx, By, Bz, psi), rho and p floored;
 *   undivided limited slopes of W (opts->limiter);
 *   half step: the values at a cell's upper and lower faces along each axis,
 *     W +- S_d/2 (floored), move by one increment
 *     dU = -dt/(2dx) sum_d [F_d(W + S_d/2) - F_d(W - S_d/2)], F_d the
 *     physical flux, in which the flux of B_d is psi and that of psi is
 *     ch^2 B_d (generalised Lagrange multiplier, Dedner et al. 2002);
 *   face flux: B_n* = (B_nL + B_nR)/2 - (psi_R - psi_L)/(2 ch) and
 *     psi* = (psi_L + psi_R)/2 - ch (B_nR - B_nL)/2 give the fluxes of B_n
 *     (psi*) and psi (ch^2 B_n*); the HLLD solver of Miyoshi & Kusano (2005)
 *     with normal field B_n* on both sides and wave speeds
 *     S_L = min(u_L - cf_L, u_R - cf_R), S_R = max(u_L + cf_L, u_R + cf_R)
 *     (cf the fast magnetosonic speed) gives the other seven;
 *   U' = U - dt/dx ((dF_x + dF_y) + dF_z), then psi' *= exp(-alpha ch dt/dx).
 *
 * dt and ch come from the host values, or from device scalars when dt_dev /
 * ch_dev are not NULL (as written by cfl_dt_mhd). u_out must not overlap
 * u_in (GD_E_ARG). The library keeps a device scratch of 54 values per cell,
 * grown on first use (the growth synchronises the device; GD_E_NOMEM if it
 * fails). Boxes with 9 nx ny nz >= 2^31 return GD_E_UNSUPPORTED. Every
 * element of u_out is written once (deterministic). */
int godunov_step_mhd(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, const void *u_in,
                     void *u_out, double gamma, double dx, double dt, const double *dt_dev,
                     double ch, const double *ch_dev, double alpha, void *hip_stream);

/* godunov_step_mhd that also writes, from the state it produces, the next
 * step's dt = cfl dx / max sum_d (|u_d| + cf_d) to *dt_next_dev and
 * ch = max_d (|u_d| + cf_d) to *ch_next_dev (device scalars, either may be
 * NULL but not both; they may be dt_dev and ch_dev themselves, which the
 * step reads before it writes them), the same values cfl_dt_mhd gives for
 * u_out. */
int godunov_step_mhd_cfl(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz,
                         const void *u_in, void *u_out, double gamma, double dx, double dt,
                         const double *dt_dev, double ch, const double *ch_dev, double alpha,
                         double cfl, double *dt_next_dev, double *ch_next_dev, void *hip_stream);

/* Time step and cleaning speed of a periodic MHD box:
 * dt = cfl dx / max over cells of sum_d (|u_d| + cf_d) into *dt_dev and
 * ch = max over cells and axes of |u_d| + cf_d into *ch_dev (device scalars;
 * either may be NULL, not both). The maxima are exact (order-independent);
 * the state's primitives are floored as in the step. */
int cfl_dt_mhd(gd_ctx *ctx, const gd_opts *opts, int nx, int ny, int nz, const void *u,
               double gamma, double dx, double cfl, double *dt_dev, double *ch_dev,
               void *hip_stream);

/* ------------------------------------------------------------ two-level AMR
 *
 * The seams of one step of a two-level hierarchy around the batched step
 * (Sec. 3: the GPU receives patches of inner cells together with boundary
 * cells taken from the neighbouring grids; Sec. 4: the step returns the
 * boundary fluxes that flux correction between levels needs). The coarse
 * level is a periodic box of ncx x ncy x ncz cells of width dx_coarse
 * (layout [5][ncz][ncy][ncx]); the fine level is a set of disjoint patches
 * refined by 2, each covering whole coarse cells strictly inside the box
 * (no patch crosses the periodic boundary), stored as a batch with ng = 2
 * (gd_patch layouts, fine cell width dx_coarse / 2). One step, with the same
 * dt on both levels:
 *   1. ghost fill: every ghost cell of a fine patch (both layers, corners
 *      included) takes the fine cell at the same place if a fine patch covers
 *      it, else the limited linear prolongation of the coarse cell
 *      containing it (per conserved variable, the coarse value plus a quarter
 *      of the minmod slope along each axis, signed by the half of the coarse
 *      cell the fine cell lies in; the eight children of a coarse cell
 *      average back to it); positions wrap periodically;
 *   2. the coarse box and the fine patches each take one step (the fine
 *      batch with its boundary fluxes);
 *   3. refluxing: an uncovered coarse cell next to a fine patch had the
 *      coarse flux F_c through the shared face in its update; the mean
 *      <F_f> of the four fine fluxes through that face replaces it:
 *      U += dt/dx_c (<F_f> - F_c) if the face is the cell's lower face along
 *      d, U += dt/dx_c (F_c - <F_f>) if it is its upper face. F_c is
 *      recomputed from the old coarse state with the step's own arithmetic;
 *      a cell's faces are applied one after another in a fixed order;
 *   4. averaging down: each covered coarse cell becomes the mean of its eight
 *      children, ((c000 + c100) + (c010 + c110)) + ((c001 + c101) + (c011 +
 *      c111)) times 1/8, x fastest.
 * The composite state (uncovered coarse cells and every fine cell) is then
 * conserved to rounding. */
typedef struct gd_amr gd_amr;

typedef struct {
    int32_t lo[3];          /* coarse cell (x, y, z) of the patch's lower corner */
    int32_t n[3];           /* interior extents in fine cells (nx, ny, nz): even, >= 2 */
    int64_t u_in_off, u_out_off, flux_off;   /* as in gd_patch; flux_off >= 0 */
} gd_amr_patch;

/* Build the device tables of a hierarchy on ctx's device (the only
 * allocation of the AMR calls; synchronises the device). patches is a HOST
 * array of npatch >= 0 entries: lo >= 0 and lo + n/2 <= nc on every axis,
 * patches disjoint, 2 nc <= 16384 per axis, ncx ncy ncz < 2^31. Violations
 * return GD_E_ARG with *plan = NULL. The plan belongs to ctx's device and
 * stays valid until gd_amr_destroy. */
int gd_amr_create(gd_ctx *ctx, int ncx, int ncy, int ncz, double dx_coarse, int npatch,
                  const gd_amr_patch *patches, gd_amr **plan);
int gd_amr_destroy(gd_amr *plan);

/* Step 1: write every ghost cell of every fine patch in fine_in_base from
 * the interiors of the fine patches and from coarse_u. Interior cells are
 * not written. dtype is a gd_dtype. */
int gd_amr_fill_ghosts(gd_ctx *ctx, const gd_amr *plan, int dtype, const void *coarse_u,
                       void *fine_in_base, void *hip_stream);

/* Steps 3 and 4 in two launches: coarse_new (the coarse box after its step)
 * is refluxed with fine_flux_base and its covered cells are averaged down
 * from fine_out_base. coarse_old is the coarse state the step started from
 * (F_c is recomputed from it), with opts' limiter, Riemann solver and floors
 * (opts->bc is ignored). dt from the host, or from *dt_dev when not NULL.
 * The recomputed face states pass through scratch memory of the plan (80
 * bytes per coarse-fine face, allocated by gd_amr_create), so two calls
 * with one plan in flight on different streams race. */
int gd_amr_reflux(gd_ctx *ctx, const gd_amr *plan, const gd_opts *opts, const void *coarse_old,
                  void *coarse_new, const void *fine_out_base, const void *fine_flux_base,
                  double gamma, double dt, const double *dt_dev, void *hip_stream);

/* Steps 1-4: ghost fill, coarse step (coarse_in -> coarse_out), batched
 * fine step (fine_in_base -> fine_out_base with fluxes into fine_flux_base),
 * refluxing and averaging down into coarse_out; five launches on
 * hip_stream, six with a host dt, which is first stored in a device scalar
 * of the plan. opts->bc is ignored. Calls with one plan in flight on
 * different streams race (the plan's dt scalar and reflux scratch). */
int gd_amr_step(gd_ctx *ctx, const gd_amr *plan, const gd_opts *opts, const void *coarse_in,
                void *coarse_out, void *fine_in_base, void *fine_out_base, void *fine_flux_base,
                double gamma, double dt, const double *dt_dev, void *hip_stream);

/* ------------------------------------------------------------ without allocation
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The batched
 * step of godunov_step_batched with no context and no library allocation:
 * its work queue, counters and work decomposition live in a static device
 * array of 786,504 bytes that the library's code object carries (each GPU
 * holds its own copy from the library's load until the process ends).
 *
 * patches_dev is a DEVICE array of npatch gd_patch records (owned by the
 * caller, read by the kernels at every launch -- so a captured graph reads
 * the records current at each replay); 1 <= npatch <= 65536, else GD_E_ARG.
 * Buffers, offsets and dt_dev as in godunov_step_batched; bflux_base may be
 * NULL. Results are bitwise those of godunov_step_batched (FP64 runs on 16x8
 * tiles, FP32 on 24x8 tiles, z-ranges of up to 32 planes). PLM limiters only
 * (GD_E_UNSUPPORTED for PPM); GD_GHOSTED only.
 *
 * Checks: the host checks opts, npatch, gamma and the pointers before
 * anything is launched (errors in gd_last_error(NULL)). The descriptors are
 * on the device, so the host cannot see them: a plan kernel checks each
 * record (extents 1..16384, 2 <= ng <= 64, dx > 0, dt >= 0 when dt_dev is
 * NULL, offsets >= 0, plane size below 2^31) and skips a failing patch,
 * whose output and flux blocks are then left untouched. Offsets beyond the
 * caller's buffers and overlapping blocks cannot be detected: the caller
 * must get them right, as the Python binding does with the host copy of
 * the table.
 *
 * Every call on a device shares that device's array (each call's first
 * launch clears what must start at zero): two calls in flight together on
 * one device, on the same or different streams, race; serialise them. */
int godunov_step_batched_noalloc(const gd_opts *opts, int npatch, const gd_patch *patches_dev,
                                 const void *u_in_base, void *u_out_base, void *bflux_base,
                                 const double *dt_dev, double gamma, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GODUNOV_H */
