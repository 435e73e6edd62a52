/*
 * godunov_oracle.c -- plain, slow FP64 CPU oracle for one unsplit
 * MUSCL-Hancock Godunov step of the 3-D Euler equations on one patch.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this code. It shares no code, header or
 * constant with the GPU library and the GPU library never calls it.
 *
 * What the paper fixes (Sec. 2, Sec. 3 and Sec. 4): the baryonic gas is an
 * ideal fluid obeying the Euler equations, integrated on the AMR mesh by a
 * Godunov-type finite-volume scheme of the piecewise-linear (PLM) family; the
 * GPU work unit is a compact patch of inner cells plus interpolated boundary
 * (ghost) cells; every face flux needed to update the patch is computed on the
 * device, and the fluxes through the patch boundary are handed back for the
 * coarse-fine flux correction of multilevel, adaptive-time-step runs.
 *
 * The paper prints no formulas. The concrete member of the PLM family is the
 * textbook unsplit MUSCL-Hancock scheme (van Leer 1979; Toro, "Riemann Solvers
 * and Numerical Methods for Fluid Dynamics", chapters 14 and 16), written out
 * in the steps below:
 *
 *   1. conserved -> primitive W = (rho, u, v, w, p), with density and
 *      pressure floors;
 *   2. undivided limited slopes of W in x, y and z (minmod, MC or none);
 *   3. Hancock half-step predictor in primitive quasi-linear form using all
 *      three directions (no transverse Riemann solves);
 *   4. face states W_L = W*_i + dW_i/2, W_R = W*_{i+1} - dW_{i+1}/2, floored;
 *   5. one Riemann flux per face: HLLC (Toro, Spruce & Speares 1994) or HLL
 *      (Harten, Lax & van Leer 1983), Davis (1988) wave-speed bounds;
 *   6. conservative update U' = U - dt/dx * sum_d (F_{d,+} - F_{d,-});
 *   7. boundary fluxes: the six sheets of face fluxes on the patch boundary,
 *      exactly as used in step 6;
 *   and the CFL signal speed max(|u|+|v|+|w|+3c) over the interior.
 *
 * Every stage is materialised in a full array over the patch plus two ghost
 * layers so that each step can be read against its formula; nothing is fused.
 *
 * The file is compiled twice: with `real` = double (the oracle proper) and
 * with `real` = double complex (-DORACLE_COMPLEX_STEP), which turns the same
 * forward code into a complex-step tangent-linear model (Squire & Trapp 1998):
 * every branch is decided on the real part, so Im f(x + i h v)/h is the
 * directional derivative along the branches the forward pass takes. The tests
 * use it to check the hand-written adjoint in godunov_oracle_adjoint.c.
 *
 * Layouts (all arrays C order, x fastest):
 *   ghosted input  u_in [5][nz+2ng][ny+2ng][nx+2ng], ng >= 2
 *   periodic input u_in [5][nz][ny][nx]  (neighbours wrap)
 *   output         u_out[5][nz][ny][nx]
 *   boundary flux  bflux = six sheets, in the order x-, x+, y-, y+, z-, z+;
 *                  x sheets [5][nz][ny], y sheets [5][nz][nx],
 *                  z sheets [5][ny][nx]; a sheet holds the face flux F_d
 *                  (positive = transport towards +d).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_COMPLEX_STEP
#include <complex.h>
typedef double complex real;
#define RE(x) creal(x)
#define r_sqrt(x) csqrt(x)
#define API(name) name##_cs
#else
typedef double real;
#define RE(x) (x)
#define r_sqrt(x) sqrt(x)
#define API(name) name
#endif

enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_NONE = 2 };
enum { RS_HLLC = 0, RS_HLL = 1 };

typedef struct {
    int nx, ny, nz;     /* interior extents */
    int ng;             /* ghost layers of a ghosted input (>= 2) */
    int periodic;       /* 1: input holds the interior only and wraps */
    int limiter;        /* LIM_* */
    int riemann;        /* RS_* */
    double gamma, dx, dt;
    double rho_floor, p_floor;
} orc_problem;

/* ---------------------------------------------------------------- helpers */

static real r_abs(real a) { return RE(a) < 0.0 ? -a : a; }
static real r_min(real a, real b) { return RE(a) <= RE(b) ? a : b; }
static real r_max(real a, real b) { return RE(a) >= RE(b) ? a : b; }

/* Work arrays cover the interior plus two layers: index i in [-2, n+2). */
typedef struct { int ex, ey, ez; } ext_box;

static size_t ext_index(const ext_box *b, int i, int j, int k)
{
    return ((size_t)(k + 2) * b->ey + (size_t)(j + 2)) * b->ex + (size_t)(i + 2);
}

static int depth_outside(int i, int n)
{
    if (i < 0) return -i;
    if (i >= n) return i - n + 1;
    return 0;
}

/* Cells the stencil reads: the interior, face ghosts up to depth 2 and edge
 * ghosts (two coordinates outside) at depth 1; corners are never read. */
static int cell_is_read(const orc_problem *P, int i, int j, int k)
{
    int di = depth_outside(i, P->nx), dj = depth_outside(j, P->ny), dk = depth_outside(k, P->nz);
    int nout = (di > 0) + (dj > 0) + (dk > 0);
    if (nout == 0) return 1;
    if (nout == 1) return di + dj + dk <= 2;
    if (nout == 2) return di <= 1 && dj <= 1 && dk <= 1;
    return 0;
}

/* Cells whose predicted state some face needs: the interior and the face
 * ghosts of depth 1. */
static int cell_is_predicted(const orc_problem *P, int i, int j, int k)
{
    int di = depth_outside(i, P->nx), dj = depth_outside(j, P->ny), dk = depth_outside(k, P->nz);
    return di + dj + dk <= 1;
}

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Position of conserved variable v of cell (i,j,k), i in [-2, nx+2) etc.,
 * in the input array (wrapped in periodic mode). */
static size_t input_index(const orc_problem *P, int v, int i, int j, int k)
{
    if (P->periodic)
        return (((size_t)v * P->nz + wrap(k, P->nz)) * P->ny + wrap(j, P->ny)) * P->nx
               + wrap(i, P->nx);
    int gx = P->nx + 2 * P->ng, gy = P->ny + 2 * P->ng, gz = P->nz + 2 * P->ng;
    return (((size_t)v * gz + (k + P->ng)) * gy + (j + P->ng)) * gx + (i + P->ng);
}

static real input_cell(const orc_problem *P, const real *u, int v, int i, int j, int k)
{
    return u[input_index(P, v, i, j, k)];
}

/* ------------------------------------------------ step 1: primitives */

/* W = (rho, u, v, w, p) from U = (rho, rho u, rho v, rho w, E) with
 * E = p/(gamma-1) + rho |u|^2 / 2. rho and p are raised to their floors. */
static void conserved_to_primitive(const orc_problem *P, const real U[5], real W[5], long *hits)
{
    real rho = U[0];
    if (RE(rho) < P->rho_floor) { rho = P->rho_floor; (*hits)++; }
    real u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
    real kinetic = 0.5 * (U[1] * u + U[2] * v + U[3] * w);
    real p = (P->gamma - 1.0) * (U[4] - kinetic);
    if (RE(p) < P->p_floor) { p = P->p_floor; (*hits)++; }
    W[0] = rho; W[1] = u; W[2] = v; W[3] = w; W[4] = p;
}

/* ------------------------------------------------ step 2: slopes */

/* a = q_i - q_{i-1}, b = q_{i+1} - q_i (undivided differences). */
static real limited_slope(int limiter, real a, real b)
{
    if (limiter == LIM_NONE) return 0.5 * (a + b);
    int same_sign = (RE(a) > 0.0 && RE(b) > 0.0) || (RE(a) < 0.0 && RE(b) < 0.0);
    if (!same_sign) return 0.0;
    if (limiter == LIM_MINMOD)
        return RE(r_abs(a)) <= RE(r_abs(b)) ? a : b;
    /* monotonised central: sign(a) min(2|a|, 2|b|, |a+b|/2) */
    real m = r_min(r_min(2.0 * r_abs(a), 2.0 * r_abs(b)), 0.5 * r_abs(a + b));
    return RE(a) > 0.0 ? m : -m;
}

/* ------------------------------------------------ step 3: predictor */

/* Half-step predictor in primitive form: W* = W - dt/(2 dx) sum_d A_d(W) dW_d
 * with A_d the Jacobian of the primitive Euler system along d.
 * S[d][q] is the slope of primitive q along direction d. */
static void hancock_predictor(const orc_problem *P, const real W[5], real S[3][5], real Ws[5])
{
    real lam = P->dt / (2.0 * P->dx);
    real rho = W[0], vel[3] = { W[1], W[2], W[3] }, p = W[4];
    real divu = S[0][1] + S[1][2] + S[2][3];
    real adv[5];
    for (int q = 0; q < 5; q++)
        adv[q] = vel[0] * S[0][q] + vel[1] * S[1][q] + vel[2] * S[2][q];
    Ws[0] = rho - lam * (adv[0] + rho * divu);
    Ws[1] = vel[0] - lam * (adv[1] + S[0][4] / rho);
    Ws[2] = vel[1] - lam * (adv[2] + S[1][4] / rho);
    Ws[3] = vel[2] - lam * (adv[3] + S[2][4] / rho);
    Ws[4] = p - lam * (adv[4] + P->gamma * p * divu);
}

/* ------------------------------------------------ step 4: face states */

static void floor_state(const orc_problem *P, real W[5], long *hits)
{
    if (RE(W[0]) < P->rho_floor) { W[0] = P->rho_floor; (*hits)++; }
    if (RE(W[4]) < P->p_floor) { W[4] = P->p_floor; (*hits)++; }
}

/* ------------------------------------------------ step 5: Riemann flux */

/* States here are rotated: W = (rho, u_n, u_t1, u_t2, p), u_n along the face
 * normal. */
static real total_energy(double gamma, const real W[5])
{
    return W[4] / (gamma - 1.0) + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

static void euler_flux(double gamma, const real W[5], real F[5])
{
    real E = total_energy(gamma, W);
    real mass = W[0] * W[1];
    F[0] = mass;
    F[1] = mass * W[1] + W[4];
    F[2] = mass * W[2];
    F[3] = mass * W[3];
    F[4] = W[1] * (E + W[4]);
}

static void conserved_of(double gamma, const real W[5], real U[5])
{
    U[0] = W[0];
    U[1] = W[0] * W[1];
    U[2] = W[0] * W[2];
    U[3] = W[0] * W[3];
    U[4] = total_energy(gamma, W);
}

/* Davis estimates of the slowest and fastest signal speeds. */
static void davis_speeds(double gamma, const real L[5], const real R[5], real *SL, real *SR)
{
    real cL = r_sqrt(gamma * L[4] / L[0]);
    real cR = r_sqrt(gamma * R[4] / R[0]);
    *SL = r_min(L[1] - cL, R[1] - cR);
    *SR = r_max(L[1] + cL, R[1] + cR);
}

static void hllc_flux(double gamma, const real L[5], const real R[5], real F[5])
{
    real SL, SR;
    davis_speeds(gamma, L, R, &SL, &SR);
    real mL = L[0] * (SL - L[1]);          /* rho_L (S_L - u_L) */
    real mR = R[0] * (SR - R[1]);
    real Sstar = (R[4] - L[4] + mL * L[1] - mR * R[1]) / (mL - mR);

    const real *K;
    real SK, mK;
    if (RE(SL) >= 0.0) { euler_flux(gamma, L, F); return; }
    if (RE(Sstar) >= 0.0) { K = L; SK = SL; mK = mL; }
    else if (RE(SR) > 0.0) { K = R; SK = SR; mK = mR; }
    else { euler_flux(gamma, R, F); return; }

    real FK[5], UK[5], Us[5];
    euler_flux(gamma, K, FK);
    conserved_of(gamma, K, UK);
    real a = mK / (SK - Sstar);
    Us[0] = a;
    Us[1] = a * Sstar;
    Us[2] = a * K[2];
    Us[3] = a * K[3];
    Us[4] = a * (UK[4] / K[0] + (Sstar - K[1]) * (Sstar + K[4] / mK));
    for (int q = 0; q < 5; q++) F[q] = FK[q] + SK * (Us[q] - UK[q]);
}

static void hll_flux(double gamma, const real L[5], const real R[5], real F[5])
{
    real SL, SR;
    davis_speeds(gamma, L, R, &SL, &SR);
    if (RE(SL) >= 0.0) { euler_flux(gamma, L, F); return; }
    if (RE(SR) <= 0.0) { euler_flux(gamma, R, F); return; }
    real FL[5], FR[5], UL[5], UR[5];
    euler_flux(gamma, L, FL);
    euler_flux(gamma, R, FR);
    conserved_of(gamma, L, UL);
    conserved_of(gamma, R, UR);
    for (int q = 0; q < 5; q++)
        F[q] = (SR * FL[q] - SL * FR[q] + SL * SR * (UR[q] - UL[q])) / (SR - SL);
}

/* Flux through a face normal to direction d from unrotated primitive states:
 * rotate so that the normal velocity comes first, solve, rotate back. */
static void face_flux(const orc_problem *P, int d, const real WL[5], const real WR[5], real F[5])
{
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    real L[5] = { WL[0], WL[1 + d], WL[1 + t1], WL[1 + t2], WL[4] };
    real R[5] = { WR[0], WR[1 + d], WR[1 + t1], WR[1 + t2], WR[4] };
    real G[5];
    if (P->riemann == RS_HLL) hll_flux(P->gamma, L, R, G);
    else hllc_flux(P->gamma, L, R, G);
    F[0] = G[0];
    F[1 + d] = G[1];
    F[1 + t1] = G[2];
    F[1 + t2] = G[3];
    F[4] = G[4];
}

/* ------------------------------------------------ the step */

static int check_problem(const orc_problem *P)
{
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return -1;
    if (!P->periodic && P->ng < 2) return -1;
    if (!(P->gamma > 1.0) || !(P->dx > 0.0) || !(P->dt >= 0.0)) return -1;
    if (P->limiter < 0 || P->limiter > 2 || P->riemann < 0 || P->riemann > 1) return -1;
    return 0;
}

/* One step. u_out may be NULL (fluxes only); bflux may be NULL.
 * Returns the number of floor applications, or -1 on a bad argument. */
long API(orc_step)(const orc_problem *P, const real *u_in, real *u_out, real *bflux)
{
    if (check_problem(P) || !u_in) return -1;
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    ext_box B = { nx + 4, ny + 4, nz + 4 };
    size_t ncell = (size_t)B.ex * B.ey * B.ez;
    real *W = malloc(sizeof(real) * 5 * ncell);        /* [cell][q] */
    real *S = malloc(sizeof(real) * 15 * ncell);       /* [cell][d][q] */
    real *Ws = malloc(sizeof(real) * 5 * ncell);       /* [cell][q] */
    size_t nfx = (size_t)(nx + 1) * ny * nz, nfy = (size_t)nx * (ny + 1) * nz,
           nfz = (size_t)nx * ny * (nz + 1);
    real *Fx = malloc(sizeof(real) * 5 * nfx);         /* [k][j][i'][q], face i'-1/2 */
    real *Fy = malloc(sizeof(real) * 5 * nfy);         /* [k][j'][i][q] */
    real *Fz = malloc(sizeof(real) * 5 * nfz);         /* [k'][j][i][q] */
    if (!W || !S || !Ws || !Fx || !Fy || !Fz) {
        free(W); free(S); free(Ws); free(Fx); free(Fy); free(Fz);
        return -2;
    }
    long hits = 0;

    /* step 1: primitives of every cell the stencil reads */
#pragma omp parallel for reduction(+ : hits) schedule(static)
    for (int k = -2; k < nz + 2; k++)
        for (int j = -2; j < ny + 2; j++)
            for (int i = -2; i < nx + 2; i++) {
                real *w = W + 5 * ext_index(&B, i, j, k);
                if (!cell_is_read(P, i, j, k)) {
                    for (int q = 0; q < 5; q++) w[q] = NAN;
                    continue;
                }
                real U[5];
                for (int q = 0; q < 5; q++) U[q] = input_cell(P, u_in, q, i, j, k);
                conserved_to_primitive(P, U, w, &hits);
            }

    /* steps 2 and 3: slopes in x, y, z and the predicted state */
#pragma omp parallel for schedule(static)
    for (int k = -1; k < nz + 1; k++)
        for (int j = -1; j < ny + 1; j++)
            for (int i = -1; i < nx + 1; i++) {
                if (!cell_is_predicted(P, i, j, k)) continue;
                size_t c = ext_index(&B, i, j, k);
                real (*s)[5] = (real (*)[5])(S + 15 * c);
                const int step[3][3] = { { 1, 0, 0 }, { 0, 1, 0 }, { 0, 0, 1 } };
                for (int d = 0; d < 3; d++) {
                    size_t cm = ext_index(&B, i - step[d][0], j - step[d][1], k - step[d][2]);
                    size_t cp = ext_index(&B, i + step[d][0], j + step[d][1], k + step[d][2]);
                    for (int q = 0; q < 5; q++)
                        s[d][q] = limited_slope(P->limiter, W[5 * c + q] - W[5 * cm + q],
                                                W[5 * cp + q] - W[5 * c + q]);
                }
                hancock_predictor(P, W + 5 * c, s, Ws + 5 * c);
            }

    /* steps 4 and 5: face states and one flux per face. Face (i'-1/2) along
     * d lies between cell i'-1 (left) and cell i' (right). */
    for (int d = 0; d < 3; d++) {
        int fx = nx + (d == 0), fy = ny + (d == 1), fz = nz + (d == 2);
        real *F = d == 0 ? Fx : (d == 1 ? Fy : Fz);
#pragma omp parallel for reduction(+ : hits) schedule(static)
        for (int k = 0; k < fz; k++)
            for (int j = 0; j < fy; j++)
                for (int i = 0; i < fx; i++) {
                    int li = i - (d == 0), lj = j - (d == 1), lk = k - (d == 2);
                    size_t cl = ext_index(&B, li, lj, lk), cr = ext_index(&B, i, j, k);
                    real WL[5], WR[5];
                    for (int q = 0; q < 5; q++) {
                        WL[q] = Ws[5 * cl + q] + 0.5 * S[15 * cl + 5 * d + q];
                        WR[q] = Ws[5 * cr + q] - 0.5 * S[15 * cr + 5 * d + q];
                    }
                    floor_state(P, WL, &hits);
                    floor_state(P, WR, &hits);
                    face_flux(P, d, WL, WR, F + 5 * (((size_t)k * fy + j) * fx + i));
                }
    }

    /* step 6: conservative update */
    if (u_out) {
        real c = P->dt / P->dx;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    const real *xm = Fx + 5 * (((size_t)k * ny + j) * (nx + 1) + i);
                    const real *xp = xm + 5;
                    const real *ym = Fy + 5 * (((size_t)k * (ny + 1) + j) * nx + i);
                    const real *yp = Fy + 5 * (((size_t)k * (ny + 1) + j + 1) * nx + i);
                    const real *zm = Fz + 5 * (((size_t)k * ny + j) * nx + i);
                    const real *zp = Fz + 5 * (((size_t)(k + 1) * ny + j) * nx + i);
                    for (int q = 0; q < 5; q++) {
                        real U = input_cell(P, u_in, q, i, j, k);
                        real div = ((xp[q] - xm[q]) + (yp[q] - ym[q])) + (zp[q] - zm[q]);
                        u_out[(((size_t)q * nz + k) * ny + j) * nx + i] = U - c * div;
                    }
                }
    }

    /* step 7: boundary-face fluxes */
    if (bflux) {
        size_t sx = (size_t)5 * nz * ny, sy = (size_t)5 * nz * nx, sz = (size_t)5 * ny * nx;
        real *bxm = bflux, *bxp = bxm + sx, *bym = bxp + sx, *byp = bym + sy,
             *bzm = byp + sy, *bzp = bzm + sz;
        for (int q = 0; q < 5; q++)
            for (int k = 0; k < nz; k++)
                for (int j = 0; j < ny; j++) {
                    size_t o = ((size_t)q * nz + k) * ny + j;
                    bxm[o] = Fx[5 * (((size_t)k * ny + j) * (nx + 1) + 0) + q];
                    bxp[o] = Fx[5 * (((size_t)k * ny + j) * (nx + 1) + nx) + q];
                }
        for (int q = 0; q < 5; q++)
            for (int k = 0; k < nz; k++)
                for (int i = 0; i < nx; i++) {
                    size_t o = ((size_t)q * nz + k) * nx + i;
                    bym[o] = Fy[5 * (((size_t)k * (ny + 1) + 0) * nx + i) + q];
                    byp[o] = Fy[5 * (((size_t)k * (ny + 1) + ny) * nx + i) + q];
                }
        for (int q = 0; q < 5; q++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t o = ((size_t)q * ny + j) * nx + i;
                    bzm[o] = Fz[5 * (((size_t)0 * ny + j) * nx + i) + q];
                    bzp[o] = Fz[5 * (((size_t)nz * ny + j) * nx + i) + q];
                }
    }

    free(W); free(S); free(Ws); free(Fx); free(Fy); free(Fz);
    return hits;
}

/* CFL signal speed: max over interior cells of |u| + |v| + |w| + 3c, with c
 * the sound speed of the floored primitive state. The stable step of the
 * unsplit scheme is dt = C dx / s with Courant number C. */
double API(orc_max_signal)(const orc_problem *P, const real *u_in)
{
    if (check_problem(P) || !u_in) return -1.0;
    double smax = 0.0;
#pragma omp parallel for reduction(max : smax) schedule(static)
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                real U[5], W[5];
                long hits = 0;
                for (int q = 0; q < 5; q++) U[q] = input_cell(P, u_in, q, i, j, k);
                conserved_to_primitive(P, U, W, &hits);
                double c = sqrt(P->gamma * RE(W[4]) / RE(W[0]));
                double s = fabs(RE(W[1])) + fabs(RE(W[2])) + fabs(RE(W[3])) + 3.0 * c;
                if (s > smax) smax = s;
            }
    return smax;
}

/* Single-face flux, exposed so the tests can probe step 5 directly.
 * d = 0, 1, 2 picks the face normal; states are unrotated primitives. */
void API(orc_face_flux)(const orc_problem *P, int d, const real *WL, const real *WR, real *F)
{
    face_flux(P, d, WL, WR, F);
}

/* Single-cell conversion, exposed for the round-trip test. */
long API(orc_primitive)(const orc_problem *P, const real *U, real *W)
{
    long hits = 0;
    conserved_to_primitive(P, U, W, &hits);
    return hits;
}
