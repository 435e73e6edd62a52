/*
 * ppm_oracle.c -- plain FP64 CPU oracle of one unsplit Godunov step of the
 * 3-D Euler equations with piecewise-parabolic (PPM) reconstruction.
 *
 * TEST INFRASTRUCTURE, like the rest of oracle/: only the test suite loads
 * it; the GPU library never does, and the two share no code.
 *
 * The paper names PPM beside PLM and TVD as the reconstructions of the codes'
 * Godunov solvers (Sec. 2; Enzo's hydro solver, Sec. 4) and prints no
 * formulas. The step is the MUSCL-Hancock step of godunov_oracle.c (whose
 * primitive conversion, Hancock predictor, floors, Riemann solvers and update
 * this file reuses) with its reconstruction replaced by the parabola of
 * Colella & Woodward (1984, section 1), built per axis and per primitive
 * variable q from the cell values a_i:
 *
 *   1. slopes: da_i = MC-limited difference of a_{i-1}, a_i, a_{i+1}
 *      (zero unless a_i is between its neighbours, else
 *      sign * min(|a_{i+1} - a_{i-1}|/2, 2|a_i - a_{i-1}|, 2|a_{i+1} - a_i|));
 *      for the unlimited variant da_i = (a_{i+1} - a_{i-1})/2;
 *   2. interface value between cells i and i+1:
 *      a_{i+1/2} = (a_i + a_{i+1})/2 - (da_{i+1} - da_i)/6, evaluated once
 *      from (a_{i-1}, a_i, a_{i+1}, a_{i+2}), so the two cells of a face
 *      see the same value; a_L,i = a_{i-1/2}, a_R,i = a_{i+1/2};
 *   3. (limited variant only) monotonicity, with D = a_R - a_L and
 *      m = a_i - (a_L + a_R)/2:
 *        (a_R - a_i)(a_i - a_L) <= 0  ->  a_L = a_R = a_i   (local extremum)
 *        else D m >  D^2/6             ->  a_L = 3 a_i - 2 a_R
 *        else D m < -D^2/6             ->  a_R = 3 a_i - 2 a_L;
 *   4. the Hancock half step of the PLM scheme with the slopes
 *      dW_d = a_R,d - a_L,d: W* = W - dt/(2dx) sum_d A_d(W) dW_d;
 *   5. face states W*_i + (a_R,i - W_i) on the upper face along d and
 *      W*_i + (a_L,i - W_i) on the lower face, floored. With a_R,L = W +- S/2
 *      these are the PLM face states.
 * No contact steepening and no flattening.
 *
 * With characteristic tracing (limiter GD_PPM_CT, or GD_PPM_CT_UNLIMITED with
 * the unlimited parabola), steps 4 and 5 become, per axis d and cell:
 *   4'. the waves of the primitive system along d at the cell's state,
 *       speeds u_d - c, u_d (entropy and the two shear waves), u_d + c, with
 *       Courant numbers s = speed dt/dx; for the upper face, each wave with
 *       s > 0 contributes l . (A(s) - a_R) r, where A(s) is the average of
 *       the parabola over the last s of the cell (Colella & Woodward's
 *       domain of dependence of the face over the half step's time average),
 *         A(s) - a_R = -(s/2) (a_R - a_L - (1 - 2s/3) a_6),
 *         a_6 = 6 (a - (a_L + a_R)/2),
 *       and l, r the left and right eigenvectors of the wave; the face state
 *       is a_R plus these contributions (for the lower face, waves with
 *       s < 0 over the first |s| of the cell, with
 *         A(s) - a_L = (|s|/2) (a_R - a_L + (1 - 2|s|/3) a_6));
 *       eigenvectors in (rho, u_n, u_t1, u_t2, p):
 *         r_-+ = (1, -+c/rho, 0, 0, c^2), l_-+ = (0, -+rho/(2c), 0, 0, 1/(2c^2)),
 *         entropy r = l' = (1, 0, 0, 0, 0) with l = (1, 0, 0, 0, -1/c^2),
 *         shear r = l = the unit vectors of u_t1 and u_t2;
 *   5'. plus the transverse terms of the Hancock half step,
 *       -dt/(2dx) sum_{d' != d} A_d'(W) (a_R,d' - a_L,d'), then floored.
 * The reference state is the edge value, not the average over the fastest
 * wave's domain: a face state then changes continuously when a wave speed
 * crosses zero. For a linear profile with every wave moving towards the
 * face the traced state is the Hancock state W* + S_d/2.
 *
 * The stencil: the cells whose face states some face needs are the interior
 * and the face ghosts of depth 1; each reads two cells either side along
 * each axis. A ghosted input needs ng >= 3 and the step reads face ghosts to
 * depth 3 and edge ghosts at depths (1, <= 2); corners never.
 */
#include "godunov_oracle.c"

enum { LIM_PPM = 3, LIM_PPM_NONE = 4, LIM_PPM_CT = 5, LIM_PPM_CT_NONE = 6 };

/* The parabola construction of a limiter value: limited or unlimited. */
static int ppm_parabola(int limiter)
{
    return limiter == LIM_PPM_NONE || limiter == LIM_PPM_CT_NONE ? LIM_PPM_NONE : LIM_PPM;
}

static int ppm_traced(int limiter) { return limiter == LIM_PPM_CT || limiter == LIM_PPM_CT_NONE; }

/* Work arrays cover the interior plus three layers: index in [-3, n+3). */
static size_t ext3_index(const ext_box *b, int i, int j, int k)
{
    return ((size_t)(k + 3) * b->ey + (size_t)(j + 3)) * b->ex + (size_t)(i + 3);
}

/* The interior and the face ghosts of depth 1. */
static int ppm_predicted(const orc_problem *P, int i, int j, int k)
{
    return depth_outside(i, P->nx) + depth_outside(j, P->ny) + depth_outside(k, P->nz) <= 1;
}

/* Cells within two steps along one axis of a predicted cell. */
static int ppm_read(const orc_problem *P, int i, int j, int k)
{
    if (ppm_predicted(P, i, j, k)) return 1;
    for (int m = -2; m <= 2; m++) {
        if (m == 0) continue;
        if (ppm_predicted(P, i + m, j, k) || ppm_predicted(P, i, j + m, k) ||
            ppm_predicted(P, i, j, k + m))
            return 1;
    }
    return 0;
}

static size_t ppm_input_index(const orc_problem *P, int v, int i, int j, int k)
{
    if (P->periodic)
        return (((size_t)v * P->nz + wrap(k, P->nz)) * P->ny + wrap(j, P->ny)) * P->nx
               + wrap(i, P->nx);
    int gx = P->nx + 2 * P->ng, gy = P->ny + 2 * P->ng, gz = P->nz + 2 * P->ng;
    return (((size_t)v * gz + (k + P->ng)) * gy + (j + P->ng)) * gx + (i + P->ng);
}

/* Slope of the parabola construction (step 1). */
static real ppm_slope(int limiter, real am, real a0, real ap)
{
    if (limiter == LIM_PPM_NONE) return 0.5 * (ap - am);
    return limited_slope(LIM_MC, a0 - am, ap - a0);
}

/* Interface value between the cells holding a0 and ap (step 2). */
static real ppm_interface(int limiter, real am, real a0, real ap, real app)
{
    real d0 = ppm_slope(limiter, am, a0, ap);
    real d1 = ppm_slope(limiter, a0, ap, app);
    return 0.5 * (a0 + ap) - (d1 - d0) / 6.0;
}

/* Edge values of the parabola of the cell holding a0 (steps 2 and 3). */
static void ppm_edges(int limiter, real amm, real am, real a0, real ap, real app, real *aL,
                      real *aR)
{
    real l = ppm_interface(limiter, amm, am, a0, ap);
    real r = ppm_interface(limiter, am, a0, ap, app);
    if (limiter == LIM_PPM) {
        if (RE((r - a0) * (a0 - l)) <= 0.0) {
            l = a0;
            r = a0;
        } else {
            real D = r - l, m = a0 - 0.5 * (l + r);
            if (RE(D * m) > RE(D * D / 6.0)) l = 3.0 * a0 - 2.0 * r;
            else if (RE(-(D * D) / 6.0) > RE(D * m)) r = 3.0 * a0 - 2.0 * l;
        }
    }
    *aL = l;
    *aR = r;
}

/* The parabola's average over the last s of the cell minus a_R (upper edge,
 * s > 0) or over the first |s| of the cell minus a_L (lower edge, s < 0). */
static real ppm_average_minus_edge(real aL, real aR, real a0, real s, int upper)
{
    real da = aR - aL, a6 = 6.0 * (a0 - 0.5 * (aL + aR));
    if (upper) return -0.5 * s * (da - (1.0 - 2.0 * s / 3.0) * a6);
    real t = -s;
    return 0.5 * t * (da + (1.0 - 2.0 * t / 3.0) * a6);
}

/* Step 4': the traced state on the upper (upper = 1) or lower face of a
 * cell along d, before the transverse terms. */
static void ppm_trace(const orc_problem *P, const real W[5], const real aL[5], const real aR[5],
                      int d, int upper, real out[5])
{
    int n = 1 + d, t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
    real rho = W[0], p = W[4], un = W[n];
    real c = r_sqrt(P->gamma * p / rho);
    real cfl = P->dt / P->dx;
    real s[3] = { (un - c) * cfl, un * cfl, (un + c) * cfl };
    for (int q = 0; q < 5; q++) out[q] = upper ? aR[q] : aL[q];
    for (int w = 0; w < 3; w++) {
        if (upper ? !(RE(s[w]) > 0.0) : !(RE(s[w]) < 0.0)) continue;
        real D[5];
        for (int q = 0; q < 5; q++) D[q] = ppm_average_minus_edge(aL[q], aR[q], W[q], s[w], upper);
        if (w == 1) {
            /* entropy and shear waves */
            out[0] += D[0] - D[4] / (c * c);
            out[t1] += D[t1];
            out[t2] += D[t2];
        } else {
            real sg = w == 0 ? -1.0 : 1.0;
            real beta = sg * rho / (2.0 * c) * D[n] + D[4] / (2.0 * c * c);
            out[0] += beta;
            out[n] += sg * c / rho * beta;
            out[4] += c * c * beta;
        }
    }
}

static int check_ppm_problem(const orc_problem *P)
{
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return -1;
    if (!P->periodic && P->ng < 3) return -1;
    if (!(P->gamma > 1.0) || !(P->dx > 0.0) || !(P->dt >= 0.0)) return -1;
    if (P->limiter < LIM_PPM || P->limiter > LIM_PPM_CT_NONE) return -1;
    if (P->riemann < 0 || P->riemann > 1) return -1;
    return 0;
}

/* One step; the layouts and the boundary-flux sheets of orc_step. Returns the
 * number of floor applications, -1 on a bad argument. */
long API(orc_step_ppm)(const orc_problem *P, const real *u_in, real *u_out, real *bflux)
{
    if (check_ppm_problem(P) || !u_in) return -1;
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    ext_box B = { nx + 6, ny + 6, nz + 6 };
    size_t ncell = (size_t)B.ex * B.ey * B.ez;
    real *W = malloc(sizeof(real) * 5 * ncell);        /* [cell][q] */
    real *E = malloc(sizeof(real) * 30 * ncell);       /* [cell][d][side L,R][q] */
    real *Ws = malloc(sizeof(real) * 5 * ncell);       /* [cell][q] */
    size_t nfx = (size_t)(nx + 1) * ny * nz, nfy = (size_t)nx * (ny + 1) * nz,
           nfz = (size_t)nx * ny * (nz + 1);
    real *Fx = malloc(sizeof(real) * 5 * nfx);
    real *Fy = malloc(sizeof(real) * 5 * nfy);
    real *Fz = malloc(sizeof(real) * 5 * nfz);
    if (!W || !E || !Ws || !Fx || !Fy || !Fz) {
        free(W); free(E); free(Ws); free(Fx); free(Fy); free(Fz);
        return -2;
    }
    long hits = 0;

    /* primitives of every cell the stencil reads */
#pragma omp parallel for reduction(+ : hits) schedule(static)
    for (int k = -3; k < nz + 3; k++)
        for (int j = -3; j < ny + 3; j++)
            for (int i = -3; i < nx + 3; i++) {
                real *w = W + 5 * ext3_index(&B, i, j, k);
                if (!ppm_read(P, i, j, k)) {
                    for (int q = 0; q < 5; q++) w[q] = NAN;
                    continue;
                }
                real U[5];
                for (int q = 0; q < 5; q++) U[q] = u_in[ppm_input_index(P, q, i, j, k)];
                conserved_to_primitive(P, U, w, &hits);
            }

    /* parabola edges along each axis, slopes a_R - a_L, predicted state */
#pragma omp parallel for schedule(static)
    for (int k = -1; k < nz + 1; k++)
        for (int j = -1; j < ny + 1; j++)
            for (int i = -1; i < nx + 1; i++) {
                if (!ppm_predicted(P, i, j, k)) continue;
                size_t c = ext3_index(&B, i, j, k);
                real *e = E + 30 * c;
                real s[3][5];
                for (int d = 0; d < 3; d++) {
                    int di = d == 0, dj = d == 1, dk = d == 2;
                    size_t cmm = ext3_index(&B, i - 2 * di, j - 2 * dj, k - 2 * dk);
                    size_t cm = ext3_index(&B, i - di, j - dj, k - dk);
                    size_t cp = ext3_index(&B, i + di, j + dj, k + dk);
                    size_t cpp = ext3_index(&B, i + 2 * di, j + 2 * dj, k + 2 * dk);
                    for (int q = 0; q < 5; q++) {
                        real aL, aR;
                        ppm_edges(ppm_parabola(P->limiter), W[5 * cmm + q], W[5 * cm + q],
                                  W[5 * c + q], W[5 * cp + q], W[5 * cpp + q], &aL, &aR);
                        e[10 * d + q] = aL;
                        e[10 * d + 5 + q] = aR;
                        s[d][q] = aR - aL;
                    }
                }
                hancock_predictor(P, W + 5 * c, s, Ws + 5 * c);
                if (ppm_traced(P->limiter)) {
                    /* steps 4' and 5': the six traced face states, stored in
                     * place of the edges (FS[d][side]: lower, upper) */
                    real fs[3][2][5];
                    for (int d = 0; d < 3; d++) {
                        real st[3][5], Wt[5];
                        for (int dd = 0; dd < 3; dd++)
                            for (int q = 0; q < 5; q++) st[dd][q] = dd == d ? 0.0 : s[dd][q];
                        hancock_predictor(P, W + 5 * c, st, Wt);
                        for (int side = 0; side < 2; side++) {
                            ppm_trace(P, W + 5 * c, e + 10 * d, e + 10 * d + 5, d, side, fs[d][side]);
                            for (int q = 0; q < 5; q++) fs[d][side][q] += Wt[q] - W[5 * c + q];
                        }
                    }
                    for (int d = 0; d < 3; d++)
                        for (int side = 0; side < 2; side++)
                            for (int q = 0; q < 5; q++) e[10 * d + 5 * side + q] = fs[d][side][q];
                }
            }

    /* face states and one flux per face; face (i'-1/2) along d lies between
     * cell i'-1 (left, its upper edge) and cell i' (right, its lower edge) */
    for (int d = 0; d < 3; d++) {
        int fx = nx + (d == 0), fy = ny + (d == 1), fz = nz + (d == 2);
        real *F = d == 0 ? Fx : (d == 1 ? Fy : Fz);
#pragma omp parallel for reduction(+ : hits) schedule(static)
        for (int k = 0; k < fz; k++)
            for (int j = 0; j < fy; j++)
                for (int i = 0; i < fx; i++) {
                    int li = i - (d == 0), lj = j - (d == 1), lk = k - (d == 2);
                    size_t cl = ext3_index(&B, li, lj, lk), cr = ext3_index(&B, i, j, k);
                    real WL[5], WR[5];
                    for (int q = 0; q < 5; q++) {
                        if (ppm_traced(P->limiter)) {
                            WL[q] = E[30 * cl + 10 * d + 5 + q];
                            WR[q] = E[30 * cr + 10 * d + q];
                        } else {
                            WL[q] = Ws[5 * cl + q] + (E[30 * cl + 10 * d + 5 + q] - W[5 * cl + q]);
                            WR[q] = Ws[5 * cr + q] + (E[30 * cr + 10 * d + q] - W[5 * cr + q]);
                        }
                    }
                    floor_state(P, WL, &hits);
                    floor_state(P, WR, &hits);
                    face_flux(P, d, WL, WR, F + 5 * (((size_t)k * fy + j) * fx + i));
                }
    }

    /* conservative update, grouped as in orc_step */
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
                        real U = u_in[ppm_input_index(P, q, i, j, k)];
                        real div = ((xp[q] - xm[q]) + (yp[q] - ym[q])) + (zp[q] - zm[q]);
                        u_out[(((size_t)q * nz + k) * ny + j) * nx + i] = U - c * div;
                    }
                }
    }

    /* boundary-face fluxes, sheets as in orc_step */
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

    free(W); free(E); free(Ws); free(Fx); free(Fy); free(Fz);
    return hits;
}

/* Step 4' for one cell, exposed for the tests: W the cell's primitive state,
 * aL, aR the parabola edges of its five primitives along axis d, upper = 1
 * for the upper face; P supplies gamma, dt and dx. */
void API(orc_ppm_trace)(const orc_problem *P, const real *W, const real *aL, const real *aR,
                        int d, int upper, real *out)
{
    ppm_trace(P, W, aL, aR, d, upper, out);
}

/* Edge values of one parabola, exposed for the tests. */
void API(orc_ppm_edges)(int limiter, const real *a5, real *aL, real *aR)
{
    ppm_edges(limiter, a5[0], a5[1], a5[2], a5[3], a5[4], aL, aR);
}
