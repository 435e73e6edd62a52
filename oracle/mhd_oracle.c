/*
 * Plain FP64 CPU oracle of one unsplit MUSCL-Hancock step of ideal
 * magnetohydrodynamics with hyperbolic divergence cleaning, on a periodic box.
 *
 * TEST INFRASTRUCTURE: only tests/ may load the library built from this file;
 * the GPU path shares no code with it.
 *
 * The paper's flagship GPU solver is Enzo's MHD code (Sec. 2, Sec. 4); it
 * names the method family but prints no formulas. The concrete scheme here:
 *
 *   conserved U = (rho, rho u, rho v, rho w, E, Bx, By, Bz, psi), with
 *     E = p/(gamma-1) + rho |u|^2 / 2 + |B|^2 / 2   (units with mu0 = 1)
 *   primitive W = (rho, u, v, w, p, Bx, By, Bz, psi), rho floored before the
 *     division, p floored after it;
 *   flux along d: the ideal-MHD flux with total pressure pT = p + |B|^2/2,
 *     plus the generalised-Lagrange-multiplier (GLM) cleaning terms of
 *     Dedner et al. (2002): the flux of B_d is psi and the flux of psi is
 *     ch^2 B_d;
 *   reconstruction: undivided limited slopes of W (minmod, MC or unlimited);
 *   predictor: the conservative MUSCL-Hancock half step (Toro, Sec. 14.4):
 *     the states at the upper and lower faces of a cell along each axis,
 *     W +- S_d/2, move by the same increment
 *     dU = -dt/(2dx) sum_d [F_d(W + S_d/2) - F_d(W - S_d/2)];
 *   face flux: the 2x2 GLM Riemann problem for (B_n, psi) gives
 *     B_n* = (B_nL + B_nR)/2 - (psi_R - psi_L)/(2 ch) and
 *     psi* = (psi_L + psi_R)/2 - ch (B_nR - B_nL)/2;
 *     B_n* is then the normal field of both sides of the HLLD solver of
 *     Miyoshi & Kusano (2005), with S_L = min(u_L - cf_L, u_R - cf_R),
 *     S_R = max(u_L + cf_L, u_R + cf_R) (cf the fast magnetosonic speed);
 *   update: U' = U - dt/dx [((dF_x + dF_y) + dF_z)], then the parabolic
 *     damping psi' <- psi' exp(-alpha ch dt/dx).
 *
 * Layout: [9][nz][ny][nx], x fastest; neighbours wrap.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NV 9

typedef struct {
    int nx, ny, nz;
    int limiter;            /* 0 minmod, 1 MC, 2 unlimited */
    double gamma, dx, dt;
    double ch;              /* cleaning wave speed */
    double alpha;           /* parabolic damping: psi *= exp(-alpha ch dt / dx) */
    double rho_floor, p_floor;
} mhd_problem;

static double min2(double a, double b) { return a < b ? a : b; }
static double max2(double a, double b) { return a > b ? a : b; }

/* limited undivided slope from the one-sided differences a = q_i - q_{i-1}
 * and b = q_{i+1} - q_i; ties take a */
static double limited_slope(int lim, double a, double b)
{
    if (lim == 2) return 0.5 * (a + b);
    if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return 0.0;
    if (lim == 0) return fabs(a) <= fabs(b) ? a : b;
    double m = min2(min2(2.0 * fabs(a), 2.0 * fabs(b)), 0.5 * fabs(a + b));
    return a > 0.0 ? m : -m;
}

/* conserved -> primitive; returns the number of floors applied */
static int cons_to_prim(const mhd_problem *P, const double *U, double *W)
{
    int hits = 0;
    double rho = U[0];
    if (rho < P->rho_floor) { rho = P->rho_floor; ++hits; }
    double u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
    double kin = 0.5 * (U[1] * u + U[2] * v + U[3] * w);
    double mag = 0.5 * (U[5] * U[5] + U[6] * U[6] + U[7] * U[7]);
    double p = (P->gamma - 1.0) * (U[4] - kin - mag);
    if (p < P->p_floor) { p = P->p_floor; ++hits; }
    W[0] = rho; W[1] = u; W[2] = v; W[3] = w; W[4] = p;
    W[5] = U[5]; W[6] = U[6]; W[7] = U[7]; W[8] = U[8];
    return hits;
}

static void prim_to_cons(const mhd_problem *P, const double *W, double *U)
{
    double rho = W[0];
    U[0] = rho;
    U[1] = rho * W[1]; U[2] = rho * W[2]; U[3] = rho * W[3];
    U[4] = W[4] / (P->gamma - 1.0) + 0.5 * rho * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3])
         + 0.5 * (W[5] * W[5] + W[6] * W[6] + W[7] * W[7]);
    U[5] = W[5]; U[6] = W[6]; U[7] = W[7]; U[8] = W[8];
}

/* fast magnetosonic speed along axis d of the primitive state W */
static double fast_speed(const mhd_problem *P, const double *W, int d)
{
    double a2 = P->gamma * W[4] / W[0];
    double b2 = (W[5] * W[5] + W[6] * W[6] + W[7] * W[7]) / W[0];
    double bn2 = W[5 + d] * W[5 + d] / W[0];
    double s = a2 + b2;
    double disc = s * s - 4.0 * a2 * bn2;
    if (disc < 0.0) disc = 0.0;
    return sqrt(0.5 * (s + sqrt(disc)));
}

/* physical flux along axis d of the GLM-MHD system */
static void phys_flux(const mhd_problem *P, const double *W, int d, double *F)
{
    double rho = W[0], p = W[4];
    const double *vel = W + 1, *B = W + 5;
    double un = vel[d], Bn = B[d];
    double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    double pT = p + 0.5 * B2;
    double uB = vel[0] * B[0] + vel[1] * B[1] + vel[2] * B[2];
    double E = p / (P->gamma - 1.0) + 0.5 * rho * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2])
             + 0.5 * B2;
    F[0] = rho * un;
    for (int k = 0; k < 3; ++k)
        F[1 + k] = rho * un * vel[k] - Bn * B[k] + (k == d ? pT : 0.0);
    F[4] = (E + pT) * un - Bn * uB;
    for (int k = 0; k < 3; ++k)
        F[5 + k] = (k == d) ? W[8] : un * B[k] - vel[k] * Bn;
    F[8] = P->ch * P->ch * Bn;
}

/* HLLD flux (Miyoshi & Kusano 2005) in the frame of the face: L and R are
 * (rho, u_n, u_t1, u_t2, p, Bn, B_t1, B_t2) with the same Bn on both sides;
 * returns the fluxes of (rho, m_n, m_t1, m_t2, E, B_t1, B_t2) in F[0..6]. */
static void hlld(const mhd_problem *P, const double *L, const double *R, double *F)
{
    const double g = P->gamma, Bn = L[5];
    const double sgn = Bn > 0.0 ? 1.0 : (Bn < 0.0 ? -1.0 : 0.0);
    double UL[8], UR[8], FL[7], FR[7], pTL, pTR;
    /* conserved state and flux of each side */
    for (int s = 0; s < 2; ++s) {
        const double *W = s ? R : L;
        double *U = s ? UR : UL, *Fs = s ? FR : FL;
        double rho = W[0], u = W[1], v = W[2], w = W[3], p = W[4], By = W[6], Bz = W[7];
        double B2 = Bn * Bn + By * By + Bz * Bz;
        double pT = p + 0.5 * B2;
        double E = p / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w) + 0.5 * B2;
        double uB = u * Bn + v * By + w * Bz;
        U[0] = rho; U[1] = rho * u; U[2] = rho * v; U[3] = rho * w; U[4] = E;
        U[5] = Bn; U[6] = By; U[7] = Bz;
        Fs[0] = rho * u;
        Fs[1] = rho * u * u + pT - Bn * Bn;
        Fs[2] = rho * u * v - Bn * By;
        Fs[3] = rho * u * w - Bn * Bz;
        Fs[4] = (E + pT) * u - Bn * uB;
        Fs[5] = u * By - v * Bn;
        Fs[6] = u * Bz - w * Bn;
        if (s) pTR = pT; else pTL = pT;
    }
    /* fast speeds along the face normal */
    double cfL, cfR;
    {
        double WL[9] = { L[0], L[1], L[2], L[3], L[4], L[5], L[6], L[7], 0.0 };
        double WR[9] = { R[0], R[1], R[2], R[3], R[4], R[5], R[6], R[7], 0.0 };
        cfL = fast_speed(P, WL, 0);
        cfR = fast_speed(P, WR, 0);
    }
    const double SL = min2(L[1] - cfL, R[1] - cfR);
    const double SR = max2(L[1] + cfL, R[1] + cfR);
    if (SL >= 0.0) { memcpy(F, FL, sizeof(FL)); return; }
    if (SR <= 0.0) { memcpy(F, FR, sizeof(FR)); return; }

    /* contact speed and total pressure of the star region */
    const double dL = (SL - L[1]) * L[0], dR = (SR - R[1]) * R[0];
    const double SM = (dR * R[1] - dL * L[1] - pTR + pTL) / (dR - dL);
    const double pTs = (dR * pTL - dL * pTR + dL * dR * (R[1] - L[1])) / (dR - dL);

    /* single-star states */
    double Us[2][8], sqr[2];
    for (int s = 0; s < 2; ++s) {
        const double *W = s ? R : L;
        const double *U = s ? UR : UL;
        const double S = s ? SR : SL;
        double rho = W[0], u = W[1], v = W[2], w = W[3], By = W[6], Bz = W[7];
        double pT = s ? pTR : pTL;
        double rs = rho * (S - u) / (S - SM);
        double den = rho * (S - u) * (S - SM) - Bn * Bn;
        double vs, ws, Bys, Bzs;
        if (fabs(den) <= 1e-12 * (rho * (S - u) * (S - u) + Bn * Bn)) {
            /* degenerate: the Alfven and fast waves coincide */
            vs = v; ws = w; Bys = By; Bzs = Bz;
        } else {
            double t = Bn * (SM - u) / den;
            vs = v - By * t;
            ws = w - Bz * t;
            double q = (rho * (S - u) * (S - u) - Bn * Bn) / den;
            Bys = By * q;
            Bzs = Bz * q;
        }
        double uB = u * Bn + v * By + w * Bz;
        double uBs = SM * Bn + vs * Bys + ws * Bzs;
        double Es = ((S - u) * U[4] - pT * u + pTs * SM + Bn * (uB - uBs)) / (S - SM);
        Us[s][0] = rs; Us[s][1] = rs * SM; Us[s][2] = rs * vs; Us[s][3] = rs * ws;
        Us[s][4] = Es; Us[s][5] = Bn; Us[s][6] = Bys; Us[s][7] = Bzs;
        sqr[s] = sqrt(rs);
    }
    const double SLs = SM - fabs(Bn) / sqr[0];
    const double SRs = SM + fabs(Bn) / sqr[1];

    /* F*_K = F_K + S_K (U*_K - U_K) */
    double FsL[7], FsR[7];
    for (int q = 0; q < 7; ++q) {
        int c = q < 5 ? q : q + 1;
        FsL[q] = FL[q] + SL * (Us[0][c] - UL[c]);
        FsR[q] = FR[q] + SR * (Us[1][c] - UR[c]);
    }
    if (SLs >= 0.0) { memcpy(F, FsL, sizeof(FsL)); return; }
    if (SRs <= 0.0 && !(SM >= 0.0)) {
        /* right of the right Alfven wave */
        memcpy(F, FsR, sizeof(FsR));
        return;
    }

    /* double-star states (between the Alfven waves) */
    const double vL = Us[0][2] / Us[0][0], wL = Us[0][3] / Us[0][0];
    const double vR = Us[1][2] / Us[1][0], wR = Us[1][3] / Us[1][0];
    const double ByL = Us[0][6], BzL = Us[0][7], ByR = Us[1][6], BzR = Us[1][7];
    const double ss = sqr[0] + sqr[1];
    const double vss = (sqr[0] * vL + sqr[1] * vR + (ByR - ByL) * sgn) / ss;
    const double wss = (sqr[0] * wL + sqr[1] * wR + (BzR - BzL) * sgn) / ss;
    const double Byss = (sqr[0] * ByR + sqr[1] * ByL + sqr[0] * sqr[1] * (vR - vL) * sgn) / ss;
    const double Bzss = (sqr[0] * BzR + sqr[1] * BzL + sqr[0] * sqr[1] * (wR - wL) * sgn) / ss;
    const double uBss = SM * Bn + vss * Byss + wss * Bzss;
    if (SM >= 0.0) {
        const double uBs = SM * Bn + vL * ByL + wL * BzL;
        double Uss[8] = { Us[0][0], Us[0][0] * SM, Us[0][0] * vss, Us[0][0] * wss,
                          Us[0][4] - sqr[0] * (uBs - uBss) * sgn, Bn, Byss, Bzss };
        for (int q = 0; q < 7; ++q) {
            int c = q < 5 ? q : q + 1;
            F[q] = FsL[q] + SLs * (Uss[c] - Us[0][c]);
        }
    } else {
        const double uBs = SM * Bn + vR * ByR + wR * BzR;
        double Uss[8] = { Us[1][0], Us[1][0] * SM, Us[1][0] * vss, Us[1][0] * wss,
                          Us[1][4] + sqr[1] * (uBs - uBss) * sgn, Bn, Byss, Bzss };
        for (int q = 0; q < 7; ++q) {
            int c = q < 5 ? q : q + 1;
            F[q] = FsR[q] + SRs * (Uss[c] - Us[1][c]);
        }
    }
}

/* flux through a face normal to axis d from the unrotated primitive states
 * on its two sides (GLM for B_n and psi, HLLD for the rest) */
void mhd_face_flux(const mhd_problem *P, int d, const double *WL, const double *WR, double *F)
{
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    const double ch = P->ch;
    const double Bns = 0.5 * (WL[5 + d] + WR[5 + d]) - (WR[8] - WL[8]) / (2.0 * ch);
    const double psis = 0.5 * (WL[8] + WR[8]) - 0.5 * ch * (WR[5 + d] - WL[5 + d]);
    double L[8] = { WL[0], WL[1 + d], WL[1 + t1], WL[1 + t2], WL[4], Bns, WL[5 + t1], WL[5 + t2] };
    double R[8] = { WR[0], WR[1 + d], WR[1 + t1], WR[1 + t2], WR[4], Bns, WR[5 + t1], WR[5 + t2] };
    double Fr[7];
    hlld(P, L, R, Fr);
    F[0] = Fr[0];
    F[1 + d] = Fr[1]; F[1 + t1] = Fr[2]; F[1 + t2] = Fr[3];
    F[4] = Fr[4];
    F[5 + d] = psis; F[5 + t1] = Fr[5]; F[5 + t2] = Fr[6];
    F[8] = ch * ch * Bns;
}

void mhd_phys_flux(const mhd_problem *P, int d, const double *W, double *F) { phys_flux(P, W, d, F); }
double mhd_fast_speed(const mhd_problem *P, int d, const double *W) { return fast_speed(P, W, d); }
int mhd_primitive(const mhd_problem *P, const double *U, double *W) { return cons_to_prim(P, U, W); }

static size_t cell(const mhd_problem *P, int i, int j, int k)
{
    i = ((i % P->nx) + P->nx) % P->nx;
    j = ((j % P->ny) + P->ny) % P->ny;
    k = ((k % P->nz) + P->nz) % P->nz;
    return ((size_t)k * P->ny + j) * P->nx + i;
}

/* One step; returns the number of floors applied, or -1 for bad arguments. */
long mhd_step(const mhd_problem *P, const double *u_in, double *u_out)
{
    if (P->nx < 1 || P->ny < 1 || P->nz < 1 || !(P->ch > 0.0)) return -1;
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const size_t n = (size_t)nx * ny * nz;
    double *W = malloc(sizeof(double) * NV * n);        /* primitives, [cell][q] */
    double *Wp = malloc(sizeof(double) * 3 * NV * n);   /* predicted upper-face state, [cell][d][q] */
    double *Wm = malloc(sizeof(double) * 3 * NV * n);   /* predicted lower-face state */
    double *Fx = malloc(sizeof(double) * 3 * NV * n);   /* flux through the lower face, [cell][d][q] */
    if (!W || !Wp || !Wm || !Fx) { free(W); free(Wp); free(Wm); free(Fx); return -1; }
    long hits = 0;

    /* 1. primitives */
#pragma omp parallel for reduction(+ : hits)
    for (size_t c = 0; c < n; ++c) {
        double U[NV];
        for (int q = 0; q < NV; ++q) U[q] = u_in[q * n + c];
        hits += cons_to_prim(P, U, W + NV * c);
    }

    /* 2.-3. slopes, face values and the conservative half step */
#pragma omp parallel for collapse(2) reduction(+ : hits)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = cell(P, i, j, k);
                const double *w = W + NV * c;
                double up[3][NV], dn[3][NV], dU[NV];
                for (int q = 0; q < NV; ++q) dU[q] = 0.0;
                for (int d = 0; d < 3; ++d) {
                    const size_t cm = cell(P, i - (d == 0), j - (d == 1), k - (d == 2));
                    const size_t cp = cell(P, i + (d == 0), j + (d == 1), k + (d == 2));
                    for (int q = 0; q < NV; ++q) {
                        double s = limited_slope(P->limiter, w[q] - W[NV * cm + q],
                                                 W[NV * cp + q] - w[q]);
                        up[d][q] = w[q] + 0.5 * s;
                        dn[d][q] = w[q] - 0.5 * s;
                    }
                    /* the extrapolated density and pressure keep the floors */
                    up[d][0] = max2(up[d][0], P->rho_floor); dn[d][0] = max2(dn[d][0], P->rho_floor);
                    up[d][4] = max2(up[d][4], P->p_floor); dn[d][4] = max2(dn[d][4], P->p_floor);
                    double Fu[NV], Fd[NV];
                    phys_flux(P, up[d], d, Fu);
                    phys_flux(P, dn[d], d, Fd);
                    for (int q = 0; q < NV; ++q) dU[q] -= Fu[q] - Fd[q];
                }
                const double h = P->dt / (2.0 * P->dx);
                for (int d = 0; d < 3; ++d) {
                    double Uu[NV], Ud[NV];
                    prim_to_cons(P, up[d], Uu);
                    prim_to_cons(P, dn[d], Ud);
                    for (int q = 0; q < NV; ++q) { Uu[q] += h * dU[q]; Ud[q] += h * dU[q]; }
                    hits += cons_to_prim(P, Uu, Wp + NV * (3 * c + d));
                    hits += cons_to_prim(P, Ud, Wm + NV * (3 * c + d));
                }
            }

    /* 4. the flux through the lower face of every cell along each axis */
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = cell(P, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    const size_t cl = cell(P, i - (d == 0), j - (d == 1), k - (d == 2));
                    mhd_face_flux(P, d, Wp + NV * (3 * cl + d), Wm + NV * (3 * c + d),
                                  Fx + NV * (3 * c + d));
                }
            }

    /* 5. conservative update, then the damping of psi */
    const double c_dx = P->dt / P->dx;
    const double damp = exp(-P->alpha * P->ch * P->dt / P->dx);
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = cell(P, i, j, k);
                const size_t cx = cell(P, i + 1, j, k), cy = cell(P, i, j + 1, k),
                             cz = cell(P, i, j, k + 1);
                for (int q = 0; q < NV; ++q) {
                    double dFx = Fx[NV * (3 * cx + 0) + q] - Fx[NV * (3 * c + 0) + q];
                    double dFy = Fx[NV * (3 * cy + 1) + q] - Fx[NV * (3 * c + 1) + q];
                    double dFz = Fx[NV * (3 * cz + 2) + q] - Fx[NV * (3 * c + 2) + q];
                    u_out[q * n + c] = u_in[q * n + c] - c_dx * ((dFx + dFy) + dFz);
                }
                u_out[8 * n + c] *= damp;
            }
    free(W); free(Wp); free(Wm); free(Fx);
    return hits;
}

/* max over cells of sum_d (|u_d| + cf_d) (the CFL signal speed of the
 * unsplit step) and of max_d (|u_d| + cf_d) */
void mhd_max_speeds(const mhd_problem *P, const double *u, double *sum_max, double *dir_max)
{
    const size_t n = (size_t)P->nx * P->ny * P->nz;
    double smax = 0.0, dmax = 0.0;
#pragma omp parallel for reduction(max : smax, dmax)
    for (size_t c = 0; c < n; ++c) {
        double U[NV], W[NV];
        for (int q = 0; q < NV; ++q) U[q] = u[q * n + c];
        cons_to_prim(P, U, W);
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            double v = fabs(W[1 + d]) + fast_speed(P, W, d);
            s += v;
            if (v > dmax) dmax = v;
        }
        if (s > smax) smax = s;
    }
    *sum_max = smax;
    *dir_max = dmax;
}
