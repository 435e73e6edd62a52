/*
 * godunov_oracle_adjoint.c -- plain FP64 reverse-mode adjoint of the oracle's
 * Godunov step, written by hand stage by stage.
 *
 * TEST INFRASTRUCTURE (see godunov_oracle.c, which this file includes so that
 * the forward recomputation is the oracle's own forward code).
 *
 * For a fixed time step dt, the step is a map U^n -> (U^{n+1}, bflux). Given
 * lam_out = dL/dU^{n+1} and optionally lam_bflux = dL/dbflux, this returns
 * lam_in = dL/dU^n in the layout of the input (ghost-cell adjoints included
 * in ghosted mode; folded onto the interior by the wrap in periodic mode).
 *
 * Non-smooth points (limiter branches, min/max of the wave speeds, the HLLC
 * region, floors) contribute the derivative of the branch the forward pass
 * took, with the forward's tie rules: an element of Clarke's generalised
 * gradient. Every reverse stage is a scatter in plain sequential loops.
 */
#include "godunov_oracle.c"

/* ------------------------------------------ adjoints of the flux helpers */

/* dE: E = p/(g-1) + rho (u^2+v^2+w^2)/2, rotated primitives. */
static void energy_adjoint(double g, const double W[5], double Eb, double Wb[5])
{
    double q2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
    Wb[4] += Eb / (g - 1.0);
    Wb[0] += Eb * 0.5 * q2;
    Wb[1] += Eb * W[0] * W[1];
    Wb[2] += Eb * W[0] * W[2];
    Wb[3] += Eb * W[0] * W[3];
}

static void euler_flux_adjoint(double g, const double W[5], const double Fb[5], double Wb[5])
{
    double rho = W[0], u = W[1], v = W[2], w = W[3], p = W[4];
    double E = total_energy(g, W);
    Wb[0] += Fb[0] * u;        Wb[1] += Fb[0] * rho;                       /* rho u        */
    Wb[0] += Fb[1] * u * u;    Wb[1] += Fb[1] * 2.0 * rho * u; Wb[4] += Fb[1]; /* rho u^2 + p */
    Wb[0] += Fb[2] * u * v;    Wb[1] += Fb[2] * rho * v; Wb[2] += Fb[2] * rho * u;
    Wb[0] += Fb[3] * u * w;    Wb[1] += Fb[3] * rho * w; Wb[3] += Fb[3] * rho * u;
    Wb[1] += Fb[4] * (E + p);  Wb[4] += Fb[4] * u;                         /* u (E + p)    */
    energy_adjoint(g, W, Fb[4] * u, Wb);
}

static void conserved_adjoint(double g, const double W[5], const double Ub[5], double Wb[5])
{
    Wb[0] += Ub[0];
    Wb[0] += Ub[1] * W[1]; Wb[1] += Ub[1] * W[0];
    Wb[0] += Ub[2] * W[2]; Wb[2] += Ub[2] * W[0];
    Wb[0] += Ub[3] * W[3]; Wb[3] += Ub[3] * W[0];
    energy_adjoint(g, W, Ub[4], Wb);
}

/* Reverse of davis_speeds: SLb, SRb -> Lb, Rb along the min/max branches. */
static void davis_speeds_adjoint(double g, const double L[5], const double R[5],
                                 double SLb, double SRb, double Lb[5], double Rb[5])
{
    double cL = sqrt(g * L[4] / L[0]), cR = sqrt(g * R[4] / R[0]);
    double cLb = 0.0, cRb = 0.0;
    if (L[1] - cL <= R[1] - cR) { Lb[1] += SLb; cLb -= SLb; }
    else { Rb[1] += SLb; cRb -= SLb; }
    if (L[1] + cL >= R[1] + cR) { Lb[1] += SRb; cLb += SRb; }
    else { Rb[1] += SRb; cRb += SRb; }
    /* c = sqrt(g p / rho): dc/dp = c/(2p), dc/drho = -c/(2 rho) */
    Lb[4] += cLb * cL / (2.0 * L[4]); Lb[0] -= cLb * cL / (2.0 * L[0]);
    Rb[4] += cRb * cR / (2.0 * R[4]); Rb[0] -= cRb * cR / (2.0 * R[0]);
}

static void hllc_flux_adjoint(double g, const double L[5], const double R[5],
                              const double Fb[5], double Lb[5], double Rb[5])
{
    double SL, SR;
    davis_speeds(g, L, R, &SL, &SR);
    double mL = L[0] * (SL - L[1]), mR = R[0] * (SR - R[1]);
    double num = R[4] - L[4] + mL * L[1] - mR * R[1];
    double den = mL - mR;
    double Sstar = num / den;

    if (SL >= 0.0) { euler_flux_adjoint(g, L, Fb, Lb); return; }
    int left;
    if (Sstar >= 0.0) left = 1;
    else if (SR > 0.0) left = 0;
    else { euler_flux_adjoint(g, R, Fb, Rb); return; }

    const double *K = left ? L : R;
    double *Kb = left ? Lb : Rb;
    double SK = left ? SL : SR, mK = left ? mL : mR;
    double FK[5], UK[5], Us[5];
    euler_flux(g, K, FK);
    conserved_of(g, K, UK);
    double a = mK / (SK - Sstar);
    double e = UK[4] / K[0] + (Sstar - K[1]) * (Sstar + K[4] / mK);
    Us[0] = a; Us[1] = a * Sstar; Us[2] = a * K[2]; Us[3] = a * K[3]; Us[4] = a * e;

    double SLb = 0.0, SRb = 0.0, Sstarb = 0.0, mLb = 0.0, mRb = 0.0, SKb = 0.0, mKb = 0.0;

    /* F = F(K) + S_K (U*_K - U_K) */
    double Usb[5], UKb[5];
    euler_flux_adjoint(g, K, Fb, Kb);
    for (int q = 0; q < 5; q++) {
        SKb += Fb[q] * (Us[q] - UK[q]);
        Usb[q] = SK * Fb[q];
        UKb[q] = -SK * Fb[q];
    }
    conserved_adjoint(g, K, UKb, Kb);

    /* U*_K = a (1, S*, v_K, w_K, e) */
    double ab = Usb[0] + Usb[1] * Sstar + Usb[2] * K[2] + Usb[3] * K[3] + Usb[4] * e;
    Sstarb += a * Usb[1];
    Kb[2] += a * Usb[2];
    Kb[3] += a * Usb[3];
    double eb = a * Usb[4];

    /* e = E_K/rho_K + (S* - u_K)(S* + p_K/m_K) */
    double t1 = Sstar - K[1], t2 = Sstar + K[4] / mK;
    energy_adjoint(g, K, eb / K[0], Kb);
    Kb[0] -= eb * UK[4] / (K[0] * K[0]);
    double t1b = eb * t2, t2b = eb * t1;
    Sstarb += t1b + t2b;
    Kb[1] -= t1b;
    Kb[4] += t2b / mK;
    mKb -= t2b * K[4] / (mK * mK);

    /* a = m_K / (S_K - S*) */
    double dd = SK - Sstar;
    mKb += ab / dd;
    double ddb = -ab * mK / (dd * dd);
    SKb += ddb;
    Sstarb -= ddb;

    if (left) { mLb += mKb; SLb += SKb; }
    else { mRb += mKb; SRb += SKb; }

    /* S* = num / den */
    double numb = Sstarb / den, denb = -Sstarb * Sstar / den;
    Rb[4] += numb; Lb[4] -= numb;
    mLb += numb * L[1]; Lb[1] += numb * mL;
    mRb -= numb * R[1]; Rb[1] -= numb * mR;
    mLb += denb; mRb -= denb;

    /* m_K = rho_K (S_K - u_K) */
    Lb[0] += mLb * (SL - L[1]); SLb += mLb * L[0]; Lb[1] -= mLb * L[0];
    Rb[0] += mRb * (SR - R[1]); SRb += mRb * R[0]; Rb[1] -= mRb * R[0];

    davis_speeds_adjoint(g, L, R, SLb, SRb, Lb, Rb);
}

static void hll_flux_adjoint(double g, const double L[5], const double R[5],
                             const double Fb[5], double Lb[5], double Rb[5])
{
    double SL, SR;
    davis_speeds(g, L, R, &SL, &SR);
    if (SL >= 0.0) { euler_flux_adjoint(g, L, Fb, Lb); return; }
    if (SR <= 0.0) { euler_flux_adjoint(g, R, Fb, Rb); return; }
    double FL[5], FR[5], UL[5], UR[5], F[5];
    euler_flux(g, L, FL); euler_flux(g, R, FR);
    conserved_of(g, L, UL); conserved_of(g, R, UR);
    double D = SR - SL;
    for (int q = 0; q < 5; q++) F[q] = (SR * FL[q] - SL * FR[q] + SL * SR * (UR[q] - UL[q])) / D;

    double Gb[5], FLb[5], FRb[5], ULb[5], URb[5], Db = 0.0, SLb = 0.0, SRb = 0.0;
    for (int q = 0; q < 5; q++) {
        Gb[q] = Fb[q] / D;
        Db -= Fb[q] * F[q] / D;
    }
    for (int q = 0; q < 5; q++) {
        FLb[q] = SR * Gb[q];
        FRb[q] = -SL * Gb[q];
        URb[q] = SL * SR * Gb[q];
        ULb[q] = -SL * SR * Gb[q];
        SRb += Gb[q] * FL[q] + SL * Gb[q] * (UR[q] - UL[q]);
        SLb += -Gb[q] * FR[q] + SR * Gb[q] * (UR[q] - UL[q]);
    }
    SRb += Db;
    SLb -= Db;
    euler_flux_adjoint(g, L, FLb, Lb);
    euler_flux_adjoint(g, R, FRb, Rb);
    conserved_adjoint(g, L, ULb, Lb);
    conserved_adjoint(g, R, URb, Rb);
    davis_speeds_adjoint(g, L, R, SLb, SRb, Lb, Rb);
}

/* Reverse of face_flux: Fb (unrotated) -> WLb, WRb (unrotated, accumulated). */
static void face_flux_adjoint(const orc_problem *P, int d, const double WL[5], const double WR[5],
                              const double Fb[5], double WLb[5], double WRb[5])
{
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    double L[5] = { WL[0], WL[1 + d], WL[1 + t1], WL[1 + t2], WL[4] };
    double R[5] = { WR[0], WR[1 + d], WR[1 + t1], WR[1 + t2], WR[4] };
    double Gb[5] = { Fb[0], Fb[1 + d], Fb[1 + t1], Fb[1 + t2], Fb[4] };
    double Lb[5] = { 0 }, Rb[5] = { 0 };
    if (P->riemann == RS_HLL) hll_flux_adjoint(P->gamma, L, R, Gb, Lb, Rb);
    else hllc_flux_adjoint(P->gamma, L, R, Gb, Lb, Rb);
    WLb[0] += Lb[0]; WLb[1 + d] += Lb[1]; WLb[1 + t1] += Lb[2]; WLb[1 + t2] += Lb[3]; WLb[4] += Lb[4];
    WRb[0] += Rb[0]; WRb[1 + d] += Rb[1]; WRb[1 + t1] += Rb[2]; WRb[1 + t2] += Rb[3]; WRb[4] += Rb[4];
}

/* Reverse of limited_slope: returns (ab, bb) for a slope adjoint sb. */
static void limited_slope_adjoint(int limiter, double a, double b, double sb, double *ab, double *bb)
{
    *ab = 0.0; *bb = 0.0;
    if (limiter == LIM_NONE) { *ab = 0.5 * sb; *bb = 0.5 * sb; return; }
    int same_sign = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
    if (!same_sign) return;
    if (limiter == LIM_MINMOD) {
        if (fabs(a) <= fabs(b)) *ab = sb; else *bb = sb;
        return;
    }
    /* MC: the same nested min as the forward; sign(a) = sign(b) = sign(a+b). */
    double m1 = 2.0 * fabs(a), m2 = 2.0 * fabs(b), m3 = 0.5 * fabs(a + b);
    int inner_is_m1 = m1 <= m2;
    double inner = inner_is_m1 ? m1 : m2;
    if (inner <= m3) {
        if (inner_is_m1) *ab = 2.0 * sb; else *bb = 2.0 * sb;
    } else {
        *ab = 0.5 * sb; *bb = 0.5 * sb;
    }
}

/* Reverse of hancock_predictor: Wsb -> Wb, Sb (accumulated). */
static void hancock_predictor_adjoint(const orc_problem *P, const double W[5], const double S[3][5],
                                      const double Wsb[5], double Wb[5], double Sb[3][5])
{
    double lam = P->dt / (2.0 * P->dx), g = P->gamma;
    double rho = W[0], vel[3] = { W[1], W[2], W[3] }, p = W[4];
    double divu = S[0][1] + S[1][2] + S[2][3];
    double velb[3] = { 0, 0, 0 }, divub = 0.0;
    double rb = Wsb[0], pb = Wsb[4];
    double mb[3] = { Wsb[1], Wsb[2], Wsb[3] };

    /* rho* = rho - lam (sum_d u_d drho_d + rho divu) */
    Wb[0] += rb * (1.0 - lam * divu);
    divub -= lam * rb * rho;
    for (int d = 0; d < 3; d++) { velb[d] -= lam * rb * S[d][0]; Sb[d][0] -= lam * rb * vel[d]; }

    /* u_m* = u_m - lam (sum_d u_d du_m,d + dp_m / rho), m = x, y, z */
    for (int m = 0; m < 3; m++) {
        velb[m] += mb[m];
        for (int d = 0; d < 3; d++) {
            velb[d] -= lam * mb[m] * S[d][1 + m];
            Sb[d][1 + m] -= lam * mb[m] * vel[d];
        }
        Sb[m][4] -= lam * mb[m] / rho;
        Wb[0] += lam * mb[m] * S[m][4] / (rho * rho);
    }

    /* p* = p - lam (sum_d u_d dp_d + g p divu) */
    Wb[4] += pb * (1.0 - lam * g * divu);
    divub -= lam * pb * g * p;
    for (int d = 0; d < 3; d++) { velb[d] -= lam * pb * S[d][4]; Sb[d][4] -= lam * pb * vel[d]; }

    /* divu = du_x + dv_y + dw_z */
    Sb[0][1] += divub; Sb[1][2] += divub; Sb[2][3] += divub;
    for (int d = 0; d < 3; d++) Wb[1 + d] += velb[d];
}

/* Reverse of conserved_to_primitive: Wb -> Ub (overwritten). */
static void primitive_adjoint(const orc_problem *P, const double U[5], const double Wb_in[5], double Ub[5])
{
    double g = P->gamma;
    int rho_floored = U[0] < P->rho_floor;
    double rho = rho_floored ? P->rho_floor : U[0];
    double vel[3] = { U[1] / rho, U[2] / rho, U[3] / rho };
    double kinetic = 0.5 * (U[1] * vel[0] + U[2] * vel[1] + U[3] * vel[2]);
    double p = (g - 1.0) * (U[4] - kinetic);
    int p_floored = p < P->p_floor;
    double pb = p_floored ? 0.0 : Wb_in[4];

    Ub[4] = (g - 1.0) * pb;
    double kb = -(g - 1.0) * pb;
    double rhob = Wb_in[0];
    for (int d = 0; d < 3; d++) {
        /* kinetic = (1/2) sum_d m_d vel_d, vel_d = m_d / rho */
        double velb = Wb_in[1 + d] + 0.5 * kb * U[1 + d];
        Ub[1 + d] = 0.5 * kb * vel[d] + velb / rho;
        rhob -= velb * vel[d] / rho;
    }
    Ub[0] = rho_floored ? 0.0 : rhob;
}

/* ------------------------------------------------------------- the step */

long orc_step_adjoint(const orc_problem *P, const double *u_in, const double *lam_out,
                      const double *lam_bflux, double *lam_in)
{
    if (check_problem(P) || !u_in || !lam_out || !lam_in) return -1;
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    ext_box B = { nx + 4, ny + 4, nz + 4 };
    size_t ncell = (size_t)B.ex * B.ey * B.ez;
    double *W = malloc(sizeof(double) * 5 * ncell);
    double *S = malloc(sizeof(double) * 15 * ncell);
    double *Ws = malloc(sizeof(double) * 5 * ncell);
    double *Wb = calloc(5 * ncell, sizeof(double));
    double *Sb = calloc(15 * ncell, sizeof(double));
    double *Wsb = calloc(5 * ncell, sizeof(double));
    if (!W || !S || !Ws || !Wb || !Sb || !Wsb) {
        free(W); free(S); free(Ws); free(Wb); free(Sb); free(Wsb);
        return -2;
    }
    long hits = 0;
    const int unit[3][3] = { { 1, 0, 0 }, { 0, 1, 0 }, { 0, 0, 1 } };

    /* forward recomputation of steps 1-3 */
    for (int k = -2; k < nz + 2; k++)
        for (int j = -2; j < ny + 2; j++)
            for (int i = -2; i < nx + 2; i++) {
                if (!cell_is_read(P, i, j, k)) continue;
                double U[5];
                for (int q = 0; q < 5; q++) U[q] = input_cell(P, u_in, q, i, j, k);
                conserved_to_primitive(P, U, W + 5 * ext_index(&B, i, j, k), &hits);
            }
    for (int k = -1; k < nz + 1; k++)
        for (int j = -1; j < ny + 1; j++)
            for (int i = -1; i < nx + 1; i++) {
                if (!cell_is_predicted(P, i, j, k)) continue;
                size_t c = ext_index(&B, i, j, k);
                double (*s)[5] = (double (*)[5])(S + 15 * c);
                for (int d = 0; d < 3; d++) {
                    size_t cm = ext_index(&B, i - unit[d][0], j - unit[d][1], k - unit[d][2]);
                    size_t cp = ext_index(&B, i + unit[d][0], j + unit[d][1], k + unit[d][2]);
                    for (int q = 0; q < 5; q++)
                        s[d][q] = limited_slope(P->limiter, W[5 * c + q] - W[5 * cm + q],
                                                W[5 * cp + q] - W[5 * c + q]);
                }
                hancock_predictor(P, W + 5 * c, s, Ws + 5 * c);
            }

    /* reverse of steps 6, 7, 5 and 4, face by face */
    const double cfac = P->dt / P->dx;
    size_t sheet[3] = { (size_t)5 * nz * ny, (size_t)5 * nz * nx, (size_t)5 * ny * nx };
    size_t sheet_off[6] = { 0, sheet[0], 2 * sheet[0], 2 * sheet[0] + sheet[1],
                            2 * sheet[0] + 2 * sheet[1], 2 * sheet[0] + 2 * sheet[1] + sheet[2] };
    for (int d = 0; d < 3; d++) {
        int fx = nx + (d == 0), fy = ny + (d == 1), fz = nz + (d == 2);
        for (int k = 0; k < fz; k++)
            for (int j = 0; j < fy; j++)
                for (int i = 0; i < fx; i++) {
                    int li = i - (d == 0), lj = j - (d == 1), lk = k - (d == 2);
                    int left_inside = li >= 0 && lj >= 0 && lk >= 0;
                    int right_inside = i < nx && j < ny && k < nz;
                    double Fb[5];
                    for (int q = 0; q < 5; q++) {
                        Fb[q] = 0.0;
                        if (right_inside) Fb[q] += cfac * lam_out[(((size_t)q * nz + k) * ny + j) * nx + i];
                        if (left_inside) Fb[q] -= cfac * lam_out[(((size_t)q * nz + lk) * ny + lj) * nx + li];
                    }
                    if (lam_bflux) {
                        /* face index along d: 0 is the minus sheet, n the plus sheet */
                        int fi = d == 0 ? i : (d == 1 ? j : k), n = d == 0 ? nx : (d == 1 ? ny : nz);
                        if (fi == 0 || fi == n) {
                            const double *sh = lam_bflux + sheet_off[2 * d + (fi == n)];
                            int b_slow = d == 2 ? j : k, b_fast = d == 0 ? j : i;
                            int n_slow = d == 2 ? ny : nz, n_fast = d == 0 ? ny : nx;
                            for (int q = 0; q < 5; q++)
                                Fb[q] += sh[((size_t)q * n_slow + b_slow) * n_fast + b_fast];
                        }
                    }
                    size_t cl = ext_index(&B, li, lj, lk), cr = ext_index(&B, i, j, k);
                    double WL[5], WR[5];
                    for (int q = 0; q < 5; q++) {
                        WL[q] = Ws[5 * cl + q] + 0.5 * S[15 * cl + 5 * d + q];
                        WR[q] = Ws[5 * cr + q] - 0.5 * S[15 * cr + 5 * d + q];
                    }
                    int rhoL_fl = WL[0] < P->rho_floor, pL_fl = WL[4] < P->p_floor;
                    int rhoR_fl = WR[0] < P->rho_floor, pR_fl = WR[4] < P->p_floor;
                    floor_state(P, WL, &hits);
                    floor_state(P, WR, &hits);
                    double WLb[5] = { 0 }, WRb[5] = { 0 };
                    face_flux_adjoint(P, d, WL, WR, Fb, WLb, WRb);
                    if (rhoL_fl) WLb[0] = 0.0;
                    if (pL_fl) WLb[4] = 0.0;
                    if (rhoR_fl) WRb[0] = 0.0;
                    if (pR_fl) WRb[4] = 0.0;
                    for (int q = 0; q < 5; q++) {
                        Wsb[5 * cl + q] += WLb[q];
                        Sb[15 * cl + 5 * d + q] += 0.5 * WLb[q];
                        Wsb[5 * cr + q] += WRb[q];
                        Sb[15 * cr + 5 * d + q] -= 0.5 * WRb[q];
                    }
                }
    }

    /* reverse of step 3, then step 2 */
    for (int k = -1; k < nz + 1; k++)
        for (int j = -1; j < ny + 1; j++)
            for (int i = -1; i < nx + 1; i++) {
                if (!cell_is_predicted(P, i, j, k)) continue;
                size_t c = ext_index(&B, i, j, k);
                hancock_predictor_adjoint(P, W + 5 * c, (const double (*)[5])(S + 15 * c),
                                          Wsb + 5 * c, Wb + 5 * c, (double (*)[5])(Sb + 15 * c));
            }
    for (int k = -1; k < nz + 1; k++)
        for (int j = -1; j < ny + 1; j++)
            for (int i = -1; i < nx + 1; i++) {
                if (!cell_is_predicted(P, i, j, k)) continue;
                size_t c = ext_index(&B, i, j, k);
                for (int d = 0; d < 3; d++) {
                    size_t cm = ext_index(&B, i - unit[d][0], j - unit[d][1], k - unit[d][2]);
                    size_t cp = ext_index(&B, i + unit[d][0], j + unit[d][1], k + unit[d][2]);
                    for (int q = 0; q < 5; q++) {
                        double a = W[5 * c + q] - W[5 * cm + q], b = W[5 * cp + q] - W[5 * c + q];
                        double ab, bb;
                        limited_slope_adjoint(P->limiter, a, b, Sb[15 * c + 5 * d + q], &ab, &bb);
                        Wb[5 * cm + q] -= ab;
                        Wb[5 * c + q] += ab - bb;
                        Wb[5 * cp + q] += bb;
                    }
                }
            }

    /* reverse of step 1 plus the identity term of step 6, into lam_in */
    size_t nin = P->periodic ? (size_t)nx * ny * nz
                             : (size_t)(nx + 2 * P->ng) * (ny + 2 * P->ng) * (nz + 2 * P->ng);
    memset(lam_in, 0, sizeof(double) * 5 * nin);
    for (int k = -2; k < nz + 2; k++)
        for (int j = -2; j < ny + 2; j++)
            for (int i = -2; i < nx + 2; i++) {
                if (!cell_is_read(P, i, j, k)) continue;
                size_t c = ext_index(&B, i, j, k);
                double U[5], Ub[5];
                for (int q = 0; q < 5; q++) U[q] = input_cell(P, u_in, q, i, j, k);
                primitive_adjoint(P, U, Wb + 5 * c, Ub);
                int inside = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
                for (int q = 0; q < 5; q++) {
                    double v = Ub[q];
                    if (inside) v += lam_out[(((size_t)q * nz + k) * ny + j) * nx + i];
                    lam_in[input_index(P, q, i, j, k)] += v;
                }
            }

    free(W); free(S); free(Ws); free(Wb); free(Sb); free(Wsb);
    return hits;
}
