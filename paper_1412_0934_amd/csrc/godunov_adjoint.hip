// Reverse-mode adjoint of the Godunov step (gfx950, FP64), for a fixed dt.
//
// The step is U -> U' = U - dt/dx sum_faces (signed F), with every face flux
// F(W_L, W_R) a function of the predicted states of its two cells, each of
// which depends on the primitive state of the cell and its limited slopes.
// The adjoint runs the chain backwards in gather form -- every output value
// is a sum written by exactly one thread, in a fixed order, with no atomics
// -- so it is bitwise deterministic. Five kernels share a scratch area laid
// out over the extended box [-2, n+2)^3 (x fastest):
//   1 prim    primitives W of every cell the forward stencil reads
//   2 slopes  slopes S and predicted state W* of every predicted cell
//   3 faces   per computed face: dL/dF = dt/dx (lam_right - lam_left)
//             (+ dL/dbflux on the patch boundary), reversed through the
//             Riemann solver and the face-state floors -> dL/dW_L, dL/dW_R
//   4 cells   per predicted cell: gather the adjoints of its face states,
//             reverse the predictor, split each slope adjoint into the parts
//             along its two one-sided differences
//   5 input   per input cell: gather dL/dW from its own predictor and the
//             slope splits of itself and its neighbours, reverse the
//             primitive conversion, add the identity term lam_out; in a
//             periodic box the images of a cell in the extended box are
//             folded onto it.
// At kinks (limiter switches, min/max of wave speeds, the HLLC region and the
// floors) the derivative of the branch the forward step takes is used, with
// the forward step's tie rules.
#include "godunov_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

namespace adj {

enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_NONE = 2 };
enum { RS_HLLC = 0, RS_HLL = 1 };

struct Geo {
    int nx, ny, nz, ng, periodic;
    int ex, ey, ez;            // extended box n + 4
    int64_t E;                 // cells of the extended box
    int64_t vin;               // input variable stride
    int gx, gy;                // input row / plane extents
    int64_t nf[3];             // computed faces per direction
    double gamma, rho_floor, p_floor, lam, c;   // lam = dt/(2dx), c = dt/dx
};

struct Scratch {
    double *W;      // [5][E]
    double *S;      // [15][E], index d*5+q
    double *Ws;     // [5][E]
    double *FL[3];  // [5][nf[d]] adjoint of the left face state
    double *FR[3];  // [5][nf[d]]
    double *Wd;     // [5][E] direct part of dL/dW from the predictor
    double *SA;     // [15][E] slope adjoint split along a = q_i - q_{i-1}
    double *SB;     // [15][E] ... along b = q_{i+1} - q_i
};

__device__ __forceinline__ int depth_out(int i, int n) { return i < 0 ? -i : (i >= n ? i - n + 1 : 0); }

__device__ __forceinline__ bool is_read(const Geo &g, int i, int j, int k)
{
    int di = depth_out(i, g.nx), dj = depth_out(j, g.ny), dk = depth_out(k, g.nz);
    int nout = (di > 0) + (dj > 0) + (dk > 0);
    if (nout == 0) return true;
    if (nout == 1) return di + dj + dk <= 2;
    if (nout == 2) return di <= 1 && dj <= 1 && dk <= 1;
    return false;
}

__device__ __forceinline__ bool is_predicted(const Geo &g, int i, int j, int k)
{
    return depth_out(i, g.nx) + depth_out(j, g.ny) + depth_out(k, g.nz) <= 1;
}

__device__ __forceinline__ int64_t ext(const Geo &g, int i, int j, int k)
{
    return ((int64_t)(k + 2) * g.ey + (j + 2)) * g.ex + (i + 2);
}

__device__ __forceinline__ void ext_coords(const Geo &g, int64_t e, int &i, int &j, int &k)
{
    i = (int)(e % g.ex) - 2;
    int64_t r = e / g.ex;
    j = (int)(r % g.ey) - 2;
    k = (int)(r / g.ey) - 2;
}

__device__ __forceinline__ int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }

// position of cell (i, j, k) of the extended box in the input array
__device__ __forceinline__ int64_t in_index(const Geo &g, int i, int j, int k)
{
    if (g.periodic) {
        i = wrap(i, g.nx); j = wrap(j, g.ny); k = wrap(k, g.nz);
        return ((int64_t)k * g.ny + j) * g.nx + i;
    }
    return ((int64_t)(k + g.ng) * g.gy + (j + g.ng)) * g.gx + (i + g.ng);
}

__device__ __forceinline__ int64_t interior_index(const Geo &g, int i, int j, int k)
{
    return ((int64_t)k * g.ny + j) * g.nx + i;
}

// Conserved -> primitive with floors; reports which floors were applied.
__device__ __forceinline__ void to_prim(const Geo &g, const double U[5], double W[5], bool &rho_fl,
                                        bool &p_fl)
{
    double rho = U[0];
    rho_fl = rho < g.rho_floor;
    if (rho_fl) rho = g.rho_floor;
    double u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
    double kin = 0.5 * (U[1] * u + U[2] * v + U[3] * w);
    double p = (g.gamma - 1.0) * (U[4] - kin);
    p_fl = p < g.p_floor;
    if (p_fl) p = g.p_floor;
    W[0] = rho; W[1] = u; W[2] = v; W[3] = w; W[4] = p;
}

template <int LIM>
__device__ __forceinline__ double slope(double a, double b)
{
    if (LIM == LIM_NONE) return 0.5 * (a + b);
    bool same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
    if (!same) return 0.0;
    if (LIM == LIM_MINMOD) return fabs(a) <= fabs(b) ? a : b;
    double m1 = 2.0 * fabs(a), m2 = 2.0 * fabs(b), m3 = 0.5 * fabs(a + b);
    double m = m1 <= m2 ? m1 : m2;
    m = m <= m3 ? m : m3;
    return a > 0.0 ? m : -m;
}

// d slope / d a and d slope / d b on the branch the forward takes
template <int LIM>
__device__ __forceinline__ void slope_partials(double a, double b, double &pa, double &pb)
{
    pa = 0.0; pb = 0.0;
    if (LIM == LIM_NONE) { pa = 0.5; pb = 0.5; return; }
    bool same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
    if (!same) return;
    if (LIM == LIM_MINMOD) {
        if (fabs(a) <= fabs(b)) pa = 1.0; else pb = 1.0;
        return;
    }
    double m1 = 2.0 * fabs(a), m2 = 2.0 * fabs(b), m3 = 0.5 * fabs(a + b);
    bool first = m1 <= m2;
    double m = first ? m1 : m2;
    if (m <= m3) { if (first) pa = 2.0; else pb = 2.0; }
    else { pa = 0.5; pb = 0.5; }
}

// ------------------------------------------------------------ 1: primitives

__global__ __launch_bounds__(256) void k_prim(Geo g, const double *__restrict__ u, Scratch s)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.E;
         e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        ext_coords(g, e, i, j, k);
        if (!is_read(g, i, j, k)) continue;
        int64_t p = in_index(g, i, j, k);
        double U[5], W[5];
        for (int q = 0; q < 5; ++q) U[q] = u[p + q * g.vin];
        bool rf, pf;
        to_prim(g, U, W, rf, pf);
        for (int q = 0; q < 5; ++q) s.W[q * g.E + e] = W[q];
    }
}

// ------------------------------------------------------------ 2: slopes, W*

template <int LIM>
__global__ __launch_bounds__(256) void k_slopes(Geo g, Scratch s)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.E;
         e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        ext_coords(g, e, i, j, k);
        if (!is_predicted(g, i, j, k)) continue;
        const int64_t st[3] = { 1, g.ex, (int64_t)g.ex * g.ey };
        double W[5], S[3][5];
        for (int q = 0; q < 5; ++q) W[q] = s.W[q * g.E + e];
        for (int d = 0; d < 3; ++d)
            for (int q = 0; q < 5; ++q) {
                double wm = s.W[q * g.E + e - st[d]], wp = s.W[q * g.E + e + st[d]];
                S[d][q] = slope<LIM>(W[q] - wm, wp - W[q]);
                s.S[(d * 5 + q) * g.E + e] = S[d][q];
            }
        double divu = S[0][1] + S[1][2] + S[2][3];
        double adv[5];
        for (int q = 0; q < 5; ++q) adv[q] = W[1] * S[0][q] + W[2] * S[1][q] + W[3] * S[2][q];
        double Ws[5];
        Ws[0] = W[0] - g.lam * (adv[0] + W[0] * divu);
        Ws[1] = W[1] - g.lam * (adv[1] + S[0][4] / W[0]);
        Ws[2] = W[2] - g.lam * (adv[2] + S[1][4] / W[0]);
        Ws[3] = W[3] - g.lam * (adv[3] + S[2][4] / W[0]);
        Ws[4] = W[4] - g.lam * (adv[4] + g.gamma * W[4] * divu);
        for (int q = 0; q < 5; ++q) s.Ws[q * g.E + e] = Ws[q];
    }
}

// ------------------------------------------------------------ 3: faces

// Forward quantities of the HLLC / HLL flux in rotated form, kept for the
// reverse sweep.
struct Fwd {
    double cL, cR, SL, SR, mL, mR, num, den, Sst;
    bool slL, srL;      // S_L took the left candidate, S_R the left candidate
};

__device__ __forceinline__ void speeds(double g, const double L[5], const double R[5], Fwd &f)
{
    f.cL = sqrt(g * L[4] / L[0]);
    f.cR = sqrt(g * R[4] / R[0]);
    double a = L[1] - f.cL, b = R[1] - f.cR;
    f.slL = a <= b;
    f.SL = f.slL ? a : b;
    double c = L[1] + f.cL, d = R[1] + f.cR;
    f.srL = c >= d;
    f.SR = f.srL ? c : d;
}

__device__ __forceinline__ void speeds_adjoint(double g, const double L[5], const double R[5],
                                               const Fwd &f, double SLb, double SRb, double Lb[5],
                                               double Rb[5])
{
    double cLb = 0.0, cRb = 0.0;
    if (f.slL) { Lb[1] += SLb; cLb -= SLb; } else { Rb[1] += SLb; cRb -= SLb; }
    if (f.srL) { Lb[1] += SRb; cLb += SRb; } else { Rb[1] += SRb; cRb += SRb; }
    // c = sqrt(g p / rho): dc = c/2 (dp/p - drho/rho)
    Lb[4] += 0.5 * cLb * f.cL / L[4];
    Lb[0] -= 0.5 * cLb * f.cL / L[0];
    Rb[4] += 0.5 * cRb * f.cR / R[4];
    Rb[0] -= 0.5 * cRb * f.cR / R[0];
    (void)g;
}

// Adjoint of the physical flux and of the conserved vector of a rotated
// primitive state W, accumulated into Wb: Fb . dF/dW + Ub . dU/dW.
__device__ __forceinline__ void flux_cons_adjoint(double g, const double W[5], const double Fb[5],
                                                  const double Ub[5], double Wb[5])
{
    const double r = W[0], u = W[1], v = W[2], w = W[3], p = W[4];
    const double q2 = u * u + v * v + w * w;
    const double E = p / (g - 1.0) + 0.5 * r * q2;
    // energy adjoint collected from F4 = u (E + p) and U4 = E
    double Eb = Fb[4] * u + Ub[4];
    // F0 = r u, F1 = r u^2 + p, F2 = r u v, F3 = r u w, F4 = u (E + p)
    Wb[0] += Fb[0] * u + Fb[1] * u * u + Fb[2] * u * v + Fb[3] * u * w;
    Wb[1] += Fb[0] * r + 2.0 * Fb[1] * r * u + Fb[2] * r * v + Fb[3] * r * w + Fb[4] * (E + p);
    Wb[2] += Fb[2] * r * u;
    Wb[3] += Fb[3] * r * u;
    Wb[4] += Fb[1] + Fb[4] * u;
    // U0 = r, U1 = r u, U2 = r v, U3 = r w
    Wb[0] += Ub[0] + Ub[1] * u + Ub[2] * v + Ub[3] * w;
    Wb[1] += Ub[1] * r;
    Wb[2] += Ub[2] * r;
    Wb[3] += Ub[3] * r;
    // E = p/(g-1) + r q2 / 2
    Wb[0] += Eb * 0.5 * q2;
    Wb[1] += Eb * r * u;
    Wb[2] += Eb * r * v;
    Wb[3] += Eb * r * w;
    Wb[4] += Eb / (g - 1.0);
}

__device__ __forceinline__ void phys_flux(double g, const double W[5], double F[5], double U[5])
{
    const double r = W[0], u = W[1], v = W[2], w = W[3], p = W[4];
    const double E = p / (g - 1.0) + 0.5 * r * (u * u + v * v + w * w);
    F[0] = r * u; F[1] = r * u * u + p; F[2] = r * u * v; F[3] = r * u * w; F[4] = u * (E + p);
    U[0] = r; U[1] = r * u; U[2] = r * v; U[3] = r * w; U[4] = E;
}

__device__ void hllc_adjoint(double g, const double L[5], const double R[5], const double Fb[5],
                             double Lb[5], double Rb[5])
{
    Fwd f;
    speeds(g, L, R, f);
    f.mL = L[0] * (f.SL - L[1]);
    f.mR = R[0] * (f.SR - R[1]);
    f.num = R[4] - L[4] + f.mL * L[1] - f.mR * R[1];
    f.den = f.mL - f.mR;
    f.Sst = f.num / f.den;
    const double zero[5] = { 0, 0, 0, 0, 0 };
    if (f.SL >= 0.0) { flux_cons_adjoint(g, L, Fb, zero, Lb); return; }
    bool left;
    if (f.Sst >= 0.0) left = true;
    else if (f.SR > 0.0) left = false;
    else { flux_cons_adjoint(g, R, Fb, zero, Rb); return; }

    const double *K = left ? L : R;
    double *Kb = left ? Lb : Rb;
    const double SK = left ? f.SL : f.SR, mK = left ? f.mL : f.mR;
    double FK[5], UK[5];
    phys_flux(g, K, FK, UK);
    const double d = SK - f.Sst;
    const double a = mK / d;
    const double t1 = f.Sst - K[1], t2 = f.Sst + K[4] / mK;
    const double e = UK[4] / K[0] + t1 * t2;
    const double Us[5] = { a, a * f.Sst, a * K[2], a * K[3], a * e };

    // F = F_K + S_K (U* - U_K)
    double SKb = 0.0, UKb[5], Usb[5];
    for (int q = 0; q < 5; ++q) {
        SKb += Fb[q] * (Us[q] - UK[q]);
        Usb[q] = SK * Fb[q];
        UKb[q] = -SK * Fb[q];
    }
    // U* = a (1, S*, v, w, e)
    double ab = Usb[0] + Usb[1] * f.Sst + Usb[2] * K[2] + Usb[3] * K[3] + Usb[4] * e;
    double Sstb = a * Usb[1];
    Kb[2] += a * Usb[2];
    Kb[3] += a * Usb[3];
    double eb = a * Usb[4];
    // e = E_K / rho_K + t1 t2
    UKb[4] += eb / K[0];
    Kb[0] -= eb * UK[4] / (K[0] * K[0]);
    Sstb += eb * (t1 + t2);
    Kb[1] -= eb * t2;
    Kb[4] += eb * t1 / mK;
    double mKb = -eb * t1 * K[4] / (mK * mK);
    // a = m_K / (S_K - S*)
    mKb += ab / d;
    double db = -ab * a / d;
    SKb += db;
    Sstb -= db;
    flux_cons_adjoint(g, K, Fb, UKb, Kb);

    double SLb = 0.0, SRb = 0.0, mLb = 0.0, mRb = 0.0;
    if (left) { SLb += SKb; mLb += mKb; } else { SRb += SKb; mRb += mKb; }
    // S* = num / den
    double numb = Sstb / f.den, denb = -Sstb * f.Sst / f.den;
    Rb[4] += numb; Lb[4] -= numb;
    mLb += numb * L[1] + denb; Lb[1] += numb * f.mL;
    mRb -= numb * R[1] + denb; Rb[1] -= numb * f.mR;
    // m_K = rho_K (S_K - u_K)
    Lb[0] += mLb * (f.SL - L[1]); SLb += mLb * L[0]; Lb[1] -= mLb * L[0];
    Rb[0] += mRb * (f.SR - R[1]); SRb += mRb * R[0]; Rb[1] -= mRb * R[0];
    speeds_adjoint(g, L, R, f, SLb, SRb, Lb, Rb);
}

__device__ void hll_adjoint(double g, const double L[5], const double R[5], const double Fb[5],
                            double Lb[5], double Rb[5])
{
    Fwd f;
    speeds(g, L, R, f);
    const double zero[5] = { 0, 0, 0, 0, 0 };
    if (f.SL >= 0.0) { flux_cons_adjoint(g, L, Fb, zero, Lb); return; }
    if (f.SR <= 0.0) { flux_cons_adjoint(g, R, Fb, zero, Rb); return; }
    double FL[5], FR[5], UL[5], UR[5];
    phys_flux(g, L, FL, UL);
    phys_flux(g, R, FR, UR);
    const double D = f.SR - f.SL;
    double FLb[5], FRb[5], ULb[5], URb[5], SLb = 0.0, SRb = 0.0, Db = 0.0;
    for (int q = 0; q < 5; ++q) {
        double F = (f.SR * FL[q] - f.SL * FR[q] + f.SL * f.SR * (UR[q] - UL[q])) / D;
        double Gb = Fb[q] / D;
        Db -= Fb[q] * F / D;
        FLb[q] = f.SR * Gb;
        FRb[q] = -f.SL * Gb;
        URb[q] = f.SL * f.SR * Gb;
        ULb[q] = -URb[q];
        SRb += Gb * FL[q] + f.SL * Gb * (UR[q] - UL[q]);
        SLb += -Gb * FR[q] + f.SR * Gb * (UR[q] - UL[q]);
    }
    SRb += Db;
    SLb -= Db;
    flux_cons_adjoint(g, L, FLb, ULb, Lb);
    flux_cons_adjoint(g, R, FRb, URb, Rb);
    speeds_adjoint(g, L, R, f, SLb, SRb, Lb, Rb);
}

// face index of direction d at (i, j, k); faces i in [0, n_d] along d
__device__ __forceinline__ int64_t face_index(const Geo &g, int d, int i, int j, int k)
{
    int fx = g.nx + (d == 0), fy = g.ny + (d == 1);
    return ((int64_t)k * fy + j) * fx + i;
}

template <int RS>
__global__ __launch_bounds__(256) void k_faces(Geo g, int d, const double *__restrict__ lam_out,
                                                const double *__restrict__ lam_bflux, Scratch s)
{
    const int fx = g.nx + (d == 0), fy = g.ny + (d == 1), fz = g.nz + (d == 2);
    const int64_t nf = (int64_t)fx * fy * fz;
    const int64_t nint = (int64_t)g.nx * g.ny * g.nz;
    const int64_t sxs = (int64_t)g.nz * g.ny, sys = (int64_t)g.nz * g.nx, szs = (int64_t)g.ny * g.nx;
    const int64_t sheet_base[3] = { 0, 10 * sxs, 10 * sxs + 10 * sys };
    const int64_t sheet_size[3] = { sxs, sys, szs };
    const int n_d = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
    const int nt1 = 1 + (d + 1) % 3, nt2 = 1 + (d + 2) % 3, nn = 1 + d;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nf;
         f += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(f % fx);
        int64_t r = f / fx;
        int j = (int)(r % fy), k = (int)(r / fy);
        // left cell (i,j,k) - e_d, right cell (i,j,k)
        int li = i - (d == 0), lj = j - (d == 1), lk = k - (d == 2);
        int64_t el = ext(g, li, lj, lk), er = ext(g, i, j, k);
        double WL[5], WR[5];
        for (int q = 0; q < 5; ++q) {
            WL[q] = s.Ws[q * g.E + el] + 0.5 * s.S[(d * 5 + q) * g.E + el];
            WR[q] = s.Ws[q * g.E + er] - 0.5 * s.S[(d * 5 + q) * g.E + er];
        }
        bool flL0 = WL[0] < g.rho_floor, flL4 = WL[4] < g.p_floor;
        bool flR0 = WR[0] < g.rho_floor, flR4 = WR[4] < g.p_floor;
        if (flL0) WL[0] = g.rho_floor;
        if (flL4) WL[4] = g.p_floor;
        if (flR0) WR[0] = g.rho_floor;
        if (flR4) WR[4] = g.p_floor;

        // dL/dF: U'_right has -c F(face i-1/2)... U'_cell = U - c (F_out - F_in)
        const bool right_in = i < g.nx && j < g.ny && k < g.nz;
        const bool left_in = li >= 0 && lj >= 0 && lk >= 0;
        double Fb[5];
        for (int q = 0; q < 5; ++q) {
            double v = 0.0;
            if (right_in) v += g.c * lam_out[q * nint + interior_index(g, i, j, k)];
            if (left_in) v -= g.c * lam_out[q * nint + interior_index(g, li, lj, lk)];
            Fb[q] = v;
        }
        const int fi = d == 0 ? i : (d == 1 ? j : k);
        if (lam_bflux && (fi == 0 || fi == n_d)) {
            const double *sh = lam_bflux + sheet_base[d] + (fi == 0 ? 0 : 5 * sheet_size[d]);
            const int slow = d == 2 ? j : k, fast = d == 0 ? j : i;
            const int nfast = d == 0 ? g.ny : g.nx;
            for (int q = 0; q < 5; ++q) Fb[q] += sh[q * sheet_size[d] + (int64_t)slow * nfast + fast];
        }

        // rotate, reverse the Riemann solver, rotate back
        const double L[5] = { WL[0], WL[nn], WL[nt1], WL[nt2], WL[4] };
        const double R[5] = { WR[0], WR[nn], WR[nt1], WR[nt2], WR[4] };
        const double Gb[5] = { Fb[0], Fb[nn], Fb[nt1], Fb[nt2], Fb[4] };
        double Lb[5] = { 0, 0, 0, 0, 0 }, Rb[5] = { 0, 0, 0, 0, 0 };
        if (RS == RS_HLL) hll_adjoint(g.gamma, L, R, Gb, Lb, Rb);
        else hllc_adjoint(g.gamma, L, R, Gb, Lb, Rb);
        double WLb[5], WRb[5];
        WLb[0] = flL0 ? 0.0 : Lb[0]; WLb[4] = flL4 ? 0.0 : Lb[4];
        WRb[0] = flR0 ? 0.0 : Rb[0]; WRb[4] = flR4 ? 0.0 : Rb[4];
        WLb[nn] = Lb[1]; WLb[nt1] = Lb[2]; WLb[nt2] = Lb[3];
        WRb[nn] = Rb[1]; WRb[nt1] = Rb[2]; WRb[nt2] = Rb[3];
        for (int q = 0; q < 5; ++q) {
            s.FL[d][q * nf + f] = WLb[q];
            s.FR[d][q * nf + f] = WRb[q];
        }
    }
}

// ------------------------------------------------------------ 4: cells

template <int LIM>
__global__ __launch_bounds__(256) void k_cells(Geo g, Scratch s)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.E;
         e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        ext_coords(g, e, i, j, k);
        if (!is_predicted(g, i, j, k)) continue;
        const int c3[3] = { i, j, k };
        const int n3[3] = { g.nx, g.ny, g.nz };
        // adjoints of the predicted state and of the slopes from the cell's
        // own face states: W_L of face +1/2 = W* + S/2, W_R of face -1/2 = W* - S/2
        double Wsb[5] = { 0, 0, 0, 0, 0 }, Sb[3][5];
        for (int d = 0; d < 3; ++d) {
            for (int q = 0; q < 5; ++q) Sb[d][q] = 0.0;
            // a face exists when the other two coordinates are inside and
            // the face index along d lies in [0, n_d]
            bool others_in = true;
            for (int o = 0; o < 3; ++o)
                if (o != d && (c3[o] < 0 || c3[o] >= n3[o])) others_in = false;
            if (!others_in) continue;
            const int64_t nf = (int64_t)(g.nx + (d == 0)) * (g.ny + (d == 1)) * (g.nz + (d == 2));
            // face +1/2 of this cell has face index c+1 along d
            if (c3[d] + 1 >= 0 && c3[d] + 1 <= n3[d]) {
                int64_t f = face_index(g, d, i + (d == 0), j + (d == 1), k + (d == 2));
                for (int q = 0; q < 5; ++q) {
                    double v = s.FL[d][q * nf + f];
                    Wsb[q] += v;
                    Sb[d][q] += 0.5 * v;
                }
            }
            // face -1/2 has face index c along d
            if (c3[d] >= 0 && c3[d] <= n3[d]) {
                int64_t f = face_index(g, d, i, j, k);
                for (int q = 0; q < 5; ++q) {
                    double v = s.FR[d][q * nf + f];
                    Wsb[q] += v;
                    Sb[d][q] -= 0.5 * v;
                }
            }
        }
        // reverse of the predictor
        double W[5], S[3][5];
        for (int q = 0; q < 5; ++q) W[q] = s.W[q * g.E + e];
        for (int d = 0; d < 3; ++d)
            for (int q = 0; q < 5; ++q) S[d][q] = s.S[(d * 5 + q) * g.E + e];
        const double lam = g.lam, gm = g.gamma;
        const double rho = W[0], p = W[4], vel[3] = { W[1], W[2], W[3] };
        const double divu = S[0][1] + S[1][2] + S[2][3];
        double Wb[5] = { 0, 0, 0, 0, 0 }, velb[3] = { 0, 0, 0 }, divub = 0.0;
        // rho* = rho - lam (sum_d u_d S_d,rho + rho divu)
        Wb[0] += Wsb[0] * (1.0 - lam * divu);
        divub -= lam * Wsb[0] * rho;
        for (int d = 0; d < 3; ++d) {
            velb[d] -= lam * Wsb[0] * S[d][0];
            Sb[d][0] -= lam * Wsb[0] * vel[d];
        }
        // u_m* = u_m - lam (sum_d u_d S_d,m + S_m,p / rho)
        for (int m = 0; m < 3; ++m) {
            const double b = Wsb[1 + m];
            velb[m] += b;
            for (int d = 0; d < 3; ++d) {
                velb[d] -= lam * b * S[d][1 + m];
                Sb[d][1 + m] -= lam * b * vel[d];
            }
            Sb[m][4] -= lam * b / rho;
            Wb[0] += lam * b * S[m][4] / (rho * rho);
        }
        // p* = p - lam (sum_d u_d S_d,p + gamma p divu)
        Wb[4] += Wsb[4] * (1.0 - lam * gm * divu);
        divub -= lam * Wsb[4] * gm * p;
        for (int d = 0; d < 3; ++d) {
            velb[d] -= lam * Wsb[4] * S[d][4];
            Sb[d][4] -= lam * Wsb[4] * vel[d];
        }
        Sb[0][1] += divub;
        Sb[1][2] += divub;
        Sb[2][3] += divub;
        for (int d = 0; d < 3; ++d) Wb[1 + d] += velb[d];
        for (int q = 0; q < 5; ++q) s.Wd[q * g.E + e] = Wb[q];

        // split every slope adjoint along its two one-sided differences
        const int64_t st[3] = { 1, g.ex, (int64_t)g.ex * g.ey };
        for (int d = 0; d < 3; ++d)
            for (int q = 0; q < 5; ++q) {
                double a = W[q] - s.W[q * g.E + e - st[d]];
                double b = s.W[q * g.E + e + st[d]] - W[q];
                double pa, pb;
                slope_partials<LIM>(a, b, pa, pb);
                s.SA[(d * 5 + q) * g.E + e] = pa * Sb[d][q];
                s.SB[(d * 5 + q) * g.E + e] = pb * Sb[d][q];
            }
    }
}

// ------------------------------------------------------------ 5: input

// dL/dW of extended cell (i, j, k): its predictor term and the slope splits
// of itself (a - b) and of its neighbours along each axis.
__device__ __forceinline__ void gather_wbar(const Geo &g, const Scratch &s, int i, int j, int k,
                                            double Wb[5])
{
    for (int q = 0; q < 5; ++q) Wb[q] = 0.0;
    if (!is_read(g, i, j, k)) return;
    const int64_t e = ext(g, i, j, k);
    const int64_t st[3] = { 1, g.ex, (int64_t)g.ex * g.ey };
    const bool self = is_predicted(g, i, j, k);
    if (self)
        for (int q = 0; q < 5; ++q) Wb[q] += s.Wd[q * g.E + e];
    for (int d = 0; d < 3; ++d) {
        const int dm[3] = { -(d == 0), -(d == 1), -(d == 2) };
        const bool lo = is_predicted(g, i + dm[0], j + dm[1], k + dm[2]);
        const bool hi = is_predicted(g, i - dm[0], j - dm[1], k - dm[2]);
        for (int q = 0; q < 5; ++q) {
            const int64_t idx = (d * 5 + q) * g.E;
            double v = 0.0;
            if (self) v += s.SA[idx + e] - s.SB[idx + e];
            if (lo) v += s.SB[idx + e - st[d]];
            if (hi) v -= s.SA[idx + e + st[d]];
            Wb[q] += v;
        }
    }
}

__device__ __forceinline__ void prim_adjoint(const Geo &g, const double U[5], const double Wb[5],
                                             double Ub[5])
{
    const bool rho_fl = U[0] < g.rho_floor;
    const double rho = rho_fl ? g.rho_floor : U[0];
    const double vel[3] = { U[1] / rho, U[2] / rho, U[3] / rho };
    const double kin = 0.5 * (U[1] * vel[0] + U[2] * vel[1] + U[3] * vel[2]);
    const double p = (g.gamma - 1.0) * (U[4] - kin);
    const double pb = p < g.p_floor ? 0.0 : Wb[4];
    Ub[4] = (g.gamma - 1.0) * pb;
    const double kb = -(g.gamma - 1.0) * pb;
    double rhob = Wb[0];
    for (int d = 0; d < 3; ++d) {
        // kin = sum_d m_d vel_d / 2, vel_d = m_d / rho
        const double vb = Wb[1 + d] + 0.5 * kb * U[1 + d];
        Ub[1 + d] = 0.5 * kb * vel[d] + vb / rho;
        rhob -= vb * vel[d] / rho;
    }
    Ub[0] = rho_fl ? 0.0 : rhob;
}

__global__ __launch_bounds__(256) void k_input(Geo g, const double *__restrict__ u,
                                               const double *__restrict__ lam_out,
                                               double *__restrict__ lam_in, Scratch s)
{
    const int64_t ncell = g.periodic ? (int64_t)g.nx * g.ny * g.nz
                                     : (int64_t)g.gx * g.gy * (g.nz + 2 * g.ng);
    const int64_t nint = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        if (g.periodic) {
            i = (int)(c % g.nx);
            int64_t r = c / g.nx;
            j = (int)(r % g.ny);
            k = (int)(r / g.ny);
        } else {
            i = (int)(c % g.gx) - g.ng;
            int64_t r = c / g.gx;
            j = (int)(r % g.gy) - g.ng;
            k = (int)(r / g.gy) - g.ng;
        }
        double Wb[5] = { 0, 0, 0, 0, 0 };
        if (g.periodic) {
            // every image of the cell inside the extended box [-2, n+2)
            // (at most 5 per axis, for an extent of 1)
            int im[3][5], nim[3];
            const int c3[3] = { i, j, k }, n3[3] = { g.nx, g.ny, g.nz };
            for (int d = 0; d < 3; ++d) {
                nim[d] = 0;
                for (int sh = -2; sh <= 2; ++sh) {
                    int v = c3[d] + sh * n3[d];
                    if (v >= -2 && v < n3[d] + 2) im[d][nim[d]++] = v;
                }
            }
            for (int a = 0; a < nim[2]; ++a)
                for (int b = 0; b < nim[1]; ++b)
                    for (int e = 0; e < nim[0]; ++e) {
                        double t[5];
                        gather_wbar(g, s, im[0][e], im[1][b], im[2][a], t);
                        for (int q = 0; q < 5; ++q) Wb[q] += t[q];
                    }
        } else if (i >= -2 && i < g.nx + 2 && j >= -2 && j < g.ny + 2 && k >= -2 && k < g.nz + 2) {
            gather_wbar(g, s, i, j, k, Wb);
        }
        double Ub[5] = { 0, 0, 0, 0, 0 };
        const bool read = g.periodic || (i >= -2 && i < g.nx + 2 && j >= -2 && j < g.ny + 2 &&
                                         k >= -2 && k < g.nz + 2 && is_read(g, i, j, k));
        if (read) {
            double U[5];
            for (int q = 0; q < 5; ++q) U[q] = u[c + q * g.vin];
            prim_adjoint(g, U, Wb, Ub);
        }
        const bool inside = i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz;
        for (int q = 0; q < 5; ++q) {
            double v = Ub[q];
            if (inside) v += lam_out[q * nint + interior_index(g, i, j, k)];
            lam_in[c + q * g.vin] = v;
        }
    }
}

}  // namespace adj

size_t adjoint_scratch_bytes(const PatchDesc &P)
{
    const int64_t E = (int64_t)(P.nx + 4) * (P.ny + 4) * (P.nz + 4);
    const int64_t nf = (int64_t)(P.nx + 1) * P.ny * P.nz + (int64_t)P.nx * (P.ny + 1) * P.nz +
                       (int64_t)P.nx * P.ny * (P.nz + 1);
    // W 5, S 15, W* 5, Wd 5, SA 15, SB 15 per extended cell; 10 per face
    return (size_t)(60 * E + 10 * nf) * sizeof(double);
}

static int grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

template <int LIM, int RS>
static int run_adjoint(const PatchDesc &P, const double *u_in, const double *lam_out,
                       const double *lam_bflux, double *lam_in, const Scalars &sc, double dt,
                       double *scratch, hipStream_t st)
{
    adj::Geo g{};
    g.nx = P.nx; g.ny = P.ny; g.nz = P.nz; g.ng = P.ng; g.periodic = P.periodic;
    g.ex = P.nx + 4; g.ey = P.ny + 4; g.ez = P.nz + 4;
    g.E = (int64_t)g.ex * g.ey * g.ez;
    g.gx = P.periodic ? P.nx : P.nx + 2 * P.ng;
    g.gy = P.periodic ? P.ny : P.ny + 2 * P.ng;
    g.vin = (int64_t)g.gx * g.gy * (P.periodic ? P.nz : P.nz + 2 * P.ng);
    g.gamma = sc.gamma; g.rho_floor = sc.rho_floor; g.p_floor = sc.p_floor;
    g.lam = dt / (2.0 * P.dx);
    g.c = dt / P.dx;
    adj::Scratch s{};
    double *q = scratch;
    s.W = q; q += 5 * g.E;
    s.S = q; q += 15 * g.E;
    s.Ws = q; q += 5 * g.E;
    s.Wd = q; q += 5 * g.E;
    s.SA = q; q += 15 * g.E;
    s.SB = q; q += 15 * g.E;
    for (int d = 0; d < 3; ++d) {
        g.nf[d] = (int64_t)(P.nx + (d == 0)) * (P.ny + (d == 1)) * (P.nz + (d == 2));
        s.FL[d] = q; q += 5 * g.nf[d];
        s.FR[d] = q; q += 5 * g.nf[d];
    }
    hipLaunchKernelGGL(adj::k_prim, dim3(grid_for(g.E)), dim3(256), 0, st, g, u_in, s);
    hipLaunchKernelGGL(adj::k_slopes<LIM>, dim3(grid_for(g.E)), dim3(256), 0, st, g, s);
    for (int d = 0; d < 3; ++d)
        hipLaunchKernelGGL(adj::k_faces<RS>, dim3(grid_for(g.nf[d])), dim3(256), 0, st, g, d,
                           lam_out, lam_bflux, s);
    hipLaunchKernelGGL(adj::k_cells<LIM>, dim3(grid_for(g.E)), dim3(256), 0, st, g, s);
    const int64_t nin = P.periodic ? (int64_t)P.nx * P.ny * P.nz : g.vin;
    hipLaunchKernelGGL(adj::k_input, dim3(grid_for(nin)), dim3(256), 0, st, g, u_in, lam_out,
                       lam_in, s);
    return (int)hipGetLastError();
}

int launch_adjoint(int limiter, int riemann, const PatchDesc &P, const double *u_in,
                   const double *lam_out, const double *lam_bflux, double *lam_in,
                   const Scalars &sc, double dt, double *scratch, hipStream_t s)
{
    if (riemann == 1) {
        if (limiter == 1) return run_adjoint<1, 1>(P, u_in, lam_out, lam_bflux, lam_in, sc, dt, scratch, s);
        if (limiter == 2) return run_adjoint<2, 1>(P, u_in, lam_out, lam_bflux, lam_in, sc, dt, scratch, s);
        return run_adjoint<0, 1>(P, u_in, lam_out, lam_bflux, lam_in, sc, dt, scratch, s);
    }
    if (limiter == 1) return run_adjoint<1, 0>(P, u_in, lam_out, lam_bflux, lam_in, sc, dt, scratch, s);
    if (limiter == 2) return run_adjoint<2, 0>(P, u_in, lam_out, lam_bflux, lam_in, sc, dt, scratch, s);
    return run_adjoint<0, 0>(P, u_in, lam_out, lam_bflux, lam_in, sc, dt, scratch, s);
}

}  // namespace gd
