// Reverse-mode adjoint of the Godunov step (gfx950, FP64), for a fixed dt.
//
// The step is U -> U' = U - dt/dx sum_faces (signed F), with every face flux
// F(W_L, W_R) a function of the predicted states of its two cells, each of
// which depends on the primitive state of the cell and its limited slopes.
// The adjoint runs the chain backwards in gather form -- every output value
// is a sum written by exactly one thread, in a fixed order, with no atomics
// -- so it is bitwise deterministic. Three kernels share a scratch area over
// the cells whose predicted states the step uses: the extended box
// [-2, n+2)^3 of a ghosted patch, or the periodic box itself, whose
// neighbours wrap (x fastest):
//   1 predict  per predicted cell: primitives of its 7-point stencil (from
//              U), limited slopes S, predicted state W*, and a 2-bit code per
//              slope recording the limiter branch taken
//   2 cells    per 16x16 column tile of predicted cells, marching up a
//              z-range: for every face of a plane of the tile, dL/dF = dt/dx
//              (lam_right - lam_left) (+ dL/dbflux on the patch boundary),
//              reversed through the Riemann solver and the face floors; the x
//              and y faces go through LDS (faces on a tile border are
//              evaluated by both tiles), the z face above a cell stays in
//              registers and serves the plane above as its lower face; then
//              per cell the reverse predictor: dL/dW (direct part) and dL/dS
//   3 input    per input cell: dL/dW gathered from its own predictor term
//              and the slope adjoints of itself and its neighbours split by
//              the recorded branches, reversed through the primitive
//              conversion, plus the identity term lam_out.
// At kinks (limiter switches, min/max of wave speeds, the HLLC region and the
// floors) the derivative of the branch the forward step takes is used, with
// the forward step's tie rules. Indices are 32-bit: the host rejects boxes
// whose scratch arrays would not fit.
#include "godunov_internal.h"
#include "godunov_math.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace gd {

namespace adj {

enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_NONE = 2 };
enum { RS_HLLC = 0, RS_HLL = 1 };

// column tile of the cells kernel (one thread per column) and its x and y
// face slots per plane
constexpr int CTX = 16, CTY = 16, CT = CTX * CTY;
constexpr int NXF = (CTX + 1) * CTY, NYF = CTX * (CTY + 1);

struct Geo {
    int nx, ny, nz, ng, periodic;
    int ex, ey, ez;            // scratch box: n + 4 (ghosted) or n (periodic)
    int E;                     // cells of the scratch box
    int lo;                    // first predicted index: -1 (ghosted) or 0
    int px, py, pz;            // predicted extents: n + 2 (ghosted) or n
    int vin;                   // input variable stride
    int gx, gy, gz;            // input extents
    int nint;                  // interior cells
    int ntx, nty, nseg, zlen;  // tiles and z-segments of the cells kernel
    int nitem, per_xcd;        // its work items, and items per XCD slice
    double gamma, inv_gm1, rho_floor, p_floor, lam, c;   // lam = dt/(2dx), c = dt/dx
};

// Per-cell records of 20 doubles, stored in blocks of 64 consecutive cells
// with the fields of a block contiguous ([E/64][20][64]): a wavefront reads
// one field of 64 neighbouring cells as one 512-byte segment, and all the
// fields of those cells lie in one 10 KB span. Records are written with
// streaming (non-temporal) stores: the next kernel reads them long after.
constexpr int NF = 20;
// fields of the forward record: slopes S at d*5+q, predicted state W* at 15+q
constexpr int F_S = 0, F_WS = 15;
// fields of the adjoint record: dL/dS at d*5+q, direct dL/dW at 15+q
constexpr int F_SB = 0, F_WD = 15;

__device__ __forceinline__ int rec(int e, int f) { return ((e >> 6) * NF + f) * 64 + (e & 63); }

struct Scratch {
    double *fw;        // forward record of each extended cell
    double *ad;        // adjoint record of each extended cell
    unsigned *code;    // [E] limiter branch per slope, 2 bits at 2(d*5+q)
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
    return g.periodic ||
           depth_out(i, g.nx) + depth_out(j, g.ny) + depth_out(k, g.nz) <= 1;
}

// i mod n for i in [-3, n+3); the general form only for boxes narrower than 3
__device__ __forceinline__ int wrap(int i, int n)
{
    if (i < 0) i += n;
    else if (i >= n) i -= n;
    if ((unsigned)i >= (unsigned)n) { i %= n; if (i < 0) i += n; }
    return i;
}

// scratch index of cell (i, j, k): the extended box of a ghosted patch, the
// wrapped interior of a periodic box
__device__ __forceinline__ int ext(const Geo &g, int i, int j, int k)
{
    if (g.periodic) {
        i = wrap(i, g.nx); j = wrap(j, g.ny); k = wrap(k, g.nz);
        return (k * g.ny + j) * g.nx + i;
    }
    return ((k + 2) * g.ey + (j + 2)) * g.ex + (i + 2);
}

// position of cell (i, j, k) of the extended box in the input array
__device__ __forceinline__ int in_index(const Geo &g, int i, int j, int k)
{
    if (g.periodic) {
        i = wrap(i, g.nx); j = wrap(j, g.ny); k = wrap(k, g.nz);
        return (k * g.ny + j) * g.nx + i;
    }
    return ((k + g.ng) * g.gy + (j + g.ng)) * g.gx + (i + g.ng);
}

__device__ __forceinline__ int interior_index(const Geo &g, int i, int j, int k)
{
    return (k * g.ny + j) * g.nx + i;
}

// Conserved -> primitive with floors.
__device__ __forceinline__ void to_prim(const Geo &g, const double U[5], double W[5],
                                        double &inv_rho)
{
    double rho = U[0];
    if (rho < g.rho_floor) rho = g.rho_floor;
    inv_rho = fast_rcp(rho);
    double u = U[1] * inv_rho, v = U[2] * inv_rho, w = U[3] * inv_rho;
    double kin = 0.5 * (U[1] * u + U[2] * v + U[3] * w);
    double p = (g.gamma - 1.0) * (U[4] - kin);
    if (p < g.p_floor) p = g.p_floor;
    W[0] = rho; W[1] = u; W[2] = v; W[3] = w; W[4] = p;
}

__device__ __forceinline__ void load_prim(const Geo &g, const double *__restrict__ u, int i, int j,
                                          int k, double W[5], double &inv_rho)
{
    const int p = in_index(g, i, j, k);
    double U[5];
    for (int q = 0; q < 5; ++q) U[q] = u[p + q * g.vin];
    to_prim(g, U, W, inv_rho);
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

// Branch of a limited slope: 0 zero slope, 1 the a-branch, 2 the b-branch,
// 3 the symmetric branch (a+b)/2 or |a+b|/2.
template <int LIM>
__device__ __forceinline__ unsigned slope_branch(double a, double b)
{
    if (LIM == LIM_NONE) return 3u;
    bool same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
    if (!same) return 0u;
    if (LIM == LIM_MINMOD) return fabs(a) <= fabs(b) ? 1u : 2u;
    double m1 = 2.0 * fabs(a), m2 = 2.0 * fabs(b), m3 = 0.5 * fabs(a + b);
    bool first = m1 <= m2;
    double m = first ? m1 : m2;
    if (m <= m3) return first ? 1u : 2u;
    return 3u;
}

// d slope / d a and d slope / d b of a recorded branch
template <int LIM>
__device__ __forceinline__ void branch_partials(unsigned br, double &pa, double &pb)
{
    const double one = LIM == LIM_MC ? 2.0 : 1.0;
    pa = br == 1u ? one : (br == 3u ? 0.5 : 0.0);
    pb = br == 2u ? one : (br == 3u ? 0.5 : 0.0);
}

// ------------------------------------------------------------ 1: predict

template <int LIM>
__global__ __launch_bounds__(256) void k_predict(Geo g, const double *__restrict__ u, Scratch s)
{
    // predicted cells lie in [lo, lo + p)^3
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.px * g.py * g.pz) return;
    const int i = t % g.px + g.lo, r = t / g.px;
    const int j = r % g.py + g.lo, k = r / g.py + g.lo;
    if (!is_predicted(g, i, j, k)) return;
    const int e = ext(g, i, j, k);
    double W[5], S[3][5], inv_rho, dummy;
    load_prim(g, u, i, j, k, W, inv_rho);
    unsigned code = 0u;
    for (int d = 0; d < 3; ++d) {
        double Wm[5], Wp[5];
        load_prim(g, u, i - (d == 0), j - (d == 1), k - (d == 2), Wm, dummy);
        load_prim(g, u, i + (d == 0), j + (d == 1), k + (d == 2), Wp, dummy);
        for (int q = 0; q < 5; ++q) {
            const double a = W[q] - Wm[q], b = Wp[q] - W[q];
            S[d][q] = slope<LIM>(a, b);
            code |= slope_branch<LIM>(a, b) << (2 * (d * 5 + q));
            __builtin_nontemporal_store(S[d][q], &s.fw[rec(e, F_S + d * 5 + q)]);
        }
    }
    s.code[e] = code;
    const double divu = S[0][1] + S[1][2] + S[2][3];
    double adv[5];
    for (int q = 0; q < 5; ++q) adv[q] = W[1] * S[0][q] + W[2] * S[1][q] + W[3] * S[2][q];
    double Ws[5];
    Ws[0] = W[0] - g.lam * (adv[0] + W[0] * divu);
    Ws[1] = W[1] - g.lam * (adv[1] + S[0][4] * inv_rho);
    Ws[2] = W[2] - g.lam * (adv[2] + S[1][4] * inv_rho);
    Ws[3] = W[3] - g.lam * (adv[3] + S[2][4] * inv_rho);
    Ws[4] = W[4] - g.lam * (adv[4] + g.gamma * W[4] * divu);
    for (int q = 0; q < 5; ++q) __builtin_nontemporal_store(Ws[q], &s.fw[rec(e, F_WS + q)]);
}

// ------------------------------------------------------------ Riemann adjoints

// Forward quantities of the HLLC / HLL flux in rotated form, kept for the
// reverse sweep.
struct Fwd {
    double cL, cR, SL, SR, iL0, iR0, iL4, iR4;
    bool slL, srL;      // S_L took the left candidate, S_R the left candidate
};

__device__ __forceinline__ void speeds(double g, const double L[5], const double R[5], Fwd &f)
{
    f.iL0 = fast_rcp(L[0]); f.iR0 = fast_rcp(R[0]);
    f.iL4 = fast_rcp(L[4]); f.iR4 = fast_rcp(R[4]);
    const double gl = g * L[4], gr = g * R[4];
    f.cL = gl * fast_rsqrt(gl * L[0]);
    f.cR = gr * fast_rsqrt(gr * R[0]);
    double a = L[1] - f.cL, b = R[1] - f.cR;
    f.slL = a <= b;
    f.SL = f.slL ? a : b;
    double c = L[1] + f.cL, d = R[1] + f.cR;
    f.srL = c >= d;
    f.SR = f.srL ? c : d;
}

__device__ __forceinline__ void speeds_adjoint(const Fwd &f, double SLb, double SRb, double Lb[5],
                                               double Rb[5])
{
    double cLb = 0.0, cRb = 0.0;
    if (f.slL) { Lb[1] += SLb; cLb -= SLb; } else { Rb[1] += SLb; cRb -= SLb; }
    if (f.srL) { Lb[1] += SRb; cLb += SRb; } else { Rb[1] += SRb; cRb += SRb; }
    // c = sqrt(g p / rho): dc = c/2 (dp/p - drho/rho)
    const double hl = 0.5 * cLb * f.cL, hr = 0.5 * cRb * f.cR;
    Lb[4] += hl * f.iL4;
    Lb[0] -= hl * f.iL0;
    Rb[4] += hr * f.iR4;
    Rb[0] -= hr * f.iR0;
}

// Adjoint of the physical flux and of the conserved vector of a rotated
// primitive state W, accumulated into Wb: Fb . dF/dW + Ub . dU/dW.
__device__ __forceinline__ void flux_cons_adjoint(double inv_gm1, const double W[5],
                                                  const double Fb[5], const double Ub[5],
                                                  double Wb[5])
{
    const double r = W[0], u = W[1], v = W[2], w = W[3], p = W[4];
    const double q2 = u * u + v * v + w * w;
    const double E = p * inv_gm1 + 0.5 * r * q2;
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
    Wb[4] += Eb * inv_gm1;
}

__device__ __forceinline__ void phys_flux(double inv_gm1, const double W[5], double F[5],
                                          double U[5])
{
    const double r = W[0], u = W[1], v = W[2], w = W[3], p = W[4];
    const double E = p * inv_gm1 + 0.5 * r * (u * u + v * v + w * w);
    F[0] = r * u; F[1] = r * u * u + p; F[2] = r * u * v; F[3] = r * u * w; F[4] = u * (E + p);
    U[0] = r; U[1] = r * u; U[2] = r * v; U[3] = r * w; U[4] = E;
}

__device__ __forceinline__ void hllc_adjoint(double g, double inv_gm1, const double L[5],
                                             const double R[5], const double Fb[5], double Lb[5],
                                             double Rb[5])
{
    Fwd f;
    speeds(g, L, R, f);
    const double zero[5] = { 0, 0, 0, 0, 0 };
    if (f.SL >= 0.0) { flux_cons_adjoint(inv_gm1, L, Fb, zero, Lb); return; }
    const double mL = L[0] * (f.SL - L[1]);
    const double mR = R[0] * (f.SR - R[1]);
    const double num = R[4] - L[4] + mL * L[1] - mR * R[1];
    const double den = mL - mR;
    const double iden = fast_rcp(den);
    const double Sst = num * iden;
    bool left;
    if (Sst >= 0.0) left = true;
    else if (f.SR > 0.0) left = false;
    else { flux_cons_adjoint(inv_gm1, R, Fb, zero, Rb); return; }

    // the star state on the side of the contact the face lies on; values
    // are selected (not pointers), so that everything stays in registers
    double K[5], Kb[5] = { 0, 0, 0, 0, 0 };
    for (int q = 0; q < 5; ++q) K[q] = left ? L[q] : R[q];
    const double SK = left ? f.SL : f.SR, mK = left ? mL : mR;
    const double iK0 = left ? f.iL0 : f.iR0;
    double FK[5], UK[5];
    phys_flux(inv_gm1, K, FK, UK);
    const double d = SK - Sst;
    const double id = fast_rcp(d), imK = fast_rcp(mK);
    const double a = mK * id;
    const double t1 = Sst - K[1], t2 = Sst + K[4] * imK;
    const double e = UK[4] * iK0 + t1 * t2;
    const double Us[5] = { a, a * Sst, a * K[2], a * K[3], a * e };

    // F = F_K + S_K (U* - U_K)
    double SKb = 0.0, UKb[5], Usb[5];
    for (int q = 0; q < 5; ++q) {
        SKb += Fb[q] * (Us[q] - UK[q]);
        Usb[q] = SK * Fb[q];
        UKb[q] = -SK * Fb[q];
    }
    // U* = a (1, S*, v, w, e)
    double ab = Usb[0] + Usb[1] * Sst + Usb[2] * K[2] + Usb[3] * K[3] + Usb[4] * e;
    double Sstb = a * Usb[1];
    Kb[2] += a * Usb[2];
    Kb[3] += a * Usb[3];
    double eb = a * Usb[4];
    // e = E_K / rho_K + t1 t2
    UKb[4] += eb * iK0;
    Kb[0] -= eb * UK[4] * iK0 * iK0;
    Sstb += eb * (t1 + t2);
    Kb[1] -= eb * t2;
    Kb[4] += eb * t1 * imK;
    double mKb = -eb * t1 * K[4] * imK * imK;
    // a = m_K / (S_K - S*)
    mKb += ab * id;
    double db = -ab * a * id;
    SKb += db;
    Sstb -= db;
    flux_cons_adjoint(inv_gm1, K, Fb, UKb, Kb);
    for (int q = 0; q < 5; ++q) {
        Lb[q] += left ? Kb[q] : 0.0;
        Rb[q] += left ? 0.0 : Kb[q];
    }

    double SLb = 0.0, SRb = 0.0, mLb = 0.0, mRb = 0.0;
    if (left) { SLb += SKb; mLb += mKb; } else { SRb += SKb; mRb += mKb; }
    // S* = num / den
    double numb = Sstb * iden, denb = -Sstb * Sst * iden;
    Rb[4] += numb; Lb[4] -= numb;
    mLb += numb * L[1] + denb; Lb[1] += numb * mL;
    mRb -= numb * R[1] + denb; Rb[1] -= numb * mR;
    // m_K = rho_K (S_K - u_K)
    Lb[0] += mLb * (f.SL - L[1]); SLb += mLb * L[0]; Lb[1] -= mLb * L[0];
    Rb[0] += mRb * (f.SR - R[1]); SRb += mRb * R[0]; Rb[1] -= mRb * R[0];
    speeds_adjoint(f, SLb, SRb, Lb, Rb);
}

__device__ __forceinline__ void hll_adjoint(double g, double inv_gm1, const double L[5],
                                            const double R[5], const double Fb[5], double Lb[5],
                                            double Rb[5])
{
    Fwd f;
    speeds(g, L, R, f);
    const double zero[5] = { 0, 0, 0, 0, 0 };
    if (f.SL >= 0.0) { flux_cons_adjoint(inv_gm1, L, Fb, zero, Lb); return; }
    if (f.SR <= 0.0) { flux_cons_adjoint(inv_gm1, R, Fb, zero, Rb); return; }
    double FL[5], FR[5], UL[5], UR[5];
    phys_flux(inv_gm1, L, FL, UL);
    phys_flux(inv_gm1, R, FR, UR);
    const double iD = fast_rcp(f.SR - f.SL);
    double FLb[5], FRb[5], ULb[5], URb[5], SLb = 0.0, SRb = 0.0, Db = 0.0;
    for (int q = 0; q < 5; ++q) {
        double F = (f.SR * FL[q] - f.SL * FR[q] + f.SL * f.SR * (UR[q] - UL[q])) * iD;
        double Gb = Fb[q] * iD;
        Db -= Gb * F;
        FLb[q] = f.SR * Gb;
        FRb[q] = -f.SL * Gb;
        URb[q] = f.SL * f.SR * Gb;
        ULb[q] = -URb[q];
        SRb += Gb * FL[q] + f.SL * Gb * (UR[q] - UL[q]);
        SLb += -Gb * FR[q] + f.SR * Gb * (UR[q] - UL[q]);
    }
    SRb += Db;
    SLb -= Db;
    flux_cons_adjoint(inv_gm1, L, FLb, ULb, Lb);
    flux_cons_adjoint(inv_gm1, R, FRb, URb, Rb);
    speeds_adjoint(f, SLb, SRb, Lb, Rb);
}

// dL/dU' of cell (i, j, k), zero for cells outside the patch interior
// (which have no update)
__device__ __forceinline__ void lam_at(const Geo &g, const double *__restrict__ lam_out, int i,
                                       int j, int k, double L[5])
{
    const bool in = g.periodic || (i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz);
    const int c = g.periodic ? ext(g, i, j, k) : (in ? interior_index(g, i, j, k) : 0);
    for (int q = 0; q < 5; ++q) L[q] = in ? lam_out[q * g.nint + c] : 0.0;
}

// Adjoint of the two face states WL, WR (before the floors) of the face
// along D whose right cell is (i, j, k) and left cell (i, j, k) - e_D, whose
// updates have adjoints lamL and lamR: dL/dF reversed through the Riemann
// solver and the face-state floors, in unrotated variables.
template <int RS, int D>
__device__ __forceinline__ void face_adjoint(const Geo &g, int i, int j, int k, double WL[5],
                                             double WR[5], const double lamL[5],
                                             const double lamR[5],
                                             const double *__restrict__ lam_bflux, double WLb[5],
                                             double WRb[5])
{
    constexpr int nt1 = 1 + (D + 1) % 3, nt2 = 1 + (D + 2) % 3, nn = 1 + D;
    const bool flL0 = WL[0] < g.rho_floor, flL4 = WL[4] < g.p_floor;
    const bool flR0 = WR[0] < g.rho_floor, flR4 = WR[4] < g.p_floor;
    if (flL0) WL[0] = g.rho_floor;
    if (flL4) WL[4] = g.p_floor;
    if (flR0) WR[0] = g.rho_floor;
    if (flR4) WR[4] = g.p_floor;

    // dL/dF: the right cell's update has -c F(face), the left cell's +c F
    double Fb[5];
    for (int q = 0; q < 5; ++q) Fb[q] = g.c * lamR[q] - g.c * lamL[q];
    const int n_d = D == 0 ? g.nx : (D == 1 ? g.ny : g.nz);
    const int fi = D == 0 ? i : (D == 1 ? j : k);
    if (lam_bflux && (fi == 0 || fi == n_d)) {
        const int sxs = g.nz * g.ny, sys = g.nz * g.nx, szs = g.ny * g.nx;
        const int base = D == 0 ? 0 : (D == 1 ? 10 * sxs : 10 * sxs + 10 * sys);
        const int size = D == 0 ? sxs : (D == 1 ? sys : szs);
        const int slow = D == 2 ? j : k, fast = D == 0 ? j : i;
        const int nfast = D == 0 ? g.ny : g.nx;
        const int at = slow * nfast + fast;
        // faces 0 and n of a periodic box are one face: both sheets hold its flux
        if (fi == 0 || g.periodic)
            for (int q = 0; q < 5; ++q) Fb[q] += lam_bflux[base + q * size + at];
        if (fi == n_d || g.periodic)
            for (int q = 0; q < 5; ++q) Fb[q] += lam_bflux[base + 5 * size + q * size + at];
    }

    // rotate, reverse the Riemann solver, rotate back
    const double L[5] = { WL[0], WL[nn], WL[nt1], WL[nt2], WL[4] };
    const double R[5] = { WR[0], WR[nn], WR[nt1], WR[nt2], WR[4] };
    const double Gb[5] = { Fb[0], Fb[nn], Fb[nt1], Fb[nt2], Fb[4] };
    double Lb[5] = { 0, 0, 0, 0, 0 }, Rb[5] = { 0, 0, 0, 0, 0 };
    if (RS == RS_HLL) hll_adjoint(g.gamma, g.inv_gm1, L, R, Gb, Lb, Rb);
    else hllc_adjoint(g.gamma, g.inv_gm1, L, R, Gb, Lb, Rb);
    WLb[0] = flL0 ? 0.0 : Lb[0]; WLb[4] = flL4 ? 0.0 : Lb[4];
    WRb[0] = flR0 ? 0.0 : Rb[0]; WRb[4] = flR4 ? 0.0 : Rb[4];
    WLb[nn] = Lb[1]; WLb[nt1] = Lb[2]; WLb[nt2] = Lb[3];
    WRb[nn] = Rb[1]; WRb[nt1] = Rb[2]; WRb[nt2] = Rb[3];
}

// ------------------------------------------------------------ 2: cells

// LDS of the cells kernel, for the x faces of one plane of the tile (and
// likewise for y): per cell of the row range [-1, CTX] (the tile and one
// halo cell on each side), plus[q] = W* + S_x/2, the left state of its upper
// face, and minus[q] = W* - S_x/2, the right state of its lower face. Each
// face task reads the plus state of its left cell and the minus state of
// its right cell and overwrites both with their adjoints; no other task
// touches them, so afterwards a cell finds the adjoints of its own two face
// states in its own slots.
// lam holds dL/dU' of the tile and its one-deep x and y halo, at tile
// coordinates + 1.
constexpr int XW = CTX + 2, YW = CTY + 2;
struct CellsSmem {
    double xp[5][CTY][XW], xm[5][CTY][XW];
    double yp[5][YW][CTX], ym[5][YW][CTX];
    double lam[5][YW][XW];
};

// A face along D exists when its index along D lies in [0, n_D] and the
// other two coordinates of its right cell are inside the patch.
template <int D>
__device__ __forceinline__ bool face_exists(const Geo &g, int i, int j, int k)
{
    const int c3[3] = { i, j, k }, n3[3] = { g.nx, g.ny, g.nz };
    bool ok = c3[D] >= 0 && c3[D] <= n3[D];
    for (int o = 0; o < 3; ++o)
        if (o != D && (c3[o] < 0 || c3[o] >= n3[o])) ok = false;
    return ok;
}

// whether cell (i, j, k) has a slot in the scratch records
__device__ __forceinline__ bool in_scratch(const Geo &g, int i, int j, int k)
{
    return g.periodic || (i >= -2 && i < g.nx + 2 && j >= -2 && j < g.ny + 2 && k >= -2 &&
                          k < g.nz + 2);
}

// W* +- S_D/2 of cell (i, j, k) (zero outside the scratch box)
template <int D>
__device__ __forceinline__ void face_states(const Geo &g, const Scratch &s, int i, int j, int k,
                                            double P[5], double M[5])
{
    if (!in_scratch(g, i, j, k)) {
        for (int q = 0; q < 5; ++q) { P[q] = 0.0; M[q] = 0.0; }
        return;
    }
    const int e = ext(g, i, j, k);
    for (int q = 0; q < 5; ++q) {
        const double w = s.fw[rec(e, F_WS + q)], h = 0.5 * s.fw[rec(e, F_S + D * 5 + q)];
        P[q] = w + h;
        M[q] = w - h;
    }
}

// The x (D = 0) or y (D = 1) face tasks of a plane, on the staged states.
template <int RS, int D>
__device__ __forceinline__ void plane_faces(const Geo &g, int i0, int j0, int k,
                                            const double *__restrict__ lam_bflux, CellsSmem &sm)
{
    constexpr int SX = CTX + (D == 0), NS = D == 0 ? NXF : NYF;
    // NS exceeds the thread count by a few tasks; the y pass hands its extra
    // tasks to the second wave, so that no wave does two extra rounds
    const int first = D == 0 ? threadIdx.x : (threadIdx.x + CT - 64) % CT;
    for (int t = first; t < NS; t += CT) {
        // slot (sx, sy): the face whose right cell is (i0 + sx, j0 + sy, k)
        const int sx = t % SX, sy = t / SX;
        const int i = i0 + sx, j = j0 + sy;
        if (!face_exists<D>(g, i, j, k)) {
            for (int q = 0; q < 5; ++q) {
                if (D == 0) { sm.xp[q][sy][sx] = 0.0; sm.xm[q][sy][sx + 1] = 0.0; }
                else { sm.yp[q][sy][sx] = 0.0; sm.ym[q][sy + 1][sx] = 0.0; }
            }
            continue;
        }
        // the left cell sits at x index sx - 1 of the staged row, i.e. slot sx
        double WL[5], WR[5], WLb[5], WRb[5], lamL[5], lamR[5];
        for (int q = 0; q < 5; ++q) {
            WL[q] = D == 0 ? sm.xp[q][sy][sx] : sm.yp[q][sy][sx];
            WR[q] = D == 0 ? sm.xm[q][sy][sx + 1] : sm.ym[q][sy + 1][sx];
            lamL[q] = D == 0 ? sm.lam[q][sy + 1][sx] : sm.lam[q][sy][sx + 1];
            lamR[q] = sm.lam[q][sy + 1][sx + 1];
        }
        face_adjoint<RS, D>(g, i, j, k, WL, WR, lamL, lamR, lam_bflux, WLb, WRb);
        for (int q = 0; q < 5; ++q) {
            if (D == 0) { sm.xp[q][sy][sx] = WLb[q]; sm.xm[q][sy][sx + 1] = WRb[q]; }
            else { sm.yp[q][sy][sx] = WLb[q]; sm.ym[q][sy + 1][sx] = WRb[q]; }
        }
    }
}

template <int RS>
__global__ __launch_bounds__(CT) void k_cells(Geo g, const double *__restrict__ u,
                                              const double *__restrict__ lam_out,
                                              const double *__restrict__ lam_bflux, Scratch s)
{
    __shared__ CellsSmem sm;
    // workgroups are dealt to the eight XCDs in turn: give each XCD a
    // contiguous range of work items, so that neighbouring tiles share its L2
    const int b = (blockIdx.x & 7) * g.per_xcd + (blockIdx.x >> 3);
    if (b >= g.nitem) return;
    const int bx = b % g.ntx, br = b / g.ntx;
    const int by = br % g.nty, bz = br / g.nty;
    // tiles and z-segments cover the predicted range [lo, lo + p)^3
    const int i0 = bx * CTX + g.lo, j0 = by * CTY + g.lo;
    const int kb = bz * g.zlen + g.lo, ke = min(kb + g.zlen, g.lo + g.pz);
    const int tx = threadIdx.x % CTX, ty = threadIdx.x / CTX;
    const int i = i0 + tx, j = j0 + ty;
    const bool col = i < g.lo + g.px && j < g.lo + g.py;

    // dL/dU' of the column's cell in the current plane, carried up the march
    double lamk[5];
    lam_at(g, lam_out, i, j, kb, lamk);
    // right-state adjoint of the z face below the first plane
    double zlo[5] = { 0, 0, 0, 0, 0 };
    if (face_exists<2>(g, i, j, kb)) {
        double P[5], M[5], WL[5], WR[5], t[5], lamb[5];
        face_states<2>(g, s, i, j, kb - 1, WL, M);
        face_states<2>(g, s, i, j, kb, P, WR);
        lam_at(g, lam_out, i, j, kb - 1, lamb);
        face_adjoint<RS, 2>(g, i, j, kb, WL, WR, lamb, lamk, lam_bflux, t, zlo);
    }
    for (int k = kb; k < ke; ++k) {
        // stage the x and y face states of the plane: every thread its own
        // cell, the first wave the 64 halo cells
        {
            double P[5], M[5];
            face_states<0>(g, s, i, j, k, P, M);
            for (int q = 0; q < 5; ++q) { sm.xp[q][ty][tx + 1] = P[q]; sm.xm[q][ty][tx + 1] = M[q]; }
            face_states<1>(g, s, i, j, k, P, M);
            for (int q = 0; q < 5; ++q) { sm.yp[q][ty + 1][tx] = P[q]; sm.ym[q][ty + 1][tx] = M[q]; }
            for (int q = 0; q < 5; ++q) sm.lam[q][ty + 1][tx + 1] = lamk[q];
            if (threadIdx.x < 2 * (CTX + CTY)) {
                const int h = threadIdx.x;
                double L[5];
                if (h < 2 * CTY) {
                    // x halo: column -1 (plus state) or column CTX (minus state)
                    const int r = h % CTY, right = h / CTY;
                    const int hx = right ? CTX : -1;
                    face_states<0>(g, s, i0 + hx, j0 + r, k, P, M);
                    lam_at(g, lam_out, i0 + hx, j0 + r, k, L);
                    for (int q = 0; q < 5; ++q) {
                        if (right) sm.xm[q][r][CTX + 1] = M[q];
                        else sm.xp[q][r][0] = P[q];
                        sm.lam[q][r + 1][hx + 1] = L[q];
                    }
                } else {
                    // y halo: row -1 (plus state) or row CTY (minus state)
                    const int c = (h - 2 * CTY) % CTX, top = (h - 2 * CTY) / CTX;
                    const int hy = top ? CTY : -1;
                    face_states<1>(g, s, i0 + c, j0 + hy, k, P, M);
                    lam_at(g, lam_out, i0 + c, j0 + hy, k, L);
                    for (int q = 0; q < 5; ++q) {
                        if (top) sm.ym[q][CTY + 1][c] = M[q];
                        else sm.yp[q][0][c] = P[q];
                        sm.lam[q][hy + 1][c + 1] = L[q];
                    }
                }
            }
        }
        // the z face above the cell, in registers
        double zl[5] = { 0, 0, 0, 0, 0 }, zr[5] = { 0, 0, 0, 0, 0 }, lamk1[5];
        lam_at(g, lam_out, i, j, k + 1, lamk1);
        if (face_exists<2>(g, i, j, k + 1)) {
            double P[5], M[5], WL[5], WR[5];
            face_states<2>(g, s, i, j, k, WL, M);
            face_states<2>(g, s, i, j, k + 1, P, WR);
            face_adjoint<RS, 2>(g, i, j, k + 1, WL, WR, lamk, lamk1, lam_bflux, zl, zr);
        }
        for (int q = 0; q < 5; ++q) lamk[q] = lamk1[q];
        __syncthreads();
        plane_faces<RS, 0>(g, i0, j0, k, lam_bflux, sm);
        plane_faces<RS, 1>(g, i0, j0, k, lam_bflux, sm);
        __syncthreads();

        // the adjoints of the cell's face states: the left state of its upper
        // face is W* + S/2, the right state of its lower face is W* - S/2
        double Wsb[5] = { 0, 0, 0, 0, 0 }, Sb[3][5];
        for (int q = 0; q < 5; ++q) {
            const double vl = sm.xp[q][ty][tx + 1], vr = sm.xm[q][ty][tx + 1];
            Wsb[q] += vl;
            Wsb[q] += vr;
            Sb[0][q] = 0.5 * vl - 0.5 * vr;
        }
        for (int q = 0; q < 5; ++q) {
            const double vl = sm.yp[q][ty + 1][tx], vr = sm.ym[q][ty + 1][tx];
            Wsb[q] += vl;
            Wsb[q] += vr;
            Sb[1][q] = 0.5 * vl - 0.5 * vr;
        }
        for (int q = 0; q < 5; ++q) {
            Wsb[q] += zl[q];
            Wsb[q] += zlo[q];
            Sb[2][q] = 0.5 * zl[q] - 0.5 * zlo[q];
            zlo[q] = zr[q];
        }
        __syncthreads();
        if (!col || !is_predicted(g, i, j, k)) continue;

        // reverse of the predictor
        const int e = ext(g, i, j, k);
        double W[5], S[3][5], inv_rho;
        load_prim(g, u, i, j, k, W, inv_rho);
        for (int d = 0; d < 3; ++d)
            for (int q = 0; q < 5; ++q) S[d][q] = s.fw[rec(e, F_S + d * 5 + q)];
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
            const double bm = Wsb[1 + m];
            velb[m] += bm;
            for (int d = 0; d < 3; ++d) {
                velb[d] -= lam * bm * S[d][1 + m];
                Sb[d][1 + m] -= lam * bm * vel[d];
            }
            Sb[m][4] -= lam * bm * inv_rho;
            Wb[0] += lam * bm * S[m][4] * inv_rho * inv_rho;
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
        for (int q = 0; q < 5; ++q) __builtin_nontemporal_store(Wb[q], &s.ad[rec(e, F_WD + q)]);
        for (int d = 0; d < 3; ++d)
            for (int q = 0; q < 5; ++q)
                __builtin_nontemporal_store(Sb[d][q], &s.ad[rec(e, F_SB + d * 5 + q)]);
    }
}

// ------------------------------------------------------------ 3: input

// dL/dW of extended cell (i, j, k): its predictor term and the slope splits
// of itself (a - b) and of its neighbours along each axis, from the branches
// recorded by the predict kernel.
template <int LIM>
__device__ __forceinline__ void gather_wbar(const Geo &g, const Scratch &s, int i, int j, int k,
                                            double Wb[5])
{
    for (int q = 0; q < 5; ++q) Wb[q] = 0.0;
    if (!is_read(g, i, j, k)) return;
    const int e = ext(g, i, j, k);
    const bool self = is_predicted(g, i, j, k);
    const unsigned cs = self ? s.code[e] : 0u;
    if (self)
        for (int q = 0; q < 5; ++q) Wb[q] += s.ad[rec(e, F_WD + q)];
    for (int d = 0; d < 3; ++d) {
        const int dm[3] = { -(d == 0), -(d == 1), -(d == 2) };
        const bool lo = is_predicted(g, i + dm[0], j + dm[1], k + dm[2]);
        const bool hi = is_predicted(g, i - dm[0], j - dm[1], k - dm[2]);
        const int el = lo ? ext(g, i + dm[0], j + dm[1], k + dm[2]) : 0;
        const int eh = hi ? ext(g, i - dm[0], j - dm[1], k - dm[2]) : 0;
        const unsigned cl = lo ? s.code[el] : 0u;
        const unsigned ch = hi ? s.code[eh] : 0u;
        for (int q = 0; q < 5; ++q) {
            const int dq = d * 5 + q;
            double v = 0.0, pa, pb;
            if (self) {
                branch_partials<LIM>((cs >> (2 * dq)) & 3u, pa, pb);
                const double x = s.ad[rec(e, F_SB + dq)];
                v += pa * x - pb * x;
            }
            if (lo) {
                branch_partials<LIM>((cl >> (2 * dq)) & 3u, pa, pb);
                v += pb * s.ad[rec(el, F_SB + dq)];
            }
            if (hi) {
                branch_partials<LIM>((ch >> (2 * dq)) & 3u, pa, pb);
                v -= pa * s.ad[rec(eh, F_SB + dq)];
            }
            Wb[q] += v;
        }
    }
}

__device__ __forceinline__ void prim_adjoint(const Geo &g, const double U[5], const double Wb[5],
                                             double Ub[5])
{
    const bool rho_fl = U[0] < g.rho_floor;
    const double rho = rho_fl ? g.rho_floor : U[0];
    const double ir = fast_rcp(rho);
    const double vel[3] = { U[1] * ir, U[2] * ir, U[3] * ir };
    const double kin = 0.5 * (U[1] * vel[0] + U[2] * vel[1] + U[3] * vel[2]);
    const double p = (g.gamma - 1.0) * (U[4] - kin);
    const double pb = p < g.p_floor ? 0.0 : Wb[4];
    Ub[4] = (g.gamma - 1.0) * pb;
    const double kb = -(g.gamma - 1.0) * pb;
    double rhob = Wb[0];
    for (int d = 0; d < 3; ++d) {
        // kin = sum_d m_d vel_d / 2, vel_d = m_d / rho
        const double vb = Wb[1 + d] + 0.5 * kb * U[1 + d];
        Ub[1 + d] = 0.5 * kb * vel[d] + vb * ir;
        rhob -= vb * vel[d] * ir;
    }
    Ub[0] = rho_fl ? 0.0 : rhob;
}

// One thread per input cell; blocks of 64 x 4 cover x-rows of the input box.
template <int LIM>
__global__ __launch_bounds__(256) void k_input(Geo g, const double *__restrict__ u,
                                               const double *__restrict__ lam_out,
                                               double *__restrict__ lam_in, Scratch s)
{
    const int ci = blockIdx.x * 64 + threadIdx.x % 64;
    const int cj = blockIdx.y * 4 + threadIdx.x / 64;
    const int ck = blockIdx.z;
    if (ci >= g.gx || cj >= g.gy) return;
    const int c = (ck * g.gy + cj) * g.gx + ci;
    const int o = g.periodic ? 0 : g.ng;
    const int i = ci - o, j = cj - o, k = ck - o;
    double Wb[5] = { 0, 0, 0, 0, 0 };
    const bool read = g.periodic ||
                      (i >= -2 && i < g.nx + 2 && j >= -2 && j < g.ny + 2 && k >= -2 &&
                       k < g.nz + 2 && is_read(g, i, j, k));
    if (read) gather_wbar<LIM>(g, s, i, j, k, Wb);
    double Ub[5] = { 0, 0, 0, 0, 0 };
    if (read) {
        double U[5];
        for (int q = 0; q < 5; ++q) U[q] = u[c + q * g.vin];
        prim_adjoint(g, U, Wb, Ub);
    }
    const bool inside = i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz;
    const int ii = inside ? interior_index(g, i, j, k) : 0;
    for (int q = 0; q < 5; ++q) {
        double v = Ub[q];
        if (inside) v += lam_out[q * g.nint + ii];
        __builtin_nontemporal_store(v, &lam_in[c + q * g.vin]);
    }
}

}  // namespace adj

size_t adjoint_scratch_bytes(const PatchDesc &P)
{
    const int pad = P.periodic ? 0 : 4;
    const int64_t E = (int64_t)(P.nx + pad) * (P.ny + pad) * (P.nz + pad);
    const int64_t Ep = (E + 63) / 64 * 64;
    // two records of 20 doubles and one branch word per extended cell
    return (size_t)(2 * adj::NF * Ep) * sizeof(double) + (size_t)Ep * sizeof(unsigned);
}

bool adjoint_fits_32bit(const PatchDesc &P)
{
    const int pad = P.periodic ? 0 : 4;
    const int64_t E = (int64_t)(P.nx + pad) * (P.ny + pad) * (P.nz + pad);
    const int64_t g = P.periodic ? 0 : 2 * (int64_t)P.ng;
    const int64_t vin = (P.nx + g) * (P.ny + g) * (P.nz + g);
    return adj::NF * (E + 63) < INT32_MAX && 5 * vin < INT32_MAX;
}

template <int LIM, int RS>
static int run_adjoint(const PatchDesc &P, const double *u_in, const double *lam_out,
                       const double *lam_bflux, double *lam_in, const Scalars &sc, double dt,
                       double *scratch, hipStream_t st)
{
    adj::Geo g{};
    g.nx = P.nx; g.ny = P.ny; g.nz = P.nz; g.ng = P.ng; g.periodic = P.periodic;
    const int pad = P.periodic ? 0 : 4;
    g.ex = P.nx + pad; g.ey = P.ny + pad; g.ez = P.nz + pad;
    g.E = g.ex * g.ey * g.ez;
    g.lo = P.periodic ? 0 : -1;
    g.px = P.periodic ? P.nx : P.nx + 2;
    g.py = P.periodic ? P.ny : P.ny + 2;
    g.pz = P.periodic ? P.nz : P.nz + 2;
    g.gx = P.periodic ? P.nx : P.nx + 2 * P.ng;
    g.gy = P.periodic ? P.ny : P.ny + 2 * P.ng;
    g.gz = P.periodic ? P.nz : P.nz + 2 * P.ng;
    g.vin = g.gx * g.gy * g.gz;
    g.nint = P.nx * P.ny * P.nz;
    g.ntx = (g.px + adj::CTX - 1) / adj::CTX;
    g.nty = (g.py + adj::CTY - 1) / adj::CTY;
    // z-segments: about 1024 work items, at least 4 planes each
    {
        const int tiles = g.ntx * g.nty;
        int nseg = (1024 + tiles - 1) / tiles;
        nseg = std::max(1, std::min(nseg, g.pz / 4));
        g.zlen = (g.pz + nseg - 1) / nseg;
        g.nseg = (g.pz + g.zlen - 1) / g.zlen;
    }
    g.nitem = g.ntx * g.nty * g.nseg;
    g.per_xcd = (g.nitem + 7) / 8;
    g.gamma = sc.gamma; g.inv_gm1 = 1.0 / (sc.gamma - 1.0);
    g.rho_floor = sc.rho_floor; g.p_floor = sc.p_floor;
    g.lam = dt / (2.0 * P.dx);
    g.c = dt / P.dx;
    adj::Scratch s{};
    const size_t Ep = ((size_t)g.E + 63) / 64 * 64;
    s.fw = scratch;
    s.ad = scratch + adj::NF * Ep;
    s.code = reinterpret_cast<unsigned *>(scratch + 2 * adj::NF * Ep);
    const int npred = g.px * g.py * g.pz;
    hipLaunchKernelGGL(adj::k_predict<LIM>, dim3((npred + 255) / 256), dim3(256), 0, st, g, u_in,
                       s);
    hipLaunchKernelGGL(adj::k_cells<RS>, dim3(8 * g.per_xcd), dim3(adj::CT), 0, st, g, u_in,
                       lam_out, lam_bflux, s);
    hipLaunchKernelGGL(adj::k_input<LIM>, dim3((g.gx + 63) / 64, (g.gy + 3) / 4, g.gz), dim3(256),
                       0, st, g, u_in, lam_out, lam_in, s);
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
