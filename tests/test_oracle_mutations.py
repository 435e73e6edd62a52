"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake -- a dropped term, a wrong sign, a swapped index
or operand -- in a private copy of the oracle's C sources, builds it, and runs
the pin suite against that copy: the suite must fail. The repository's oracle
is never modified.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
FWD, ADJ, MHD = "godunov_oracle.c", "godunov_oracle_adjoint.c", "mhd_oracle.c"
AMR, PPMF = "amr.py", "ppm_oracle.c"
PINS = {FWD: "test_oracle_pins.py", ADJ: "test_oracle_pins.py", MHD: "test_mhd_oracle_pins.py",
        AMR: "test_amr_oracle_pins.py", PPMF: "test_ppm_oracle_pins.py"}

# (file, text, replacement, the mistake it plants)
MUTATIONS = [
    (FWD, "(adv[0] + rho * divu)", "(adv[0])", "density predictor drops rho div(u)"),
    (FWD, "(adv[4] + P->gamma * p * divu)", "(adv[4] + p * divu)", "pressure predictor drops gamma"),
    (FWD, "Ws[2] = vel[1] - lam * (adv[2] + S[1][4] / rho);",
     "Ws[2] = vel[1] - lam * (adv[2] + S[0][4] / rho);", "y-velocity predictor uses dp/dx"),
    (FWD, "WL[q] = Ws[5 * cl + q] + 0.5 * S[15 * cl + 5 * d + q];",
     "WL[q] = Ws[5 * cl + q] - 0.5 * S[15 * cl + 5 * d + q];", "left face state sign"),
    (FWD, "limited_slope(P->limiter, W[5 * c + q] - W[5 * cm + q],",
     "limited_slope(P->limiter, W[5 * cm + q] - W[5 * c + q],", "slope difference transposed"),
    (FWD, "*SL = r_min(L[1] - cL, R[1] - cR);", "*SL = r_min(L[1] - cL, R[1] + cR);",
     "Davis lower speed sign"),
    (FWD, "(Sstar + K[4] / mK)", "(Sstar - K[4] / mK)", "HLLC star energy sign"),
    (FWD, "Us[2] = a * K[2];", "Us[2] = a * K[3];", "HLLC transverse momentum index"),
    (FWD, "((xp[q] - xm[q]) + (yp[q] - ym[q])) + (zp[q] - zm[q])",
     "((xp[q] - xm[q]) + (yp[q] - ym[q])) + (zm[q] - zp[q])", "z flux difference sign"),
    (FWD, "(P->gamma - 1.0) * (U[4] - kinetic)", "(P->gamma - 1.0) * (U[4] + kinetic)",
     "pressure from total energy"),
    (FWD, "bxp[o] = Fx[5 * (((size_t)k * ny + j) * (nx + 1) + nx) + q];",
     "bxp[o] = Fx[5 * (((size_t)k * ny + j) * (nx + 1) + nx - 1) + q];", "x+ boundary sheet index"),
    (FWD, "int same_sign = (RE(a) > 0.0 && RE(b) > 0.0) || (RE(a) < 0.0 && RE(b) < 0.0);",
     "int same_sign = (RE(a) > 0.0 && RE(b) > 0.0);", "limiter same-sign test"),
    (ADJ, "Sb[m][4] -= lam * mb[m] / rho;", "Sb[m][4] += lam * mb[m] / rho;",
     "adjoint of the pressure-gradient term"),
    (ADJ, "Lb[0] += mLb * (SL - L[1]);", "Lb[0] += mLb * (SR - L[1]);",
     "adjoint of the left wave mass flux"),
    (MHD, "- (WR[8] - WL[8]) / (2.0 * ch);", "+ (WR[8] - WL[8]) / (2.0 * ch);",
     "GLM normal field: sign of the psi jump"),
    (MHD, "vs = v - By * t;", "vs = v + By * t;", "HLLD star transverse velocity sign"),
    (MHD, "double q = (rho * (S - u) * (S - u) - Bn * Bn) / den;",
     "double q = (rho * (S - u) * (S - u) + Bn * Bn) / den;", "HLLD star transverse field"),
    (MHD, "Us[0][4] - sqr[0] * (uBs - uBss) * sgn", "Us[0][4] + sqr[0] * (uBs - uBss) * sgn",
     "HLLD left double-star energy sign"),
    (MHD, "un * B[k] - vel[k] * Bn;", "un * B[k] + vel[k] * Bn;", "induction flux sign"),
    (MHD, "rho * un * vel[k] - Bn * B[k]", "rho * un * vel[k] + Bn * B[k]", "magnetic tension sign"),
    (MHD, "4.0 * a2 * bn2", "2.0 * a2 * bn2", "fast magnetosonic speed"),
    (MHD, "(U[4] - kin - mag)", "(U[4] - kin)", "pressure ignores the magnetic energy"),
    (MHD, "exp(-P->alpha", "exp(P->alpha", "psi damping grows instead"),
    (MHD, "const double h = P->dt / (2.0 * P->dx);", "const double h = P->dt / P->dx;",
     "full step instead of a half step in the predictor"),
    (AMR, "corr = c * (Ff - Fc) if side else c * (Fc - Ff)",
     "corr = c * (Fc - Ff) if side else c * (Ff - Fc)", "reflux correction sign"),
    (AMR, "blk = sheet[:, loc[2]:loc[2] + 2, loc[1]:loc[1] + 2]",
     "blk = sheet[:, loc[1]:loc[1] + 2, loc[2]:loc[2] + 2]", "x sheet read transposed"),
    (AMR, "right = out_cell if side else cell", "right = cell if side else out_cell",
     "coarse flux taken at the wrong face"),
    (AMR, "o[d] = (c[d] + (1 if side else -1)) % nc", "o[d] = (c[d] + 1) % nc",
     "lower-side interface corrects the wrong cell"),
    (AMR, "c = dt / dxc\n", "c = dt / (2 * dxc)\n", "reflux scaled by the fine spacing"),
    (AMR, "(blk[:, 1, 0] + blk[:, 1, 1])) * 0.25", "(blk[:, 1, 0] + blk[:, 1, 1])) * 0.5",
     "fine flux summed instead of averaged"),
    (AMR, "(z[0] + z[1]) * 0.125", "(z[0] + z[1]) * 0.25", "average down over four children"),
    (AMR, "uc = coarse[:, cz, cy, cx]", "uc = coarse[:, cy, cz, cx]",
     "coarse parent with y and z swapped"),
    (AMR, "return uc + 0.25 * ((sx + sy) + sz)", "return uc + 0.5 * ((sx + sy) + sz)",
     "prolongation slope doubled"),
    (AMR, "(slope[d] if g % 2 else -slope[d]", "(-slope[d] if g % 2 else slope[d]",
     "prolongation slope with its sign reversed"),
    (AMR, "np.where(np.abs(a) <= np.abs(b), a, b))", "np.where(np.abs(a) <= np.abs(b), b, a))",
     "prolongation limiter taking the larger slope"),
    (AMR, "gx = (2 * h.lo[p][0] + ii - 2) % m", "gx = (2 * h.lo[p][0] + ii - 1) % m",
     "ghost position off by one"),
    (AMR, "gz - 2 * h.lo[q][2] + 2,", "gz - 2 * h.lo[q][2] + 1,", "fine source cell off by one"),
    (AMR, "dxc / 2, dt,", "dxc, dt,", "fine patches stepped at the coarse spacing"),
    (PPMF, "return 0.5 * (a0 + ap) - (d1 - d0) / 6.0;", "return 0.5 * (a0 + ap) + (d1 - d0) / 6.0;",
     "PPM interface correction sign"),
    (PPMF, "return 0.5 * (a0 + ap) - (d1 - d0) / 6.0;", "return 0.5 * (a0 + ap) - (d1 - d0) / 3.0;",
     "PPM interface correction weight"),
    (PPMF, "return 0.5 * (ap - am);", "return 0.5 * (ap - a0);", "unlimited PPM slope one-sided"),
    (PPMF, "l = 3.0 * a0 - 2.0 * r;", "l = 3.0 * a0 - 2.0 * l;", "PPM overshoot fix of the left edge"),
    (PPMF, "r = 3.0 * a0 - 2.0 * l;", "r = 2.0 * a0 - l;", "PPM overshoot fix of the right edge"),
    (PPMF, "            l = a0;\n            r = a0;", "            r = a0;",
     "PPM extremum flattens one edge only"),
    (PPMF, "if (limiter == LIM_PPM) {", "if (limiter == LIM_PPM_NONE) {",
     "monotonicity applied to the unlimited parabola"),
    (PPMF, "s[d][q] = aR - aL;", "s[d][q] = aL - aR;", "PPM predictor slope sign"),
    (PPMF, "WL[q] = Ws[5 * cl + q] + (E[30 * cl + 10 * d + 5 + q] - W[5 * cl + q]);",
     "WL[q] = Ws[5 * cl + q] + (E[30 * cl + 10 * d + q] - W[5 * cl + q]);",
     "left face state from the lower edge"),
    (PPMF, "WR[q] = Ws[5 * cr + q] + (E[30 * cr + 10 * d + q] - W[5 * cr + q]);",
     "WR[q] = Ws[5 * cr + q] - (E[30 * cr + 10 * d + q] - W[5 * cr + q]);",
     "right face state offset sign"),
    (PPMF, "size_t cpp = ext3_index(&B, i + 2 * di, j + 2 * dj, k + 2 * dk);",
     "size_t cpp = ext3_index(&B, i + di, j + dj, k + dk);", "PPM stencil's far right cell"),
    (PPMF, "return -0.5 * s * (da - (1.0 - 2.0 * s / 3.0) * a6);",
     "return -0.5 * s * (da - (1.0 - s / 3.0) * a6);", "tracing: upper average's curvature weight"),
    (PPMF, "return 0.5 * t * (da + (1.0 - 2.0 * t / 3.0) * a6);",
     "return 0.5 * t * (da - (1.0 - 2.0 * t / 3.0) * a6);", "tracing: lower average's curvature sign"),
    (PPMF, "out[n] += sg * c / rho * beta;", "out[n] += sg * rho / c * beta;",
     "tracing: acoustic eigenvector's velocity component"),
    (PPMF, "if (upper ? !(RE(s[w]) > 0.0) : !(RE(s[w]) < 0.0)) continue;",
     "if (upper ? !(RE(s[w]) > -1.0) : !(RE(s[w]) < 1.0)) continue;",
     "tracing: waves moving away from the face included"),
    (PPMF, "for (int q = 0; q < 5; q++) fs[d][side][q] += Wt[q] - W[5 * c + q];",
     "for (int q = 0; q < 5; q++) fs[d][side][q] += 0.0 * (Wt[q] - W[5 * c + q]);",
     "tracing: transverse terms dropped"),
    (PPMF, "out[0] += D[0] - D[4] / (c * c);", "out[0] += D[0] + D[4] / (c * c);",
     "tracing: entropy wave's pressure weight"),
]


def _run_mutant(case):
    fname, text, repl, what = case
    if fname == AMR:
        return _run_python_mutant(case)
    with tempfile.TemporaryDirectory() as tmp:
        for f in (FWD, ADJ, MHD, PPMF):
            shutil.copy(os.path.join(ORACLE, f), tmp)
        path = os.path.join(tmp, fname)
        src = open(path).read()
        if src.count(text) != 1:
            return what, "pattern not found exactly once"
        open(path, "w").write(src.replace(text, repl))
        env = dict(os.environ, OMP_NUM_THREADS="2")
        build = subprocess.run(
            [sys.executable, "-c",
             f"import sys; sys.path.insert(0, {ROOT!r}); import oracle; "
             f"oracle.build(src_dir={tmp!r}, out_dir={tmp!r})"],
            env=env, capture_output=True, text=True)
        if build.returncode != 0:
            return what, "mutant does not compile: " + build.stderr[-300:]
        env["ORACLE_LIB_DIR"] = tmp
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", PINS[fname])],
                           cwd=ROOT, env=env, capture_output=True, text=True)
        return what, ("caught" if r.returncode != 0 else "NOT CAUGHT")


def _run_python_mutant(case):
    """The AMR oracle is Python: the pins load a mutated copy of it named by
    ORACLE_AMR_FILE, on top of the repository's own compiled oracle."""
    fname, text, repl, what = case
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, fname)
        src = open(os.path.join(ORACLE, fname)).read()
        if src.count(text) != 1:
            return what, "pattern not found exactly once"
        open(path, "w").write(src.replace(text, repl))
        env = dict(os.environ, OMP_NUM_THREADS="2", ORACLE_AMR_FILE=path)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", PINS[fname])],
                           cwd=ROOT, env=env, capture_output=True, text=True)
        return what, ("caught" if r.returncode != 0 else "NOT CAUGHT")


def test_every_planted_mistake_fails_a_pin():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(_run_mutant, MUTATIONS))
    bad = [(w, r) for w, r in results if r != "caught"]
    assert not bad, bad
