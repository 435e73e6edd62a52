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
PINS = {FWD: "test_oracle_pins.py", ADJ: "test_oracle_pins.py", MHD: "test_mhd_oracle_pins.py"}

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
]


def _run_mutant(case):
    fname, text, repl, what = case
    with tempfile.TemporaryDirectory() as tmp:
        for f in (FWD, ADJ, MHD):
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


def test_every_planted_mistake_fails_a_pin():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(_run_mutant, MUTATIONS))
    bad = [(w, r) for w, r in results if r != "caught"]
    assert not bad, bad
