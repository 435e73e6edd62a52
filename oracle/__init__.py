"""Plain FP64 CPU oracle of the unsplit MUSCL-Hancock Godunov step.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The GPU library never
loads it, and it shares no code with the GPU path: the C sources here are
compiled by gcc into ``liboracle.so`` (double), ``liboracle_cs.so``
(double complex, a complex-step tangent-linear model of the same forward code)
``libmhd_oracle.so`` (the ideal-MHD step, wrapped by ``oracle.mhd``) and
``libppm_oracle.so`` (the step with piecewise-parabolic reconstruction,
reached through ``step(..., limiter="ppm" | "ppm_unlimited", ng=3)``);
``oracle.amr`` (Python) runs one step of a two-level hierarchy -- ghost fill,
refluxing, averaging down -- around the single-patch step.

The step follows the paper's method family (Sec. 2: Euler equations of an
ideal gas, piecewise-linear Godunov scheme; Sec. 3: ghost-zoned patches;
Sec. 4: every face flux computed, boundary fluxes returned for flux
correction), made concrete as textbook MUSCL-Hancock with HLLC/HLL fluxes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# The pin tests can be pointed at a deliberately broken copy of the oracle
# (tests/test_oracle_mutations.py) through ORACLE_LIB_DIR.
_LIB_DIR = os.environ.get("ORACLE_LIB_DIR", _HERE)
_LIB = os.path.join(_LIB_DIR, "liboracle.so")
_LIB_CS = os.path.join(_LIB_DIR, "liboracle_cs.so")
_LIB_PPM = os.path.join(_LIB_DIR, "libppm_oracle.so")

LIMITERS = {"minmod": 0, "mc": 1, "none": 2, "unlimited": 2, "ppm": 3, "ppm_unlimited": 4,
            "ppm_ct": 5, "ppm_ct_unlimited": 6}
PPM = ("ppm", "ppm_unlimited", "ppm_ct", "ppm_ct_unlimited")
RIEMANN = {"hllc": 0, "hll": 1}
RHO_FLOOR = 1e-10
P_FLOOR = 1e-10


def build(verbose: bool = False, src_dir: str = _HERE, out_dir: str = _HERE,
          extra_flags=(), cc: str = "gcc") -> None:
    """Compile the oracle libraries (plain C11 + OpenMP, gcc by default). The
    default build has no FMA contraction (x86-64-v2); extra_flags (e.g.
    "-mfma", "-ffp-contract=fast") give another valid rounding of the same
    arithmetic, or sanitizer instrumentation."""
    common = [cc, "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-march=x86-64-v2",
              *extra_flags]
    cmds = [
        common + ["-o", os.path.join(out_dir, "liboracle.so"),
                  os.path.join(src_dir, "godunov_oracle_adjoint.c"), "-lm"],
        common + ["-DORACLE_COMPLEX_STEP", "-o", os.path.join(out_dir, "liboracle_cs.so"),
                  os.path.join(src_dir, "godunov_oracle.c"), "-lm"],
    ]
    mhd_src = os.path.join(src_dir, "mhd_oracle.c")
    if os.path.exists(mhd_src):
        cmds.append(common + ["-o", os.path.join(out_dir, "libmhd_oracle.so"), mhd_src, "-lm"])
    ppm_src = os.path.join(src_dir, "ppm_oracle.c")
    if os.path.exists(ppm_src):
        cmds.append(common + ["-o", os.path.join(out_dir, "libppm_oracle.so"), ppm_src, "-lm"])
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("ng", ctypes.c_int), ("periodic", ctypes.c_int),
        ("limiter", ctypes.c_int), ("riemann", ctypes.c_int),
        ("gamma", ctypes.c_double), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
    ]


_libs: dict[str, ctypes.CDLL] = {}


def _load(path: str) -> ctypes.CDLL:
    if path not in _libs:
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        _libs[path] = lib
    return _libs[path]


def _lib() -> ctypes.CDLL:
    lib = _load(_LIB)
    P = ctypes.POINTER(_Problem)
    dp = ctypes.c_void_p
    lib.orc_step.argtypes = [P, dp, dp, dp]
    lib.orc_step.restype = ctypes.c_long
    lib.orc_max_signal.argtypes = [P, dp]
    lib.orc_max_signal.restype = ctypes.c_double
    lib.orc_step_adjoint.argtypes = [P, dp, dp, dp, dp]
    lib.orc_step_adjoint.restype = ctypes.c_long
    lib.orc_face_flux.argtypes = [P, ctypes.c_int, dp, dp, dp]
    lib.orc_face_flux.restype = None
    lib.orc_primitive.argtypes = [P, dp, dp]
    lib.orc_primitive.restype = ctypes.c_long
    return lib


def _lib_cs() -> ctypes.CDLL:
    lib = _load(_LIB_CS)
    P = ctypes.POINTER(_Problem)
    dp = ctypes.c_void_p
    lib.orc_step_cs.argtypes = [P, dp, dp, dp]
    lib.orc_step_cs.restype = ctypes.c_long
    lib.orc_face_flux_cs.argtypes = [P, ctypes.c_int, dp, dp, dp]
    lib.orc_face_flux_cs.restype = None
    return lib


def _lib_ppm() -> ctypes.CDLL:
    lib = _load(_LIB_PPM)
    P = ctypes.POINTER(_Problem)
    dp = ctypes.c_void_p
    lib.orc_step_ppm.argtypes = [P, dp, dp, dp]
    lib.orc_step_ppm.restype = ctypes.c_long
    lib.orc_ppm_edges.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.orc_ppm_edges.restype = None
    lib.orc_ppm_trace.argtypes = [P, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp]
    lib.orc_ppm_trace.restype = None
    return lib


def ppm_trace(W, aL, aR, d, upper, gamma, dx, dt):
    """The characteristically traced state on the upper (upper=True) or lower
    face along axis d of a cell with primitive state W and parabola edges
    aL, aR (five primitives each), before the transverse terms."""
    P = _Problem(1, 1, 1, 3, 1, LIMITERS["ppm_ct"], 0, float(gamma), float(dx), float(dt),
                 RHO_FLOOR, P_FLOOR)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (W, aL, aR)]
    out = np.empty(5)
    _lib_ppm().orc_ppm_trace(ctypes.byref(P), *(a.ctypes.data for a in arrs), int(d), int(upper),
                             out.ctypes.data)
    return out


def ppm_edges(a5, limiter="ppm"):
    """Edge values (a_L, a_R) of the parabola of the middle of five cell values."""
    a = np.ascontiguousarray(a5, dtype=np.float64)
    if a.shape != (5,):
        raise ValueError("five cell values")
    aL, aR = ctypes.c_double(), ctypes.c_double()
    _lib_ppm().orc_ppm_edges(LIMITERS[limiter], a.ctypes.data, ctypes.byref(aL), ctypes.byref(aR))
    return aL.value, aR.value


def _problem(shape, *, gamma, dx, dt, ng, periodic, limiter, riemann, rho_floor, p_floor):
    if len(shape) != 4 or shape[0] != 5:
        raise ValueError(f"state must have shape (5, z, y, x), got {shape}")
    gz, gy, gx = shape[1:]
    if periodic:
        nz, ny, nx = gz, gy, gx
        ng = 0
    else:
        nz, ny, nx = gz - 2 * ng, gy - 2 * ng, gx - 2 * ng
    return _Problem(nx, ny, nz, ng, int(bool(periodic)), LIMITERS[limiter], RIEMANN[riemann],
                    float(gamma), float(dx), float(dt), float(rho_floor), float(p_floor))


def bflux_size(nx: int, ny: int, nz: int) -> int:
    return 10 * (nz * ny + nz * nx + ny * nx)


def split_bflux(b: np.ndarray, nx: int, ny: int, nz: int) -> dict:
    """View the flat boundary-flux buffer as its six named sheets."""
    sx, sy, sz = 5 * nz * ny, 5 * nz * nx, 5 * ny * nx
    o = np.cumsum([0, sx, sx, sy, sy, sz])
    return {
        "x-": b[o[0]:o[0] + sx].reshape(5, nz, ny), "x+": b[o[1]:o[1] + sx].reshape(5, nz, ny),
        "y-": b[o[2]:o[2] + sy].reshape(5, nz, nx), "y+": b[o[3]:o[3] + sy].reshape(5, nz, nx),
        "z-": b[o[4]:o[4] + sz].reshape(5, ny, nx), "z+": b[o[5]:o[5] + sz].reshape(5, ny, nx),
    }


def step(u, gamma, dx, dt, *, ng=2, periodic=False, limiter="minmod", riemann="hllc",
         rho_floor=RHO_FLOOR, p_floor=P_FLOOR):
    """One Godunov step. Returns (u_out [5,nz,ny,nx], flat bflux, floor_hits)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    P = _problem(u.shape, gamma=gamma, dx=dx, dt=dt, ng=ng, periodic=periodic,
                 limiter=limiter, riemann=riemann, rho_floor=rho_floor, p_floor=p_floor)
    out = np.empty((5, P.nz, P.ny, P.nx))
    bflux = np.empty(bflux_size(P.nx, P.ny, P.nz))
    fn = _lib_ppm().orc_step_ppm if limiter in PPM else _lib().orc_step
    hits = fn(ctypes.byref(P), u.ctypes.data, out.ctypes.data, bflux.ctypes.data)
    if hits < 0:
        raise ValueError("oracle rejected the problem")
    return out, bflux, int(hits)


def step_tangent(u, v, gamma, dx, dt, *, h=1e-30, **kw):
    """Complex-step directional derivative of (u_out, bflux) along v."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    z = np.ascontiguousarray(u + 1j * h * np.asarray(v, dtype=np.float64), dtype=np.complex128)
    P = _problem(u.shape, gamma=gamma, dx=dx, dt=dt, ng=kw.get("ng", 2),
                 periodic=kw.get("periodic", False), limiter=kw.get("limiter", "minmod"),
                 riemann=kw.get("riemann", "hllc"), rho_floor=kw.get("rho_floor", RHO_FLOOR),
                 p_floor=kw.get("p_floor", P_FLOOR))
    out = np.empty((5, P.nz, P.ny, P.nx), dtype=np.complex128)
    bflux = np.empty(bflux_size(P.nx, P.ny, P.nz), dtype=np.complex128)
    if _lib_cs().orc_step_cs(ctypes.byref(P), z.ctypes.data, out.ctypes.data, bflux.ctypes.data) < 0:
        raise ValueError("oracle rejected the problem")
    return out.real.copy(), out.imag / h, bflux.imag / h


def step_adjoint(u, lam_out, gamma, dx, dt, *, lam_bflux=None, ng=2, periodic=False,
                 limiter="minmod", riemann="hllc", rho_floor=RHO_FLOOR, p_floor=P_FLOOR):
    """dL/dU^n given dL/dU^{n+1} (and optionally dL/dbflux); shape of u."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    P = _problem(u.shape, gamma=gamma, dx=dx, dt=dt, ng=ng, periodic=periodic,
                 limiter=limiter, riemann=riemann, rho_floor=rho_floor, p_floor=p_floor)
    lo = np.ascontiguousarray(lam_out, dtype=np.float64)
    if lo.shape != (5, P.nz, P.ny, P.nx):
        raise ValueError("lam_out has the wrong shape")
    lb = None
    if lam_bflux is not None:
        lb = np.ascontiguousarray(lam_bflux, dtype=np.float64)
        if lb.size != bflux_size(P.nx, P.ny, P.nz):
            raise ValueError("lam_bflux has the wrong size")
    lam_in = np.empty_like(u)
    r = _lib().orc_step_adjoint(ctypes.byref(P), u.ctypes.data, lo.ctypes.data,
                                None if lb is None else lb.ctypes.data, lam_in.ctypes.data)
    if r < 0:
        raise ValueError("oracle rejected the problem")
    return lam_in


def max_signal(u, gamma, *, ng=2, periodic=False, rho_floor=RHO_FLOOR, p_floor=P_FLOOR):
    """max over interior cells of |u|+|v|+|w|+3c."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    P = _problem(u.shape, gamma=gamma, dx=1.0, dt=0.0, ng=ng, periodic=periodic,
                 limiter="minmod", riemann="hllc", rho_floor=rho_floor, p_floor=p_floor)
    return float(_lib().orc_max_signal(ctypes.byref(P), u.ctypes.data))


def cfl_dt(u, gamma, dx, cfl=0.5, **kw):
    """dt = C dx / max(|u|+|v|+|w|+3c) over the interior."""
    return cfl * dx / max_signal(u, gamma, **kw)


def cfl_dt_batched(patches, gamma, cfl=0.5, **kw):
    """dt = min over patches of C dx_p / s_p; patches = [(u_ghosted, dx), ...]."""
    return min(cfl * dx / max_signal(u, gamma, **kw) for u, dx in patches)


def face_flux(d, WL, WR, gamma, riemann="hllc"):
    """Flux through one face normal to axis d from primitive states (unrotated)."""
    P = _Problem(1, 1, 1, 2, 0, 0, RIEMANN[riemann], float(gamma), 1.0, 0.0, RHO_FLOOR, P_FLOOR)
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.empty(5)
    _lib().orc_face_flux(ctypes.byref(P), int(d), WL.ctypes.data, WR.ctypes.data, F.ctypes.data)
    return F


def face_flux_tangent(d, WL, WR, dWL, dWR, gamma, riemann="hllc", h=1e-30):
    P = _Problem(1, 1, 1, 2, 0, 0, RIEMANN[riemann], float(gamma), 1.0, 0.0, RHO_FLOOR, P_FLOOR)
    zL = np.ascontiguousarray(np.asarray(WL) + 1j * h * np.asarray(dWL), dtype=np.complex128)
    zR = np.ascontiguousarray(np.asarray(WR) + 1j * h * np.asarray(dWR), dtype=np.complex128)
    F = np.empty(5, dtype=np.complex128)
    _lib_cs().orc_face_flux_cs(ctypes.byref(P), int(d), zL.ctypes.data, zR.ctypes.data,
                               F.ctypes.data)
    return F.imag / h


def primitive(U, gamma, rho_floor=RHO_FLOOR, p_floor=P_FLOOR):
    P = _Problem(1, 1, 1, 2, 0, 0, 0, float(gamma), 1.0, 0.0, rho_floor, p_floor)
    U = np.ascontiguousarray(U, dtype=np.float64)
    W = np.empty(5)
    hits = _lib().orc_primitive(ctypes.byref(P), U.ctypes.data, W.ctypes.data)
    return W, int(hits)
