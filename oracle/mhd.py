"""Plain FP64 CPU oracle of the ideal-MHD step (HLLD + GLM divergence
cleaning) on periodic boxes: ctypes wrapper of ``libmhd_oracle.so``.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/`` may import
it. The scheme is described in ``mhd_oracle.c``: the Euler step's method
family (Sec. 2) carried to the MHD equations of the paper's Enzo solver
(Sec. 4), with Miyoshi & Kusano's HLLD fluxes and Dedner et al.'s
hyperbolic-parabolic cleaning of div B.

Arrays are [9][nz][ny][nx] float64, variables (rho, rho u, rho v, rho w, E,
Bx, By, Bz, psi); primitive vectors (rho, u, v, w, p, Bx, By, Bz, psi).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _LIB_DIR, LIMITERS, P_FLOOR, RHO_FLOOR, build

_PATH = os.path.join(_LIB_DIR, "libmhd_oracle.so")
_lib_handle = None


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("limiter", ctypes.c_int),
        ("gamma", ctypes.c_double), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("ch", ctypes.c_double), ("alpha", ctypes.c_double),
        ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
    ]


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_PATH):
            build()
        lib = ctypes.CDLL(_PATH)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.c_void_p
        lib.mhd_step.argtypes = [P, dp, dp]
        lib.mhd_step.restype = ctypes.c_long
        lib.mhd_face_flux.argtypes = [P, ctypes.c_int, dp, dp, dp]
        lib.mhd_phys_flux.argtypes = [P, ctypes.c_int, dp, dp]
        lib.mhd_fast_speed.argtypes = [P, ctypes.c_int, dp]
        lib.mhd_fast_speed.restype = ctypes.c_double
        lib.mhd_primitive.argtypes = [P, dp, dp]
        lib.mhd_primitive.restype = ctypes.c_int
        lib.mhd_max_speeds.argtypes = [P, dp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
        _lib_handle = lib
    return _lib_handle


def _problem(shape=(9, 1, 1, 1), gamma=5.0 / 3.0, dx=1.0, dt=0.0, ch=1.0, alpha=0.0,
             limiter="minmod", rho_floor=RHO_FLOOR, p_floor=P_FLOOR):
    _, nz, ny, nx = shape
    return _Problem(nx, ny, nz, LIMITERS[limiter], float(gamma), float(dx), float(dt),
                    float(ch), float(alpha), float(rho_floor), float(p_floor))


def step(u, gamma, dx, dt, ch, *, alpha=0.0, limiter="minmod", rho_floor=RHO_FLOOR,
         p_floor=P_FLOOR):
    """One step of the periodic box u; returns (u_out, floor_hits)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.ndim != 4 or u.shape[0] != 9:
        raise ValueError("u must be [9][nz][ny][nx]")
    P = _problem(u.shape, gamma, dx, dt, ch, alpha, limiter, rho_floor, p_floor)
    out = np.empty_like(u)
    hits = _lib().mhd_step(ctypes.byref(P), u.ctypes.data, out.ctypes.data)
    if hits < 0:
        raise ValueError("oracle rejected the problem")
    return out, int(hits)


def max_speeds(u, gamma, rho_floor=RHO_FLOOR, p_floor=P_FLOOR):
    """(max over cells of sum_d (|u_d| + cf_d), max over cells and d of |u_d| + cf_d)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    P = _problem(u.shape, gamma, rho_floor=rho_floor, p_floor=p_floor)
    a, b = ctypes.c_double(), ctypes.c_double()
    _lib().mhd_max_speeds(ctypes.byref(P), u.ctypes.data, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def cfl(u, gamma, dx, cfl=0.4):
    """(dt, ch): dt = C dx / max sum_d (|u_d| + cf_d); ch = max_d (|u_d| + cf_d)."""
    s, m = max_speeds(u, gamma)
    return cfl * dx / s, m


def face_flux(d, WL, WR, gamma, ch):
    P = _problem(gamma=gamma, ch=ch)
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.empty(9)
    _lib().mhd_face_flux(ctypes.byref(P), int(d), WL.ctypes.data, WR.ctypes.data, F.ctypes.data)
    return F


def phys_flux(d, W, gamma, ch):
    P = _problem(gamma=gamma, ch=ch)
    W = np.ascontiguousarray(W, dtype=np.float64)
    F = np.empty(9)
    _lib().mhd_phys_flux(ctypes.byref(P), int(d), W.ctypes.data, F.ctypes.data)
    return F


def fast_speed(d, W, gamma):
    P = _problem(gamma=gamma)
    W = np.ascontiguousarray(W, dtype=np.float64)
    return float(_lib().mhd_fast_speed(ctypes.byref(P), int(d), W.ctypes.data))


def primitive(U, gamma):
    P = _problem(gamma=gamma)
    U = np.ascontiguousarray(U, dtype=np.float64)
    W = np.empty(9)
    hits = _lib().mhd_primitive(ctypes.byref(P), U.ctypes.data, W.ctypes.data)
    return W, int(hits)
