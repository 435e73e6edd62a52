"""Python binding of libgodunov.so (ctypes), plus a differentiable rollout.

Argument marshalling only: every step of the scheme runs in the library's HIP
kernels. PyTorch supplies the device memory (tensors) and the stream (the
current torch stream). There is no CPU fallback: if the library is not built
or no GPU is present, the calls raise.

Entry points (same names as the C ABI, see include/godunov.h):
    step(u, gamma, dx, dt)            one patch (ghosted or periodic)
    step_batched(...)                 many ghost-zoned patches, one launch
    step_batched_streamed(...)        the same for a batch in host memory, streamed
                                      through the device in chunks with copy/compute
                                      overlap
    step_adjoint(u, lam_out, ...)     reverse mode of step for a fixed dt
    cfl_dt(u, gamma, dx, cfl)         CFL time step as a device scalar
    step_mhd(u, gamma, dx, dt, ch)    ideal-MHD step (HLLD + GLM) of a periodic box
    cfl_dt_mhd(u, gamma, dx, cfl)     its time step and cleaning speed
    AmrPlan(nc, dx_coarse, table)     two-level hierarchy: ghost fill, refluxing,
                                      averaging down, the whole two-level step
    GodunovRollout                    torch.autograd.Function over K steps
                                      with checkpointed recomputation
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the library to load: the in-tree build, or another build of the same
# sources named by GODUNOV_LIB (e.g. the host-sanitized one)
LIB_PATH = os.environ.get("GODUNOV_LIB", os.path.join(_HERE, "libgodunov.so"))

GD_OK, GD_E_ARG, GD_E_HIP, GD_E_NOMEM, GD_E_UNSUPPORTED = 0, -1, -2, -3, -4
DTYPES = {torch.float64: 0, torch.float32: 1}
LIMITERS = {"minmod": 0, "mc": 1, "unlimited": 2, "none": 2, "ppm": 3, "ppm_unlimited": 4,
            "ppm_ct": 5, "ppm_ct_unlimited": 6}
RIEMANN = {"hllc": 0, "hll": 1}
RHO_FLOOR = 1e-10
P_FLOOR = 1e-10


class GodunovError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


class gd_opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("bc", ctypes.c_int32), ("limiter", ctypes.c_int32),
                ("riemann", ctypes.c_int32), ("rho_floor", ctypes.c_double),
                ("p_floor", ctypes.c_double)]


class gd_patch(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ng", ctypes.c_int32), ("u_in_off", ctypes.c_int64),
                ("u_out_off", ctypes.c_int64), ("flux_off", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double)]


PATCH_DTYPE = np.dtype([("nx", "<i4"), ("ny", "<i4"), ("nz", "<i4"), ("ng", "<i4"),
                        ("u_in_off", "<i8"), ("u_out_off", "<i8"), ("flux_off", "<i8"),
                        ("dx", "<f8"), ("dt", "<f8")], align=True)
assert PATCH_DTYPE.itemsize == ctypes.sizeof(gd_patch)


class gd_amr_patch(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("n", ctypes.c_int32 * 3),
                ("u_in_off", ctypes.c_int64), ("u_out_off", ctypes.c_int64),
                ("flux_off", ctypes.c_int64)]


AMR_PATCH_DTYPE = np.dtype([("lo", "<i4", (3,)), ("n", "<i4", (3,)), ("u_in_off", "<i8"),
                            ("u_out_off", "<i8"), ("flux_off", "<i8")], align=True)
assert AMR_PATCH_DTYPE.itemsize == ctypes.sizeof(gd_amr_patch)

EXPORTS = ("gd_create", "gd_destroy", "gd_last_error", "gd_get_stats", "gd_reset_stats",
           "godunov_step", "godunov_step_batched", "godunov_step_adjoint", "cfl_dt",
           "gd_autotune_step", "gd_autotune_batched", "gd_get_config", "gd_set_config",
           "godunov_step_cfl", "godunov_step_batched_cfl", "godunov_step_mhd", "godunov_step_mhd_cfl",
           "cfl_dt_mhd", "gd_amr_create", "gd_amr_destroy", "gd_amr_fill_ghosts", "gd_amr_reflux",
           "gd_amr_step", "godunov_step_batched_streamed", "godunov_step_batched_noalloc")

_lib = None
_lock = threading.Lock()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgodunov.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        P = ctypes.POINTER
        lib.gd_create.argtypes = [P(vp), i32]
        lib.gd_destroy.argtypes = [vp]
        lib.gd_last_error.argtypes = [vp]
        lib.gd_last_error.restype = ctypes.c_char_p
        lib.gd_get_stats.argtypes = [vp, P(ctypes.c_uint64)]
        lib.gd_reset_stats.argtypes = [vp]
        lib.godunov_step.argtypes = [vp, P(gd_opts), i32, i32, i32, i32, vp, vp, vp, dbl, dbl, dbl,
                                     vp, vp]
        lib.godunov_step_batched.argtypes = [vp, P(gd_opts), i32, vp, vp, vp, vp, vp, dbl, vp]
        lib.godunov_step_adjoint.argtypes = [vp, P(gd_opts), i32, i32, i32, i32, vp, vp, vp, vp,
                                             dbl, dbl, dbl, vp]
        lib.cfl_dt.argtypes = [vp, P(gd_opts), i32, vp, vp, dbl, dbl, vp, vp]
        lib.godunov_step_cfl.argtypes = [vp, P(gd_opts), i32, i32, i32, i32, vp, vp, vp, dbl, dbl,
                                         dbl, vp, dbl, vp, vp]
        lib.godunov_step_batched_cfl.argtypes = [vp, P(gd_opts), i32, vp, vp, vp, vp, vp, dbl, dbl,
                                                 vp, vp]
        ip = P(ctypes.c_int)
        lib.gd_autotune_step.argtypes = [vp, P(gd_opts), i32, i32, i32, i32, vp, vp, dbl, dbl, dbl,
                                         vp, ip]
        lib.gd_autotune_batched.argtypes = [vp, P(gd_opts), i32, vp, vp, vp, vp, dbl, vp, ip]
        lib.gd_get_config.argtypes = [vp, i32, ip, ip, ip, ip]
        lib.gd_set_config.argtypes = [vp, i32, i32, i32, i32, i32]
        lib.godunov_step_mhd.argtypes = [vp, P(gd_opts), i32, i32, i32, vp, vp, dbl, dbl, dbl, vp,
                                         dbl, vp, dbl, vp]
        lib.cfl_dt_mhd.argtypes = [vp, P(gd_opts), i32, i32, i32, vp, dbl, dbl, dbl, vp, vp, vp]
        lib.godunov_step_mhd_cfl.argtypes = [vp, P(gd_opts), i32, i32, i32, vp, vp, dbl, dbl, dbl,
                                             vp, dbl, vp, dbl, dbl, vp, vp, vp]
        lib.gd_amr_create.argtypes = [vp, i32, i32, i32, dbl, i32, vp, P(vp)]
        lib.gd_amr_destroy.argtypes = [vp]
        lib.gd_amr_fill_ghosts.argtypes = [vp, vp, i32, vp, vp, vp]
        lib.gd_amr_reflux.argtypes = [vp, vp, P(gd_opts), vp, vp, vp, vp, dbl, dbl, vp, vp]
        lib.gd_amr_step.argtypes = [vp, vp, P(gd_opts), vp, vp, vp, vp, vp, dbl, dbl, vp, vp]
        lib.godunov_step_batched_streamed.argtypes = [vp, P(gd_opts), i32, vp, vp, vp, vp, vp, dbl,
                                                      ctypes.c_size_t, vp]
        lib.godunov_step_batched_noalloc.argtypes = [P(gd_opts), i32, vp, vp, vp, vp, vp, dbl, vp]
        for name in EXPORTS:
            if name != "gd_last_error":
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
        return lib


class Context:
    """A gd_ctx bound to one device. One per (thread, device) via `context()`."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        r = self.lib.gd_create(ctypes.byref(h), device)
        if r != GD_OK:
            raise GodunovError(r, self.lib.gd_last_error(None).decode())
        self.handle = h

    def check(self, r: int) -> None:
        if r != GD_OK:
            raise GodunovError(r, self.lib.gd_last_error(self.handle).decode())

    def floor_hits(self) -> int:
        v = ctypes.c_uint64()
        self.check(self.lib.gd_get_stats(self.handle, ctypes.byref(v)))
        return int(v.value)

    def reset_stats(self) -> None:
        self.check(self.lib.gd_reset_stats(self.handle))

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None and self.handle.value:
                self.lib.gd_destroy(self.handle)
        except Exception:
            pass


_contexts: dict = {}


def context(device=None) -> Context:
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the Godunov library has no CPU path")
    dev = torch.cuda.current_device() if device is None else int(device)
    key = (threading.get_ident(), dev)
    if key not in _contexts:
        _contexts[key] = Context(dev)
    return _contexts[key]


def _opts(dtype, periodic, limiter, riemann, rho_floor, p_floor) -> gd_opts:
    if dtype not in DTYPES:
        raise TypeError(f"unsupported dtype {dtype}")
    return gd_opts(DTYPES[dtype], 1 if periodic else 0, LIMITERS[limiter], RIEMANN[riemann],
                   float(rho_floor), float(p_floor))


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_tensor(t, name, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")


def _check_scalar(t, name):
    """A device scalar argument: a float64 CUDA tensor with at least one element."""
    _check_tensor(t, name, torch.float64)
    if t.numel() < 1:
        raise ValueError(f"{name} must hold at least one element")


def _check_size(t, name, need, shape=None):
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.numel() < need:
        raise ValueError(f"{name} holds {t.numel()} values, {need} are needed")


def bflux_size(nx, ny, nz) -> int:
    return 10 * (nz * ny + nz * nx + ny * nx)


def batch_extents(table) -> tuple:
    """Elements each buffer of a batched call must hold for the offsets in
    `table` (gd_patch records): (u_in, out, bflux); the library cannot see
    the buffers' sizes, so the binding checks them before any launch."""
    table = np.asarray(table, dtype=PATCH_DTYPE)
    if len(table) == 0:
        return 0, 0, 0
    d = np.stack([table["nx"], table["ny"], table["nz"]], axis=1).astype(np.int64)
    g = 2 * table["ng"].astype(np.int64)[:, None]
    need_in = int((table["u_in_off"] + 5 * np.prod(d + g, axis=1)).max())
    need_out = int((table["u_out_off"] + 5 * np.prod(d, axis=1)).max())
    fl = 10 * (d[:, 2] * d[:, 1] + d[:, 2] * d[:, 0] + d[:, 1] * d[:, 0])
    has = table["flux_off"] >= 0
    need_fl = int((table["flux_off"][has] + fl[has]).max()) if has.any() else 0
    return need_in, need_out, need_fl


def _check_batch(table, u_in, out=None, bflux=None):
    need_in, need_out, need_fl = batch_extents(table)
    for name, t, need in (("u_in", u_in, need_in), ("out", out, need_out), ("bflux", bflux, need_fl)):
        if t is not None:
            _check_size(t, name, need)


def interior_shape(u, ng, periodic):
    if u.dim() != 4 or u.shape[0] != 5:
        raise ValueError(f"state must have shape (5, z, y, x), got {tuple(u.shape)}")
    gz, gy, gx = u.shape[1:]
    if periodic:
        return gx, gy, gz
    return gx - 2 * ng, gy - 2 * ng, gz - 2 * ng


def step(u, gamma, dx, dt=None, *, dt_dev=None, ng=2, periodic=False, limiter="minmod",
         riemann="hllc", want_bflux=True, out=None, bflux=None, rho_floor=RHO_FLOOR,
         p_floor=P_FLOOR, stream=None, cfl=None, dt_next=None):
    """One Godunov step of one patch. Returns (u_new [5,nz,ny,nx], bflux or None).
    With cfl and dt_next (a 1-element float64 device tensor, which may be
    dt_dev itself) the launch also writes the CFL step of u_new to dt_next."""
    _check_tensor(u, "u")
    nx, ny, nz = interior_shape(u, ng, periodic)
    if out is None:
        out = torch.empty((5, nz, ny, nx), dtype=u.dtype, device=u.device)
    _check_tensor(out, "out", u.dtype)
    _check_size(out, "out", 0, (5, nz, ny, nx))
    if want_bflux and bflux is None:
        bflux = torch.empty(bflux_size(nx, ny, nz), dtype=u.dtype, device=u.device)
    if not want_bflux:
        bflux = None
    if bflux is not None:
        _check_tensor(bflux, "bflux", u.dtype)
        _check_size(bflux, "bflux", bflux_size(nx, ny, nz))
    if dt_dev is not None:
        _check_scalar(dt_dev, "dt_dev")
    if dt is None and dt_dev is None:
        raise ValueError("give dt or dt_dev")
    ctx = context(u.device.index)
    o = _opts(u.dtype, periodic, limiter, riemann, rho_floor, p_floor)
    if dt_next is not None:
        _check_scalar(dt_next, "dt_next")
        ctx.check(ctx.lib.godunov_step_cfl(ctx.handle, ctypes.byref(o), nx, ny, nz, ng, _ptr(u),
                                           _ptr(out), _ptr(bflux), float(gamma), float(dx),
                                           float(dt if dt is not None else 0.0), _ptr(dt_dev),
                                           float(0.5 if cfl is None else cfl), _ptr(dt_next),
                                           _stream(stream)))
        return out, bflux
    ctx.check(ctx.lib.godunov_step(ctx.handle, ctypes.byref(o), nx, ny, nz, ng, _ptr(u), _ptr(out),
                                   _ptr(bflux), float(gamma), float(dx),
                                   float(dt if dt is not None else 0.0), _ptr(dt_dev),
                                   _stream(stream)))
    return out, bflux


def cfl_dt(u, gamma, dx, cfl=0.5, *, ng=2, periodic=False, out=None, rho_floor=RHO_FLOOR,
           p_floor=P_FLOOR, stream=None):
    """CFL step of one patch as a 1-element float64 device tensor."""
    _check_tensor(u, "u")
    nx, ny, nz = interior_shape(u, ng, periodic)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=u.device)
    _check_scalar(out, "out")
    ctx = context(u.device.index)
    o = _opts(u.dtype, periodic, "minmod", "hllc", rho_floor, p_floor)
    desc = np.zeros(1, dtype=PATCH_DTYPE)
    desc[0] = (nx, ny, nz, 0 if periodic else ng, 0, 0, -1, float(dx), 0.0)
    ctx.check(ctx.lib.cfl_dt(ctx.handle, ctypes.byref(o), 1, desc.ctypes.data, _ptr(u),
                             float(gamma), float(cfl), _ptr(out), _stream(stream)))
    return out


def patch_table(dims, ng, u_in_off, u_out_off, flux_off, dx, dt=0.0) -> np.ndarray:
    """Structured array of gd_patch records (host memory)."""
    dims = np.asarray(dims)
    n = len(dims)
    t = np.zeros(n, dtype=PATCH_DTYPE)
    t["nx"], t["ny"], t["nz"] = dims[:, 0], dims[:, 1], dims[:, 2]
    t["ng"] = ng
    t["u_in_off"], t["u_out_off"] = u_in_off, u_out_off
    t["flux_off"] = flux_off
    t["dx"] = dx
    t["dt"] = dt
    return t


def step_batched(u_in, table, gamma, *, out, bflux=None, dt_dev=None, limiter="minmod",
                 riemann="hllc", rho_floor=RHO_FLOOR, p_floor=P_FLOOR, stream=None, cfl=None,
                 dt_next=None):
    """One step of every patch in `table` (see patch_table), one launch.
    With cfl and dt_next the launch also writes the batch's next CFL step."""
    _check_tensor(u_in, "u_in")
    _check_tensor(out, "out", u_in.dtype)
    if bflux is not None:
        _check_tensor(bflux, "bflux", u_in.dtype)
    if dt_dev is not None:
        _check_scalar(dt_dev, "dt_dev")
    table = np.ascontiguousarray(table, dtype=PATCH_DTYPE)
    _check_batch(table, u_in, out, bflux)
    ctx = context(u_in.device.index)
    o = _opts(u_in.dtype, False, limiter, riemann, rho_floor, p_floor)
    if dt_next is not None:
        _check_scalar(dt_next, "dt_next")
        ctx.check(ctx.lib.godunov_step_batched_cfl(
            ctx.handle, ctypes.byref(o), len(table), table.ctypes.data, _ptr(u_in), _ptr(out),
            _ptr(bflux), _ptr(dt_dev), float(gamma), float(0.5 if cfl is None else cfl),
            _ptr(dt_next), _stream(stream)))
        return out, bflux
    ctx.check(ctx.lib.godunov_step_batched(ctx.handle, ctypes.byref(o), len(table),
                                           table.ctypes.data, _ptr(u_in), _ptr(out), _ptr(bflux),
                                           _ptr(dt_dev), float(gamma), _stream(stream)))
    return out, bflux


def step_batched_streamed(u_in, table, gamma, *, out, bflux=None, chunk_bytes=256 << 20,
                          dt_dev=None, limiter="minmod", riemann="hllc", rho_floor=RHO_FLOOR,
                          p_floor=P_FLOOR, stream=None, device=None):
    """step_batched for a batch in host memory: u_in, out and bflux are CPU
    tensors (pinned for copy/compute overlap) in the batched layout. The call
    is asynchronous on the current (or given) stream: synchronise it before
    reading out and bflux."""
    for name, t in (("u_in", u_in), ("out", out), ("bflux", bflux)):
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or t.is_cuda:
            raise TypeError(f"{name} must be a CPU tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.dtype != u_in.dtype:
            raise TypeError(f"{name} must have dtype {u_in.dtype}")
    if dt_dev is not None:
        _check_scalar(dt_dev, "dt_dev")
    table = np.ascontiguousarray(table, dtype=PATCH_DTYPE)
    _check_batch(table, u_in, out, bflux)
    ctx = context(device)
    o = _opts(u_in.dtype, False, limiter, riemann, rho_floor, p_floor)
    ctx.check(ctx.lib.godunov_step_batched_streamed(
        ctx.handle, ctypes.byref(o), len(table), table.ctypes.data, _ptr(u_in), _ptr(out),
        _ptr(bflux), _ptr(dt_dev), float(gamma), int(chunk_bytes), _stream(stream)))
    return out, bflux


NOALLOC_MAX_PATCHES = 65536


def step_batched_noalloc(u_in, patches_dev, npatch, gamma, *, out, bflux=None, dt_dev=None,
                         table=None, limiter="minmod", riemann="hllc", rho_floor=RHO_FLOOR,
                         p_floor=P_FLOOR, stream=None):
    """godunov_step_batched_noalloc: the batched step with no allocation by
    the library. patches_dev is a uint8 CUDA tensor holding npatch gd_patch
    records (e.g. device_table(table)); the kernels read it at every launch.
    Give the host table too (table=) to have the buffers checked against its
    offsets; the library cannot see the device records on the host."""
    _check_tensor(u_in, "u_in")
    _check_tensor(out, "out", u_in.dtype)
    if bflux is not None:
        _check_tensor(bflux, "bflux", u_in.dtype)
    _check_tensor(patches_dev, "patches_dev", torch.uint8)
    _check_size(patches_dev, "patches_dev", int(npatch) * PATCH_DTYPE.itemsize)
    if patches_dev.device != u_in.device:
        raise ValueError("patches_dev must be on the device of u_in")
    if dt_dev is not None:
        _check_scalar(dt_dev, "dt_dev")
    if table is not None:
        table = np.ascontiguousarray(table, dtype=PATCH_DTYPE)
        if len(table) != npatch:
            raise ValueError("table and npatch disagree")
        _check_batch(table, u_in, out, bflux)
    lib = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the Godunov library has no CPU path")
    o = _opts(u_in.dtype, False, limiter, riemann, rho_floor, p_floor)
    with torch.cuda.device(u_in.device):
        r = lib.godunov_step_batched_noalloc(ctypes.byref(o), int(npatch), _ptr(patches_dev),
                                             _ptr(u_in), _ptr(out), _ptr(bflux), _ptr(dt_dev),
                                             float(gamma), _stream(stream))
    if r != GD_OK:
        raise GodunovError(r, lib.gd_last_error(None).decode())
    return out, bflux


def device_table(table, device=None) -> torch.Tensor:
    """The gd_patch records of a host table as a uint8 CUDA tensor."""
    table = np.ascontiguousarray(table, dtype=PATCH_DTYPE)
    return torch.from_numpy(table.view(np.uint8).copy()).to(
        torch.device("cuda", torch.cuda.current_device() if device is None else device))


def cfl_dt_batched(u_in, table, gamma, cfl=0.5, *, out=None, rho_floor=RHO_FLOOR,
                   p_floor=P_FLOOR, stream=None):
    _check_tensor(u_in, "u_in")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=u_in.device)
    _check_scalar(out, "out")
    table = np.ascontiguousarray(table, dtype=PATCH_DTYPE)
    _check_batch(table, u_in)
    ctx = context(u_in.device.index)
    o = _opts(u_in.dtype, False, "minmod", "hllc", rho_floor, p_floor)
    ctx.check(ctx.lib.cfl_dt(ctx.handle, ctypes.byref(o), len(table), table.ctypes.data,
                             _ptr(u_in), float(gamma), float(cfl), _ptr(out), _stream(stream)))
    return out


def step_adjoint(u, lam_out, gamma, dx, dt, *, lam_bflux=None, ng=2, periodic=False,
                 limiter="minmod", riemann="hllc", out=None, rho_floor=RHO_FLOOR,
                 p_floor=P_FLOOR, stream=None):
    """dL/dU^n of one step (fixed dt) from dL/dU^{n+1} (and dL/dbflux)."""
    _check_tensor(u, "u", torch.float64)
    _check_tensor(lam_out, "lam_out", torch.float64)
    nx, ny, nz = interior_shape(u, ng, periodic)
    if tuple(lam_out.shape) != (5, nz, ny, nx):
        raise ValueError("lam_out has the wrong shape")
    if lam_bflux is not None:
        _check_tensor(lam_bflux, "lam_bflux", torch.float64)
        _check_size(lam_bflux, "lam_bflux", bflux_size(nx, ny, nz))
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out", torch.float64)
    _check_size(out, "out", 0, u.shape)
    ctx = context(u.device.index)
    o = _opts(torch.float64, periodic, limiter, riemann, rho_floor, p_floor)
    ctx.check(ctx.lib.godunov_step_adjoint(ctx.handle, ctypes.byref(o), nx, ny, nz, ng, _ptr(u),
                                           _ptr(lam_out), _ptr(lam_bflux), _ptr(out),
                                           float(gamma), float(dx), float(dt), _stream(stream)))
    return out


TILE_SHAPES = ("16x16", "8x8", "32x8", "16x8", "24x8")
# a batched launch may also pair 16x8 and 24x8 tiles, the shape chosen per patch
BATCHED_SHAPES = TILE_SHAPES + ("16x8+24x8",)


def autotune_step(u, gamma, dx, dt, *, ng=2, periodic=False, limiter="minmod", riemann="hllc",
                  out=None, rho_floor=RHO_FLOOR, p_floor=P_FLOOR, stream=None) -> int:
    """Time the tile/z-range candidates of godunov_step on this problem and
    keep the fastest in the context. Returns the candidate index."""
    _check_tensor(u, "u")
    nx, ny, nz = interior_shape(u, ng, periodic)
    if out is None:
        out = torch.empty((5, nz, ny, nx), dtype=u.dtype, device=u.device)
    _check_tensor(out, "out", u.dtype)
    _check_size(out, "out", 0, (5, nz, ny, nx))
    ctx = context(u.device.index)
    o = _opts(u.dtype, periodic, limiter, riemann, rho_floor, p_floor)
    choice = ctypes.c_int(-1)
    ctx.check(ctx.lib.gd_autotune_step(ctx.handle, ctypes.byref(o), nx, ny, nz, ng, _ptr(u),
                                       _ptr(out), float(gamma), float(dx), float(dt),
                                       _stream(stream), ctypes.byref(choice)))
    return choice.value


def autotune_batched(u_in, table, gamma, *, out, bflux=None, limiter="minmod", riemann="hllc",
                     rho_floor=RHO_FLOOR, p_floor=P_FLOOR, stream=None) -> int:
    _check_tensor(u_in, "u_in")
    _check_tensor(out, "out", u_in.dtype)
    if bflux is not None:
        _check_tensor(bflux, "bflux", u_in.dtype)
    table = np.ascontiguousarray(table, dtype=PATCH_DTYPE)
    _check_batch(table, u_in, out, bflux)
    ctx = context(u_in.device.index)
    o = _opts(u_in.dtype, False, limiter, riemann, rho_floor, p_floor)
    choice = ctypes.c_int(-1)
    ctx.check(ctx.lib.gd_autotune_batched(ctx.handle, ctypes.byref(o), len(table),
                                          table.ctypes.data, _ptr(u_in), _ptr(out), _ptr(bflux),
                                          float(gamma), _stream(stream), ctypes.byref(choice)))
    return choice.value


def get_config(dtype=torch.float64) -> dict:
    ctx = context()
    v = [ctypes.c_int() for _ in range(4)]
    ctx.check(ctx.lib.gd_get_config(ctx.handle, DTYPES[dtype], *[ctypes.byref(x) for x in v]))
    return {"shape_single": TILE_SHAPES[v[0].value], "zlen_single": v[1].value,
            "shape_batched": BATCHED_SHAPES[v[2].value], "zpolicy_batched": v[3].value}


def set_config(dtype=torch.float64, *, shape_single="16x16", zlen_single=32,
               shape_batched="16x16", zpolicy_batched=1) -> None:
    ctx = context()
    ctx.check(ctx.lib.gd_set_config(ctx.handle, DTYPES[dtype], TILE_SHAPES.index(shape_single),
                                    int(zlen_single), BATCHED_SHAPES.index(shape_batched),
                                    int(zpolicy_batched)))


class GodunovRollout(torch.autograd.Function):
    """K periodic steps with a fixed dt, differentiable with respect to the
    initial state. The forward keeps every `every`-th state; the backward
    recomputes each segment from its checkpoint and runs the adjoint steps
    in reverse (checkpointed recomputation)."""

    @staticmethod
    def forward(ctx, u0, gamma, dx, dt, nsteps, every, limiter, riemann):
        u = u0.contiguous()
        checkpoints = [u]
        for k in range(nsteps):
            u, _ = step(u, gamma, dx, dt, periodic=True, limiter=limiter, riemann=riemann,
                        want_bflux=False)
            if (k + 1) % every == 0 and k + 1 < nsteps:
                checkpoints.append(u)
        ctx.save_for_backward(*checkpoints)
        ctx.args = (gamma, dx, dt, nsteps, every, limiter, riemann)
        return u

    @staticmethod
    def backward(ctx, grad_out):
        gamma, dx, dt, nsteps, every, limiter, riemann = ctx.args
        checkpoints = ctx.saved_tensors
        lam = grad_out.contiguous()
        for seg in reversed(range(len(checkpoints))):
            start = seg * every
            stop = min(start + every, nsteps)
            states = [checkpoints[seg]]
            for _ in range(start, stop - 1):
                states.append(step(states[-1], gamma, dx, dt, periodic=True, limiter=limiter,
                                   riemann=riemann, want_bflux=False)[0])
            for s in reversed(states):
                lam = step_adjoint(s, lam, gamma, dx, dt, periodic=True, limiter=limiter,
                                   riemann=riemann)
        return lam, None, None, None, None, None, None, None


def rollout(u0, gamma, dx, dt, nsteps, every=5, limiter="minmod", riemann="hllc"):
    return GodunovRollout.apply(u0, gamma, dx, dt, nsteps, every, limiter, riemann)


# ------------------------------------------------------------ ideal MHD

def _mhd_shape(u):
    if u.dim() != 4 or u.shape[0] != 9:
        raise ValueError(f"MHD state must have shape (9, z, y, x), got {tuple(u.shape)}")
    return u.shape[3], u.shape[2], u.shape[1]


def step_mhd(u, gamma, dx, dt=None, ch=None, *, dt_dev=None, ch_dev=None, alpha=0.1,
             limiter="minmod", out=None, rho_floor=RHO_FLOOR, p_floor=P_FLOOR, stream=None,
             cfl=None, dt_next=None, ch_next=None):
    """One ideal-MHD step (HLLD + GLM cleaning) of the periodic box u
    [9, nz, ny, nx]; dt and ch from host values or 1-element float64 device
    tensors. With cfl and dt_next / ch_next (1-element float64 device tensors,
    which may be dt_dev / ch_dev) the launch also writes the next step's dt
    and cleaning speed from u_new. Returns u_new."""
    _check_tensor(u, "u")
    nx, ny, nz = _mhd_shape(u)
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out", u.dtype)
    _check_size(out, "out", 0, u.shape)
    if dt is None and dt_dev is None:
        raise ValueError("give dt or dt_dev")
    if ch is None and ch_dev is None:
        raise ValueError("give ch or ch_dev")
    for t, name in ((dt_dev, "dt_dev"), (ch_dev, "ch_dev")):
        if t is not None:
            _check_scalar(t, name)
    ctx = context(u.device.index)
    o = _opts(u.dtype, True, limiter, "hllc", rho_floor, p_floor)
    if dt_next is None and ch_next is None:
        ctx.check(ctx.lib.godunov_step_mhd(ctx.handle, ctypes.byref(o), nx, ny, nz, _ptr(u),
                                           _ptr(out), float(gamma), float(dx), float(dt or 0.0),
                                           _ptr(dt_dev), float(ch or 0.0), _ptr(ch_dev),
                                           float(alpha), _stream(stream)))
        return out
    for t, name in ((dt_next, "dt_next"), (ch_next, "ch_next")):
        if t is not None:
            _check_scalar(t, name)
    if cfl is None:
        raise ValueError("dt_next / ch_next need cfl")
    ctx.check(ctx.lib.godunov_step_mhd_cfl(ctx.handle, ctypes.byref(o), nx, ny, nz, _ptr(u),
                                           _ptr(out), float(gamma), float(dx), float(dt or 0.0),
                                           _ptr(dt_dev), float(ch or 0.0), _ptr(ch_dev),
                                           float(alpha), float(cfl), _ptr(dt_next), _ptr(ch_next),
                                           _stream(stream)))
    return out


def cfl_dt_mhd(u, gamma, dx, cfl=0.4, *, out_dt=None, out_ch=None, rho_floor=RHO_FLOOR,
               p_floor=P_FLOOR, stream=None):
    """(dt, ch) of the periodic MHD box u as 1-element float64 device tensors:
    dt = cfl dx / max sum_d (|u_d| + cf_d), ch = max_d (|u_d| + cf_d)."""
    _check_tensor(u, "u")
    nx, ny, nz = _mhd_shape(u)
    if out_dt is None:
        out_dt = torch.empty(1, dtype=torch.float64, device=u.device)
    if out_ch is None:
        out_ch = torch.empty(1, dtype=torch.float64, device=u.device)
    _check_scalar(out_dt, "out_dt")
    _check_scalar(out_ch, "out_ch")
    ctx = context(u.device.index)
    o = _opts(u.dtype, True, "minmod", "hllc", rho_floor, p_floor)
    ctx.check(ctx.lib.cfl_dt_mhd(ctx.handle, ctypes.byref(o), nx, ny, nz, _ptr(u), float(gamma),
                                 float(dx), float(cfl), _ptr(out_dt), _ptr(out_ch),
                                 _stream(stream)))
    return out_dt, out_ch


# ------------------------------------------------------------ two-level AMR

def amr_patch_table(lo, n, u_in_off, u_out_off, flux_off) -> np.ndarray:
    """Structured array of gd_amr_patch records: lo (P, 3) coarse cells
    (x, y, z), n (P, 3) fine interior extents (nx, ny, nz)."""
    lo = np.asarray(lo).reshape(-1, 3)
    t = np.zeros(len(lo), dtype=AMR_PATCH_DTYPE)
    t["lo"], t["n"] = lo, np.asarray(n).reshape(-1, 3)
    t["u_in_off"], t["u_out_off"], t["flux_off"] = u_in_off, u_out_off, flux_off
    return t


class AmrPlan:
    """A gd_amr: the device tables of a periodic coarse box of nc = (ncx, ncy,
    ncz) cells of width dx_coarse and fine patches refined by 2 (see
    amr_patch_table; fine buffers in the batched layout with ng = 2)."""

    def __init__(self, nc, dx_coarse, table, device=None):
        self.ctx = context(device)
        self.nc = tuple(int(v) for v in nc)
        self.dx_coarse = float(dx_coarse)
        self.table = np.ascontiguousarray(table, dtype=AMR_PATCH_DTYPE)
        n = self.table["n"].astype(np.int64)
        if len(n):
            self.in_end = int((self.table["u_in_off"] + 5 * np.prod(n + 4, axis=1)).max())
            self.out_end = int((self.table["u_out_off"] + 5 * np.prod(n, axis=1)).max())
            self.flux_end = int((self.table["flux_off"] + 10 * (n[:, 2] * n[:, 1] + n[:, 2] * n[:, 0]
                                                                + n[:, 1] * n[:, 0])).max())
        else:
            self.in_end = self.out_end = self.flux_end = 0
        h = ctypes.c_void_p()
        self.ctx.check(self.ctx.lib.gd_amr_create(self.ctx.handle, *self.nc, self.dx_coarse,
                                                  len(self.table), self.table.ctypes.data,
                                                  ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None and self.handle.value:
                self.ctx.lib.gd_amr_destroy(self.handle)
        except Exception:
            pass

    def _check(self, coarse=(), fine_in=None, fine_out=None, fine_flux=None):
        for name, t in coarse:
            _check_tensor(t, name)
            if t.numel() != 5 * self.nc[0] * self.nc[1] * self.nc[2]:
                raise ValueError(f"{name} must hold 5 x {self.nc} values")
        for name, t, need in (("fine_in", fine_in, self.in_end), ("fine_out", fine_out, self.out_end),
                              ("fine_flux", fine_flux, self.flux_end)):
            if t is not None:
                _check_tensor(t, name)
                if t.numel() < need:
                    raise ValueError(f"{name} holds {t.numel()} values, the patches need {need}")

    def fill_ghosts(self, coarse, fine_in, stream=None):
        """Write every ghost cell of the fine patches in fine_in."""
        self._check([("coarse", coarse)], fine_in=fine_in)
        _check_tensor(fine_in, "fine_in", coarse.dtype)
        self.ctx.check(self.ctx.lib.gd_amr_fill_ghosts(
            self.ctx.handle, self.handle, DTYPES[coarse.dtype], _ptr(coarse), _ptr(fine_in),
            _stream(stream)))
        return fine_in

    def reflux(self, coarse_old, coarse_new, fine_out, fine_flux, gamma, dt=None, *, dt_dev=None,
               limiter="minmod", riemann="hllc", rho_floor=RHO_FLOOR, p_floor=P_FLOOR,
               stream=None):
        """Refluxing and averaging down into coarse_new, in place."""
        self._check([("coarse_old", coarse_old), ("coarse_new", coarse_new)], fine_out=fine_out,
                    fine_flux=fine_flux)
        if dt_dev is not None:
            _check_scalar(dt_dev, "dt_dev")
        o = _opts(coarse_old.dtype, True, limiter, riemann, rho_floor, p_floor)
        self.ctx.check(self.ctx.lib.gd_amr_reflux(
            self.ctx.handle, self.handle, ctypes.byref(o), _ptr(coarse_old), _ptr(coarse_new),
            _ptr(fine_out), _ptr(fine_flux), float(gamma), float(dt or 0.0), _ptr(dt_dev),
            _stream(stream)))
        return coarse_new

    def step(self, coarse_in, fine_in, gamma, dt=None, *, coarse_out, fine_out, fine_flux,
             dt_dev=None, limiter="minmod", riemann="hllc", rho_floor=RHO_FLOOR, p_floor=P_FLOOR,
             stream=None):
        """One two-level step: ghost fill (into fine_in), coarse and fine
        steps, refluxing and averaging down into coarse_out."""
        self._check([("coarse_in", coarse_in), ("coarse_out", coarse_out)], fine_in=fine_in,
                    fine_out=fine_out, fine_flux=fine_flux)
        for name, t in (("fine_in", fine_in), ("fine_out", fine_out), ("fine_flux", fine_flux),
                        ("coarse_out", coarse_out)):
            if t.dtype != coarse_in.dtype:
                raise TypeError(f"{name} must have dtype {coarse_in.dtype}")
        if dt_dev is not None:
            _check_scalar(dt_dev, "dt_dev")
        elif dt is None:
            raise ValueError("give dt or dt_dev")
        o = _opts(coarse_in.dtype, True, limiter, riemann, rho_floor, p_floor)
        self.ctx.check(self.ctx.lib.gd_amr_step(
            self.ctx.handle, self.handle, ctypes.byref(o), _ptr(coarse_in), _ptr(coarse_out),
            _ptr(fine_in), _ptr(fine_out), _ptr(fine_flux), float(gamma), float(dt or 0.0),
            _ptr(dt_dev), _stream(stream)))
        return coarse_out, fine_out, fine_flux
