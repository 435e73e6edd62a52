"""Seeded synthetic inputs for the Godunov step.

This module is the one piece that both the GPU path and the CPU oracle
consume: it turns prescribed physical fields (density, velocity, pressure)
into conserved states and lays them out. It contains none of the scheme's own
arithmetic (no reconstruction, no fluxes, no update, no time step).

The paper's workloads are cosmological AMR runs (Sec. 3, Table 1; Sec. 4) whose
initial conditions are not available; these generators stand in for them:

* ``sod_patch``       one 32^3 ghost-zoned patch with a planar density and
                      pressure jump plus 1% density noise (the shock-tube
                      problem inside a single patch);
* ``turbulent_box``   a periodic box with log-normal density (sigma_ln = 1)
                      built from a Gaussian random field with a k^-11/3 power
                      spectrum and Gaussian random velocities at rms Mach 2,
                      mimicking the cosmic-web density PDF;
* ``amr_batch``       thousands of ghost-zoned patches of uneven size
                      (8^3..32^3) holding a smooth sine background cut by a
                      planar Mach-3 shock of random orientation, mimicking
                      patches at refinement fronts;
* ``smooth_box``      a periodic box of a few low Fourier modes at 5%
                      amplitude, for gradient checks.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import os

import numpy as np
from scipy import fft as _fft

GAMMA = 5.0 / 3.0
_WORKERS = min(16, os.cpu_count() or 1)


def conserved(rho, vx, vy, vz, p, gamma=GAMMA, out=None):
    """Stack (rho, rho v, E) with E = p/(gamma-1) + rho |v|^2 / 2 (into `out`
    of shape (5, ...) when given)."""
    rho, vx, vy, vz, p = (np.asarray(a, dtype=np.float64) for a in (rho, vx, vy, vz, p))
    shape = np.broadcast_shapes(rho.shape, vx.shape, vy.shape, vz.shape, p.shape)
    if out is None:
        out = np.empty((5,) + shape)
    out[0] = rho
    out[1] = rho * vx
    out[2] = rho * vy
    out[3] = rho * vz
    out[4] = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return out


def outflow_fill(interior, ng=2):
    """Ghost-zoned copy of a (5, nz, ny, nx) state with zero-gradient ghosts
    (every ghost, edges and corners included, copies the nearest interior cell)."""
    return np.pad(interior, ((0, 0), (ng, ng), (ng, ng), (ng, ng)), mode="edge")


def sod_patch(n=32, ng=2, gamma=GAMMA, noise=0.01, seed=0, axis=0):
    """Shock-tube patch: (rho, p) = (1, 1) for x < 1/2 and (0.125, 0.1) beyond,
    v = 0, interior density times (1 + noise U(-1, 1)); outflow ghosts.
    Returns (u_ghosted, dx) with dx = 1/n."""
    x = (np.arange(n) + 0.5) / n
    left = x < 0.5
    shape = [1, 1, 1]
    shape[2 - axis] = n
    left = left.reshape(shape)
    rho = np.where(left, 1.0, 0.125) * np.ones((n, n, n))
    p = np.where(left, 1.0, 0.1) * np.ones((n, n, n))
    if noise:
        rng = np.random.default_rng(seed)
        rho = rho * (1.0 + noise * rng.uniform(-1.0, 1.0, size=(n, n, n)))
    zero = np.zeros((n, n, n))
    return outflow_fill(conserved(rho, zero, zero, zero, p, gamma), ng), 1.0 / n


@functools.lru_cache(maxsize=4)
def _spectral_filter(n, spectral_index):
    k1 = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    kk = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kz[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (spectral_index / 2.0)
    return amp


def gaussian_random_field(n, seed, spectral_index=-11.0 / 3.0):
    """Zero-mean, unit-variance periodic field whose power spectrum is
    P(k) ~ k^spectral_index: white noise filtered by k^(spectral_index/2)."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    fk = _fft.rfftn(white, workers=_WORKERS)
    fk *= _spectral_filter(n, spectral_index)
    f = _fft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2), workers=_WORKERS)
    f -= f.mean()
    f /= f.std()
    return f


def turbulent_box(n=256, gamma=GAMMA, mach=2.0, sigma_ln=1.0, seeds=(1, 2, 3, 4)):
    """Periodic (5, n, n, n) state: rho = exp(sigma s - sigma^2/2) with s a
    k^-11/3 Gaussian random field; velocities independent fields of the same
    spectrum scaled to rms |v| = mach c_s; p = 0.6 rho / gamma, so c_s^2 = 0.6."""
    s = gaussian_random_field(n, seeds[0])
    rho = np.exp(sigma_ln * s - 0.5 * sigma_ln ** 2)
    vel = [gaussian_random_field(n, sd) for sd in seeds[1:4]]
    vel = [v - v.mean() for v in vel]
    rms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)))
    scale = mach * math.sqrt(0.6) / rms
    p = 0.6 * rho / gamma
    return conserved(rho, vel[0] * scale, vel[1] * scale, vel[2] * scale, p, gamma)


def _random_unit(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def _random_wavevector(rng, kmax, generic=False):
    """Integer wavevector in [-kmax, kmax]^3, not zero; with generic=True no
    component is zero (the field then varies along every axis)."""
    while True:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.all(k != 0) if generic else np.any(k != 0):
            return k.astype(np.float64)


def shocked_patch(rng, nx, ny, nz, ng=2, dx=1.0 / 256, gamma=GAMMA, mach=3.0, out=None,
                  generic=False):
    """One ghost-zoned patch (5, nz+2ng, ny+2ng, nx+2ng): smooth sine background
    (rho and p at 1 +- 0.2, |v| <= 0.1) evaluated at cell centres from a random
    origin, cut by a planar shock of random normal through a random interior
    point. The post-shock side carries the Rankine-Hugoniot state of a Mach
    `mach` shock relative to the local background."""
    origin = rng.uniform(0.0, 1.0, size=3)
    kr, kp, kv = (_random_wavevector(rng, 2, generic) for _ in range(3))
    phr, php, phv = rng.uniform(0.0, 2 * math.pi, size=3)
    ev = _random_unit(rng)
    normal = _random_unit(rng)
    through = origin + dx * rng.uniform(0.0, 1.0, size=3) * np.array([nx, ny, nz])

    X = (origin[0] + (np.arange(-ng, nx + ng) + 0.5) * dx)[None, None, :]
    Y = (origin[1] + (np.arange(-ng, ny + ng) + 0.5) * dx)[None, :, None]
    Z = (origin[2] + (np.arange(-ng, nz + ng) + 0.5) * dx)[:, None, None]

    def wave(k, ph):
        return np.sin(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)

    rho1 = 1.0 + 0.2 * wave(kr, phr)
    p1 = 1.0 + 0.2 * wave(kp, php)
    vmag = 0.1 * wave(kv, phv)
    v1 = [vmag * ev[d] for d in range(3)]

    c1 = np.sqrt(gamma * p1 / rho1)
    m2 = mach * mach
    ratio = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    pjump = (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    du = (1.0 - 1.0 / ratio) * mach * c1
    behind = (normal[0] * (X - through[0]) + normal[1] * (Y - through[1])
              + normal[2] * (Z - through[2])) <= 0.0
    rho = np.where(behind, rho1 * ratio, rho1)
    p = np.where(behind, p1 * pjump, p1)
    v = [np.where(behind, v1[d] + du * normal[d], v1[d]) for d in range(3)]
    return conserved(rho, v[0], v[1], v[2], p, gamma, out=out)


@dataclass
class Batch:
    """A packed batch of ghost-zoned patches.

    dims[p] = (nx, ny, nz); all arrays of patch p live in flat buffers at the
    element offsets u_in_off[p] (shape [5][nz+2ng][ny+2ng][nx+2ng]),
    u_out_off[p] ([5][nz][ny][nx]) and flux_off[p] (six boundary sheets,
    10 (nz ny + nz nx + ny nx) values)."""
    dims: np.ndarray
    ng: int
    dx: np.ndarray
    u_in: np.ndarray
    u_in_off: np.ndarray
    u_out_off: np.ndarray
    flux_off: np.ndarray
    u_out_size: int
    flux_size: int

    @property
    def npatch(self):
        return len(self.dims)

    @property
    def interior_cells(self):
        return int(np.prod(self.dims, axis=1).sum())

    def patch_in(self, p):
        nx, ny, nz = (int(v) for v in self.dims[p])
        g = self.ng
        n = 5 * (nz + 2 * g) * (ny + 2 * g) * (nx + 2 * g)
        return self.u_in[self.u_in_off[p]:self.u_in_off[p] + n].reshape(
            5, nz + 2 * g, ny + 2 * g, nx + 2 * g)

    def patch_out(self, flat_out, p):
        nx, ny, nz = (int(v) for v in self.dims[p])
        return flat_out[self.u_out_off[p]:self.u_out_off[p] + 5 * nx * ny * nz].reshape(5, nz, ny, nx)

    def patch_flux(self, flat_flux, p):
        nx, ny, nz = (int(v) for v in self.dims[p])
        return flat_flux[self.flux_off[p]:self.flux_off[p] + 10 * (nz * ny + nz * nx + ny * nx)]


def batch_layout(dims, ng, dx, order_seed=None):
    """An empty Batch for patches of the given interior extents (nx, ny, nz).
    With order_seed, patches are laid out in memory in a seeded random order
    (the descriptor list keeps the given order)."""
    dims = np.asarray(dims, dtype=np.int64).reshape(-1, 3)
    npatch = len(dims)
    place = np.arange(npatch)
    if order_seed is not None:
        place = np.random.default_rng(order_seed).permutation(npatch)
    in_sizes = 5 * np.prod(dims + 2 * ng, axis=1)
    out_sizes = 5 * np.prod(dims, axis=1)
    fl_sizes = 10 * (dims[:, 2] * dims[:, 1] + dims[:, 2] * dims[:, 0] + dims[:, 1] * dims[:, 0])

    def offsets(sizes):
        off = np.zeros(npatch, dtype=np.int64)
        if npatch == 0:
            return off, 0
        ordered = sizes[place]
        off[place] = np.concatenate([[0], np.cumsum(ordered)[:-1]])
        return off, int(sizes.sum())

    u_in_off, n_in = offsets(in_sizes)
    u_out_off, n_out = offsets(out_sizes)
    flux_off, n_fl = offsets(fl_sizes)
    dxs = np.full(npatch, float(dx)) if np.isscalar(dx) else np.asarray(dx, dtype=np.float64)
    return Batch(dims, ng, dxs, np.empty(n_in, dtype=np.float64), u_in_off, u_out_off, flux_off,
                 n_out, n_fl)


def pack_batch(states, ng, dx, order_seed=None):
    """Pack a list of ghost-zoned (5, gz, gy, gx) states into one Batch."""
    dims = [[s.shape[3] - 2 * ng, s.shape[2] - 2 * ng, s.shape[1] - 2 * ng] for s in states]
    batch = batch_layout(dims, ng, dx, order_seed)
    for p, s in enumerate(states):
        batch.patch_in(p)[...] = s
    return batch


def amr_batch(npatch=4096, seed=5, ng=2, dx=1.0 / 256, gamma=GAMMA,
              sizes=(8, 16, 24, 32), probs=(0.5, 0.3, 0.15, 0.05), mach=3.0):
    """Batch of cubic patches with edge lengths drawn from `sizes` with
    probabilities `probs`; each holds a shocked_patch field; packed in a
    seeded random memory order."""
    rng = np.random.default_rng(seed)
    edge = rng.choice(np.asarray(sizes), size=npatch, p=np.asarray(probs))
    batch = batch_layout(np.repeat(edge[:, None], 3, axis=1), ng, dx, order_seed=seed + 1000)
    for p, n in enumerate(edge):
        shocked_patch(rng, int(n), int(n), int(n), ng, dx, gamma, mach, out=batch.patch_in(p))
    return batch


def random_patch(nx, ny, nz, ng=2, seed=0, dx=None, gamma=GAMMA, mach=3.0, generic=False):
    """Test patch: the shocked_patch field of the given extents. generic=True
    draws background waves that vary along every axis, so that no primitive
    is constant along an axis (whose slopes would be pure rounding noise)."""
    rng = np.random.default_rng(seed)
    return shocked_patch(rng, nx, ny, nz, ng, 1.0 / 64 if dx is None else dx, gamma, mach,
                         generic=generic)


def smooth_direction(shape, seed, nmodes=4, kmax=3):
    """A smooth random perturbation field (each of the 5 variables a sum of
    low Fourier modes with N(0,1) amplitudes), for directional derivatives."""
    rng = np.random.default_rng(seed)
    n = shape[-1]
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    out = np.zeros(shape)
    for v in range(shape[0]):
        for _ in range(nmodes):
            k = _random_wavevector(rng, kmax)
            out[v] += rng.standard_normal() * np.sin(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z)
                                                     + rng.uniform(0, 2 * math.pi))
    return out


def _mode_sum(n, rng, nmodes=8, kmax=4):
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    f = np.zeros((n, n, n))
    for _ in range(nmodes):
        k = _random_wavevector(rng, kmax)
        ph = rng.uniform(0.0, 2 * math.pi)
        f += np.sin(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
    return f / np.max(np.abs(f))


def smooth_box(n=128, gamma=GAMMA, amplitude=0.05, seeds=(13, 14, 15, 16, 17, 18)):
    """Periodic smooth state and a density target: rho, p = 1 + a f_m with f_m
    a sum of 8 random Fourier modes (integer wavevectors in [-4, 4]^3)
    normalised to max |f_m| = 1; velocities a c_s f_m. Returns (U0, rho_target)."""
    rho = 1.0 + amplitude * _mode_sum(n, np.random.default_rng(seeds[0]))
    p = 1.0 + amplitude * _mode_sum(n, np.random.default_rng(seeds[1]))
    cs = math.sqrt(gamma)
    vel = [amplitude * cs * _mode_sum(n, np.random.default_rng(s)) for s in seeds[2:5]]
    target = 1.0 + amplitude * _mode_sum(n, np.random.default_rng(seeds[5]))
    return conserved(rho, vel[0], vel[1], vel[2], p, gamma), target


# ------------------------------------------------------------ ideal MHD

def mhd_conserved(rho, vx, vy, vz, p, bx, by, bz, psi=None, gamma=GAMMA):
    """(9, ...) conserved MHD state (rho, rho v, E, B, psi) from primitives,
    E = p/(gamma-1) + rho |v|^2/2 + |B|^2/2 (units with mu0 = 1)."""
    rho, vx, vy, vz, p, bx, by, bz = np.broadcast_arrays(rho, vx, vy, vz, p, bx, by, bz)
    out = np.empty((9,) + rho.shape)
    out[0] = rho
    out[1] = rho * vx
    out[2] = rho * vy
    out[3] = rho * vz
    out[4] = (p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
              + 0.5 * (bx * bx + by * by + bz * bz))
    out[5], out[6], out[7] = bx, by, bz
    out[8] = 0.0 if psi is None else psi
    return out


def alfven_wave(n, amplitude=0.1, gamma=GAMMA, axis=0):
    """Circularly polarised Alfven wave along `axis` on a periodic n-cell line
    (the other extents 1): rho = 1, p = 0.1, B_par = 1, B_perp of constant
    magnitude `amplitude` rotating with phase 2 pi x, v_perp = -B_perp / sqrt(rho)
    (a wave moving in +x at v_A = 1; an exact nonlinear solution, period 1)."""
    x = (np.arange(n) + 0.5) / n
    b1, b2 = amplitude * np.sin(2 * np.pi * x), amplitude * np.cos(2 * np.pi * x)
    shape = [1, 1, 1]
    shape[2 - axis] = n
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    vel, B = [None] * 3, [None] * 3
    vel[axis], B[axis] = np.zeros(n), np.ones(n)
    vel[t1], vel[t2], B[t1], B[t2] = -b1, -b2, b1, b2
    one = np.ones(n)
    U = mhd_conserved(one, vel[0], vel[1], vel[2], 0.1 * one, B[0], B[1], B[2], gamma=gamma)
    return U.reshape((9,) + tuple(shape))


def mhd_turbulent_box(n=128, gamma=GAMMA, mach=1.0, beta=100.0, sigma_ln=1.0,
                      seeds=(1, 2, 3, 4, 5, 6, 7)):
    """Periodic (9, n, n, n) MHD state: density and velocities as in
    turbulent_box at rms Mach `mach`; B from three independent k^-11/3
    Gaussian random fields (not projected, so div B is not zero), scaled so
    that the mean plasma beta 2<p>/<|B|^2> equals `beta`; psi = 0."""
    s = gaussian_random_field(n, seeds[0])
    rho = np.exp(sigma_ln * s - 0.5 * sigma_ln ** 2)
    vel = [gaussian_random_field(n, sd) for sd in seeds[1:4]]
    vel = [v - v.mean() for v in vel]
    rms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)))
    vscale = mach * math.sqrt(0.6) / rms
    p = 0.6 * rho / gamma
    B = [gaussian_random_field(n, sd) for sd in seeds[4:7]]
    b2 = float(np.mean(B[0] ** 2 + B[1] ** 2 + B[2] ** 2))
    bscale = math.sqrt(2.0 * float(np.mean(p)) / beta / b2)
    return mhd_conserved(rho, vel[0] * vscale, vel[1] * vscale, vel[2] * vscale, p,
                         B[0] * bscale, B[1] * bscale, B[2] * bscale, gamma=gamma)


def mhd_random_box(nx, ny, nz, seed=0, gamma=GAMMA, generic=True):
    """Small periodic (9, nz, ny, nx) MHD test state: a few random Fourier
    modes in every primitive (density and pressure kept positive), magnetic
    field of order one and psi of order 0.1, for parity and invariance tests."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny,
                          (np.arange(nx) + 0.5) / nx, indexing="ij")

    def field(amp, base=0.0):
        f = np.full(x.shape, base)
        for _ in range(3):
            k = _random_wavevector(rng, 2, generic=generic)
            ph = rng.uniform(0, 2 * np.pi)
            f += amp * rng.uniform(0.3, 1.0) * np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        return f

    rho = field(0.15, 1.0)
    p = field(0.15, 1.0)
    v = [field(0.3) for _ in range(3)]
    B = [field(0.4, rng.uniform(-0.5, 0.5)) for _ in range(3)]
    psi = field(0.1)
    return mhd_conserved(rho, v[0], v[1], v[2], p, B[0], B[1], B[2], psi=psi, gamma=gamma)


# ------------------------------------------------------------ two-level AMR

@dataclass
class Hierarchy:
    """A periodic coarse box of nc^3 cells and fine patches refined by 2.
    Fine patch p covers the coarse cells [lo[p], lo[p] + n[p]/2); n[p] are its
    interior extents in fine cells (x, y, z), even. The fine patches live in a
    Batch (two ghost layers) whose ghost cells are left NaN: filling them is
    part of the step."""
    nc: int
    coarse: np.ndarray          # (5, nc, nc, nc)
    lo: np.ndarray              # (P, 3) int, (x, y, z) coarse indices
    n: np.ndarray               # (P, 3) int, (nx, ny, nz) fine cells
    fine: Batch

    @property
    def dx_coarse(self):
        return 1.0 / self.nc


def _smooth_state(rng, gamma):
    """A smooth periodic analytic state on the unit box (rho, p = 1 +- 0.2,
    |v| <= 0.3), returned as a function of cell-centre coordinates."""
    ks = [rng.integers(-2, 3, size=3) for _ in range(5)]
    for k in ks:
        if not np.any(k):
            k[0] = 1
    ph = rng.uniform(0, 2 * math.pi, size=5)
    amp = [0.2, 0.3, 0.3, 0.3, 0.2]

    def at(X, Y, Z):
        f = [amp[i] * np.sin(2 * math.pi * (ks[i][0] * X + ks[i][1] * Y + ks[i][2] * Z) + ph[i])
             for i in range(5)]
        return conserved(1.0 + f[0], f[1], f[2], f[3], 1.0 + f[4], gamma)

    return at


def amr_hierarchy(nc=32, nfine=8, seed=11, gamma=GAMMA, max_size=5, touch=0.5, boxes=None):
    """Seeded two-level hierarchy: the same smooth analytic state sampled at
    the coarse cell centres and at the fine cell centres of each patch.
    Patches are random boxes of 2..max_size coarse cells per axis, disjoint,
    inside [2, nc - 2) (no periodic crossing); with probability `touch` a new
    patch is placed against an existing one, so fine-fine faces occur.
    boxes, a list of (lo, size) in coarse cells, replaces the random ones."""
    rng = np.random.default_rng(seed)
    at = _smooth_state(rng, gamma)
    owner = -np.ones((nc, nc, nc), dtype=np.int64)          # [x][y][z]
    los, sizes = [], []
    tries = 0
    if boxes is not None:
        los = [np.asarray(b[0], dtype=np.int64) for b in boxes]
        sizes = [np.asarray(b[1], dtype=np.int64) for b in boxes]
        nfine = 0
    while len(los) < nfine and tries < 5000:
        tries += 1
        size = rng.integers(2, max_size + 1, size=3)
        if los and rng.uniform() < touch:
            q = rng.integers(len(los))
            axis = rng.integers(3)
            lo = los[q].copy()
            lo[axis] = los[q][axis] + sizes[q][axis] if rng.uniform() < 0.5 else los[q][axis] - size[axis]
            for a in range(3):
                if a != axis:
                    lo[a] = los[q][a] + rng.integers(-1, 2)
        else:
            lo = rng.integers(2, nc - 2 - size + 1, size=3) if np.all(nc - 2 - size + 1 > 2) else None
            if lo is None:
                continue
        if np.any(lo < 2) or np.any(lo + size > nc - 2):
            continue
        box = owner[lo[0]:lo[0] + size[0], lo[1]:lo[1] + size[1], lo[2]:lo[2] + size[2]]
        if np.any(box >= 0):
            continue
        box[...] = len(los)
        los.append(np.asarray(lo))
        sizes.append(np.asarray(size))
    lo = np.array(los, dtype=np.int64).reshape(-1, 3)
    n = 2 * np.array(sizes, dtype=np.int64).reshape(-1, 3)
    xc = (np.arange(nc) + 0.5) / nc
    coarse = at(xc[None, None, :], xc[None, :, None], xc[:, None, None])
    fine = batch_layout(n, 2, 0.5 / nc)
    fine.u_in[:] = np.nan
    for p in range(len(lo)):
        nx, ny, nz = (int(v) for v in n[p])
        X = (2 * lo[p][0] + np.arange(nx) + 0.5) / (2 * nc)
        Y = (2 * lo[p][1] + np.arange(ny) + 0.5) / (2 * nc)
        Z = (2 * lo[p][2] + np.arange(nz) + 0.5) / (2 * nc)
        fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2] = at(X[None, None, :], Y[None, :, None],
                                                   Z[:, None, None])
    return Hierarchy(nc, coarse, lo, n, fine)
