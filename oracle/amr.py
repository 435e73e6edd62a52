"""Plain CPU oracle of one non-subcycled step of a two-level AMR hierarchy
around the Godunov step: the seams on either side of the batched call.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/`` may import
it. It is written from the definitions, cell by cell and face by face, on top
of the oracle's single-patch step.

The paper's Ramses port hands the GPU patches of inner cells plus boundary
cells interpolated from the neighbouring level (Sec. 3), and Enzo returns the
fluxes a multilevel run needs for flux correction (Sec. 4). One step, with the
same dt on both levels:

1. ghost fill: every ghost cell (two layers) of a fine patch takes the value of
   the fine cell at the same place if another fine patch covers it, else the
   limited linear prolongation of the coarse cell containing it: per conserved
   variable, the coarse value plus a quarter of the minmod slope (undivided,
   from the two periodic neighbours) along each axis, signed by the half of
   the coarse cell the fine cell lies in -- the eight children of a coarse
   cell average back to its value;
2. the coarse box (periodic) and every fine patch take one Godunov step; the
   fine patches return their boundary fluxes;
3. refluxing: a coarse cell outside the fine patches that shares a face with
   one had that face's coarse flux F_c in its update; it is replaced by the
   mean <F_f> of the four fine fluxes through the same face:
   U' += dt/dx (F_c - <F_f>) if the face is the cell's upper face along d,
   U' += dt/dx (<F_f> - F_c) if it is its lower face;
4. averaging down: a coarse cell covered by a fine patch becomes the mean of
   its eight fine children.
The composite state -- uncovered coarse cells and all fine cells -- is then
conserved to rounding.
"""
from __future__ import annotations

import numpy as np

from . import step as _step


def owner_map(h):
    """[x][y][z] array: the fine patch covering each coarse cell, or -1."""
    own = -np.ones((h.nc,) * 3, dtype=np.int64)
    for p in range(len(h.lo)):
        x, y, z = h.lo[p]
        sx, sy, sz = h.n[p] // 2
        own[x:x + sx, y:y + sy, z:z + sz] = p
    return own


def minmod(a, b):
    """0 where a and b differ in sign or one is zero, else the one of smaller
    magnitude."""
    return np.where(a * b <= 0.0, 0.0, np.where(np.abs(a) <= np.abs(b), a, b))


def prolong(coarse, gx, gy, gz):
    """Value at fine cell (gx, gy, gz) of the limited linear prolongation of
    its coarse parent (periodic box): U_c + ((sx Sx + sy Sy) + sz Sz) / 4 with
    S_d the minmod slope of U along d and s_d = +1 in the parent's upper half
    along d, -1 in its lower half."""
    nc = coarse.shape[1]
    cx, cy, cz = gx // 2, gy // 2, gz // 2
    uc = coarse[:, cz, cy, cx]
    slope = []
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        lo = coarse[:, (cz - e[2]) % nc, (cy - e[1]) % nc, (cx - e[0]) % nc]
        hi = coarse[:, (cz + e[2]) % nc, (cy + e[1]) % nc, (cx + e[0]) % nc]
        slope.append(minmod(uc - lo, hi - uc))
    sx, sy, sz = (slope[d] if g % 2 else -slope[d] for d, g in enumerate((gx, gy, gz)))
    return uc + 0.25 * ((sx + sy) + sz)


def fill_ghosts(h, coarse):
    """A copy of the fine input buffer with every ghost cell filled."""
    own = owner_map(h)
    buf = h.fine.u_in.copy()
    m = 2 * h.nc
    for p in range(len(h.lo)):
        nx, ny, nz = (int(v) for v in h.n[p])
        view = buf[h.fine.u_in_off[p]:h.fine.u_in_off[p] + 5 * (nx + 4) * (ny + 4) * (nz + 4)]
        view = view.reshape(5, nz + 4, ny + 4, nx + 4)
        for kk in range(nz + 4):
            for jj in range(ny + 4):
                for ii in range(nx + 4):
                    if 2 <= ii < nx + 2 and 2 <= jj < ny + 2 and 2 <= kk < nz + 2:
                        continue
                    # global fine cell, periodic
                    gx = (2 * h.lo[p][0] + ii - 2) % m
                    gy = (2 * h.lo[p][1] + jj - 2) % m
                    gz = (2 * h.lo[p][2] + kk - 2) % m
                    q = own[gx // 2, gy // 2, gz // 2]
                    if q >= 0:
                        src = h.fine.patch_in(q)
                        view[:, kk, jj, ii] = src[:, gz - 2 * h.lo[q][2] + 2,
                                                  gy - 2 * h.lo[q][1] + 2,
                                                  gx - 2 * h.lo[q][0] + 2]
                    else:
                        view[:, kk, jj, ii] = prolong(coarse, gx, gy, gz)
    return buf


def coarse_face_flux(coarse, d, right, gamma, dx, dt, limiter, riemann):
    """Flux through the coarse face along d whose right cell is `right`
    (x, y, z), as the periodic coarse step computes it: the lower d-face flux
    of a one-cell patch cut from the box with its two ghost layers."""
    nc = coarse.shape[1]
    x, y, z = right
    idx = [np.arange(c - 2, c + 3) % nc for c in (z, y, x)]
    cell = coarse[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]
    _, bflux, _ = _step(cell, gamma, dx, dt, limiter=limiter, riemann=riemann)
    # sheets x-, x+, y-, y+, z-, z+ of a 1x1x1 patch: 5 values each
    return bflux[10 * d:10 * d + 5].copy()


def interface_faces(h):
    """Every coarse face between a fine patch and an uncovered coarse cell:
    (patch, axis d, side (0 lower, 1 upper), footprint cell (x, y, z),
    outside cell (x, y, z))."""
    own = owner_map(h)
    nc = h.nc
    faces = []
    for p in range(len(h.lo)):
        lo = h.lo[p]
        size = h.n[p] // 2
        for d in range(3):
            t1, t2 = (d + 1) % 3, (d + 2) % 3
            for side in (0, 1):
                for b in range(size[t2]):
                    for a in range(size[t1]):
                        c = np.array(lo)
                        c[t1] += a
                        c[t2] += b
                        c[d] = lo[d] + (size[d] - 1 if side else 0)
                        o = c.copy()
                        o[d] = (c[d] + (1 if side else -1)) % nc
                        if own[o[0], o[1], o[2]] < 0:
                            faces.append((p, d, side, tuple(c), tuple(o)))
    return faces


def fine_face_mean(h, fine_flux, p, d, side, cell):
    """Mean of the four fine fluxes through the coarse face of footprint cell
    `cell` on side `side` of axis d of patch p, from its boundary sheets."""
    nx, ny, nz = (int(v) for v in h.n[p])
    flat = h.fine.patch_flux(fine_flux, p)
    sx, sy, sz = 5 * nz * ny, 5 * nz * nx, 5 * ny * nx
    base = [0, sx, 2 * sx, 2 * sx + sy, 2 * sx + 2 * sy, 2 * sx + 2 * sy + sz][2 * d + side]
    shape = [(5, nz, ny), (5, nz, nx), (5, ny, nx)][d]
    size = [sx, sy, sz][d]
    sheet = flat[base:base + size].reshape(shape)
    loc = [2 * (cell[a] - h.lo[p][a]) for a in range(3)]
    # sheet axes: x sheets (z, y), y sheets (z, x), z sheets (y, x)
    if d == 0:
        blk = sheet[:, loc[2]:loc[2] + 2, loc[1]:loc[1] + 2]
    elif d == 1:
        blk = sheet[:, loc[2]:loc[2] + 2, loc[0]:loc[0] + 2]
    else:
        blk = sheet[:, loc[1]:loc[1] + 2, loc[0]:loc[0] + 2]
    # pairwise, so that four equal fluxes average to exactly that flux
    return ((blk[:, 0, 0] + blk[:, 0, 1]) + (blk[:, 1, 0] + blk[:, 1, 1])) * 0.25


def step(h, gamma, dt, *, limiter="minmod", riemann="hllc", reflux=True):
    """One two-level step. Returns (coarse', fine input with ghosts,
    fine output flat buffer, fine boundary fluxes flat buffer)."""
    dxc = h.dx_coarse
    fine_in = fill_ghosts(h, h.coarse)
    coarse_new, _, _ = _step(h.coarse, gamma, dxc, dt, periodic=True, limiter=limiter,
                             riemann=riemann)
    fine_out = np.empty(h.fine.u_out_size)
    fine_flux = np.empty(h.fine.flux_size)
    for p in range(len(h.lo)):
        nx, ny, nz = (int(v) for v in h.n[p])
        uin = fine_in[h.fine.u_in_off[p]:h.fine.u_in_off[p] + 5 * (nx + 4) * (ny + 4) * (nz + 4)]
        out, fl, _ = _step(uin.reshape(5, nz + 4, ny + 4, nx + 4), gamma, dxc / 2, dt,
                           limiter=limiter, riemann=riemann)
        h.fine.patch_out(fine_out, p)[...] = out
        n_fl = 10 * (nz * ny + nz * nx + ny * nx)
        fine_flux[h.fine.flux_off[p]:h.fine.flux_off[p] + n_fl] = fl
    if reflux:
        apply_reflux(h, h.coarse, coarse_new, fine_flux, gamma, dt, limiter=limiter,
                     riemann=riemann)
    average_down(h, fine_out, coarse_new)
    return coarse_new, fine_in, fine_out, fine_flux


def apply_reflux(h, coarse_old, coarse_new, fine_flux, gamma, dt, *, limiter="minmod",
                 riemann="hllc"):
    """Step 3 in place on coarse_new: at every coarse-fine interface face, swap
    the coarse flux (recomputed from coarse_old) for the mean fine flux."""
    dxc = h.dx_coarse
    c = dt / dxc
    for p, d, side, cell, out_cell in interface_faces(h):
        right = out_cell if side else cell
        Fc = coarse_face_flux(coarse_old, d, right, gamma, dxc, dt, limiter, riemann)
        Ff = fine_face_mean(h, fine_flux, p, d, side, cell)
        corr = c * (Ff - Fc) if side else c * (Fc - Ff)
        x, y, z = out_cell
        coarse_new[:, z, y, x] += corr


def average_down(h, fine_out, coarse_new):
    """Step 4 in place: each covered coarse cell becomes the mean of its eight
    children, summed as a fixed pairwise tree (x pairs, then y, then z)."""
    for p in range(len(h.lo)):
        fo = h.fine.patch_out(fine_out, p)
        sx, sy, sz = (int(v) for v in h.n[p] // 2)
        for k in range(sz):
            for j in range(sy):
                for i in range(sx):
                    ch = fo[:, 2 * k:2 * k + 2, 2 * j:2 * j + 2, 2 * i:2 * i + 2]
                    zy = [[ch[:, a, b, 0] + ch[:, a, b, 1] for b in (0, 1)] for a in (0, 1)]
                    z = [zy[a][0] + zy[a][1] for a in (0, 1)]
                    coarse_new[:, h.lo[p][2] + k, h.lo[p][1] + j, h.lo[p][0] + i] = \
                        (z[0] + z[1]) * 0.125


def composite_sums(h, coarse, fine_interiors):
    """Per variable: sum over uncovered coarse cells of U dx_c^3 plus sum over
    fine cells of U dx_f^3, with exact (fsum) accumulation.
    fine_interiors(p) returns patch p's interior (5, nz, ny, nx)."""
    import math
    own = owner_map(h)
    uncovered = (own < 0).transpose(2, 1, 0)   # to [z][y][x]
    dxc3 = h.dx_coarse ** 3
    out = []
    for v in range(5):
        terms = list((coarse[v][uncovered] * dxc3).ravel())
        for p in range(len(h.lo)):
            terms.extend((fine_interiors(p)[v] * (dxc3 / 8.0)).ravel())
        out.append(math.fsum(terms))
    return np.array(out)
