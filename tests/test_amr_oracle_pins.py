"""Pins of the two-level AMR oracle (CPU only).

The seams around the batched step -- ghost fill from the same level or the
coarse level, refluxing at coarse-fine faces and averaging down -- are checked
against what the definitions and the conservation law fix, not against the
oracle's own code:
  * ghost fill: every ghost cell of a hierarchy whose cells hold their own
    global coordinates decodes to the right cell, found by brute force over
    the patch boxes;
  * a uniform state is left unchanged, bit for bit;
  * a face shared by two fine patches carries the same flux in both;
  * the composite state (uncovered coarse cells + fine cells) is conserved to
    rounding, and after averaging down the coarse box carries the same totals;
  * each coarse cell next to a fine patch equals a direct update of that cell
    from its six face fluxes, each computed from a one-cell patch cut out of
    the coarse box or, across a coarse-fine face, the mean of four one-cell
    patches cut out of the ghost-filled fine data;
  * averaging down reproduces a linear field at the coarse cell centres.
"""
import importlib.util
import math
import os

import numpy as np
import pytest

import oracle
from paper_1412_0934_amd import inputs


def _load_amr():
    # the mutation test points the pins at a broken copy of the AMR oracle
    path = os.environ.get("ORACLE_AMR_FILE")
    if not path:
        from oracle import amr
        return amr
    spec = importlib.util.spec_from_file_location("oracle.amr_mutant", path,
                                                  submodule_search_locations=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    spec.loader.exec_module(mod)
    return mod


amr = _load_amr()
G = 1.4


@pytest.fixture(scope="module")
def run():
    h = inputs.amr_hierarchy(gamma=G)
    dt = 0.3 * (h.dx_coarse / 2) / 2.5
    return h, dt, amr.step(h, G, dt)


def _covering_patch(h, c):
    """Brute force: the patch whose coarse box holds coarse cell c, or -1."""
    for p in range(len(h.lo)):
        lo, hi = h.lo[p], h.lo[p] + h.n[p] // 2
        if all(lo[a] <= c[a] < hi[a] for a in range(3)):
            return p
    return -1


def test_hierarchy_has_touching_patches_and_interfaces():
    h = inputs.amr_hierarchy(gamma=G)
    assert len(h.lo) == 8
    touching = 0
    for p in range(len(h.lo)):
        for q in range(p + 1, len(h.lo)):
            a0, a1 = h.lo[p], h.lo[p] + h.n[p] // 2
            b0, b1 = h.lo[q], h.lo[q] + h.n[q] // 2
            gap = [max(b0[a] - a1[a], a0[a] - b1[a]) for a in range(3)]
            if sorted(gap)[-1] == 0 and sorted(gap)[1] < 0:
                touching += 1
    assert touching >= 2


def test_ghost_fill_takes_fine_cells_else_the_prolonged_coarse_parent():
    """Coarse variables linear in x, y, z, one quadratic in x and one uniform:
    a ghost cell over a fine patch takes that fine cell; any other takes its
    parent plus a quarter of the smaller one-sided difference along each axis
    -- for the linear fields the field at its own centre, g/2 - 1/4 in coarse
    units (exact in binary) -- except where the parent sits on the periodic
    seam, whose jump limits the slope to zero."""
    h = inputs.amr_hierarchy(gamma=G)
    nc = h.nc
    X = np.arange(nc, dtype=float)
    h.coarse[0] = X[None, None, :]
    h.coarse[1] = X[None, :, None]
    h.coarse[2] = X[:, None, None]
    h.coarse[3] = (X * X)[None, None, :]
    h.coarse[4] = -1.0
    for p in range(len(h.lo)):
        nx, ny, nz = (int(v) for v in h.n[p])
        blk = h.fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2]
        blk[0] = (2 * h.lo[p][0] + np.arange(nx))[None, None, :]
        blk[1] = (2 * h.lo[p][1] + np.arange(ny))[None, :, None]
        blk[2] = (2 * h.lo[p][2] + np.arange(nz))[:, None, None]
        blk[3] = 1.0
        blk[4] = p
    before = h.fine.u_in.copy()
    buf = amr.fill_ghosts(h, h.coarse)
    m = 2 * nc
    checked = 0
    for p in range(len(h.lo)):
        nx, ny, nz = (int(v) for v in h.n[p])
        off = h.fine.u_in_off[p]
        size = 5 * (nx + 4) * (ny + 4) * (nz + 4)
        v = buf[off:off + size].reshape(5, nz + 4, ny + 4, nx + 4)
        b = before[off:off + size].reshape(v.shape)
        assert np.array_equal(v[:, 2:-2, 2:-2, 2:-2], b[:, 2:-2, 2:-2, 2:-2])
        for kk in range(nz + 4):
            for jj in range(ny + 4):
                for ii in range(nx + 4):
                    if 2 <= ii < nx + 2 and 2 <= jj < ny + 2 and 2 <= kk < nz + 2:
                        continue
                    g = [(2 * h.lo[p][0] + ii - 2) % m, (2 * h.lo[p][1] + jj - 2) % m,
                         (2 * h.lo[p][2] + kk - 2) % m]
                    q = _covering_patch(h, [g[0] // 2, g[1] // 2, g[2] // 2])

                    def lin(gi):
                        c = gi // 2
                        return float(c) if c in (0, nc - 1) else gi / 2 - 0.25

                    def quad(gi):
                        # x^2: one-sided differences 2c - 1 and 2c + 1, minmod the first
                        c = gi // 2
                        if c in (0, nc - 1):
                            return float(c * c)
                        return c * c + (0.25 if gi % 2 else -0.25) * (2 * c - 1)

                    want = ([g[0], g[1], g[2], 1.0, q] if q >= 0 else
                            [lin(g[0]), lin(g[1]), lin(g[2]), quad(g[0]), -1.0])
                    assert list(v[:, kk, jj, ii]) == want, (p, ii, jj, kk)
                    checked += 1
    assert checked > 1000


def test_prolonged_children_average_to_their_parent():
    """The eight children of an uncovered coarse cell, all ghost cells of the
    patch beside it, average back to the coarse value (the slopes enter with
    both signs), and each child differs from it by at most three quarters of
    the largest slope magnitude allowed by its neighbours."""
    h = inputs.amr_hierarchy(gamma=G, seed=17)
    buf = amr.fill_ghosts(h, h.coarse)
    own = amr.owner_map(h)
    nc = h.nc
    checked = 0
    for p in range(len(h.lo)):
        nx, ny, nz = (int(v) for v in h.n[p])
        off = h.fine.u_in_off[p]
        v = buf[off:off + 5 * (nx + 4) * (ny + 4) * (nz + 4)].reshape(5, nz + 4, ny + 4, nx + 4)
        x = int(h.lo[p][0]) - 1                     # the coarse column beside the lower x face
        if own[x % nc, h.lo[p][1], h.lo[p][2]] >= 0:
            continue
        for b in range(ny // 2):
            for a in range(nz // 2):
                y, z = int(h.lo[p][1]) + b, int(h.lo[p][2]) + a
                if own[x % nc, y, z] >= 0:
                    continue
                kids = v[:, 2 + 2 * a:4 + 2 * a, 2 + 2 * b:4 + 2 * b, 0:2]
                uc = h.coarse[:, z, y, x % nc]
                scale = np.abs(h.coarse).reshape(5, -1).max(axis=1)
                assert np.all(np.abs(kids.reshape(5, -1).mean(axis=1) - uc) <= 1e-15 * scale)
                nb = [h.coarse[:, z, y, (x + dx) % nc] for dx in (-1, 1)] + \
                     [h.coarse[:, z, (y + dy) % nc, x % nc] for dy in (-1, 1)] + \
                     [h.coarse[:, (z + dz) % nc, y, x % nc] for dz in (-1, 1)]
                smax = np.max(np.abs(np.array(nb) - uc), axis=0)
                dev = np.abs(kids.reshape(5, -1) - uc[:, None]).max(axis=1)
                assert np.all(dev <= 0.75 * smax + 1e-15 * scale)
                checked += 1
    assert checked > 0


def test_uniform_state_is_unchanged_bit_for_bit():
    h = inputs.amr_hierarchy(gamma=G)
    U = inputs.conserved(np.array(1.3), 0.4, -0.25, 0.15, np.array(0.9), G)
    U = np.array([float(x) for x in U])
    h.coarse[...] = U[:, None, None, None]
    for p in range(len(h.lo)):
        h.fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2] = U[:, None, None, None]
    cn, _, fout, _ = amr.step(h, G, 1e-3)
    assert np.array_equal(cn, h.coarse)
    for p in range(len(h.lo)):
        assert np.array_equal(h.fine.patch_out(fout, p), h.fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2])


def _sheet(h, flux, p, d, side):
    nx, ny, nz = (int(v) for v in h.n[p])
    sx, sy, sz = 5 * nz * ny, 5 * nz * nx, 5 * ny * nx
    starts = [0, sx, 2 * sx, 2 * sx + sy, 2 * sx + 2 * sy, 2 * sx + 2 * sy + sz]
    shape = [(5, nz, ny), (5, nz, nx), (5, ny, nx)][d]
    fl = flux[h.fine.flux_off[p]:h.fine.flux_off[p] + 10 * (nz * ny + nz * nx + ny * nx)]
    return fl[starts[2 * d + side]:starts[2 * d + side] + [sx, sy, sz][d]].reshape(shape)


def test_shared_fine_faces_carry_identical_fluxes(run):
    h, _, (_, _, _, ffl) = run
    shared = 0
    for p in range(len(h.lo)):
        for q in range(len(h.lo)):
            for d in range(3):
                # p's upper d-face against q's lower d-face
                if 2 * (h.lo[p][d] + h.n[p][d] // 2) != 2 * h.lo[q][d]:
                    continue
                t = [a for a in range(3) if a != d]       # sheet axes, slow = t[1]
                lo = [max(2 * h.lo[p][a], 2 * h.lo[q][a]) for a in t]
                hi = [min(2 * h.lo[p][a] + h.n[p][a], 2 * h.lo[q][a] + h.n[q][a]) for a in t]
                if hi[0] <= lo[0] or hi[1] <= lo[1]:
                    continue
                sp, sq = _sheet(h, ffl, p, d, 1), _sheet(h, ffl, q, d, 0)
                for s in range(lo[1], hi[1]):
                    for f in range(lo[0], hi[0]):
                        a = sp[:, s - 2 * h.lo[p][t[1]], f - 2 * h.lo[p][t[0]]]
                        b = sq[:, s - 2 * h.lo[q][t[1]], f - 2 * h.lo[q][t[0]]]
                        assert np.array_equal(a, b), (p, q, d, s, f)
                        shared += 1
    assert shared >= 8


def _totals(h, coarse, interiors):
    own = np.array([[[_covering_patch(h, (x, y, z)) for x in range(h.nc)]
                     for y in range(h.nc)] for z in range(h.nc)])
    unc = own < 0
    dv = h.dx_coarse ** 3
    tot, mag = [], []
    for v in range(5):
        terms = list(coarse[v][unc] * dv)
        for p in range(len(h.lo)):
            terms.extend((interiors(p)[v] * (dv / 8)).ravel())
        tot.append(math.fsum(terms))
        mag.append(math.fsum(abs(t) for t in terms))
    return np.array(tot), np.array(mag)


def test_composite_state_is_conserved(run):
    h, _, (cn, _, fout, _) = run
    t0, mag = _totals(h, h.coarse, lambda p: h.fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2])
    t1, _ = _totals(h, cn, lambda p: h.fine.patch_out(fout, p))
    assert np.all(np.abs(t1 - t0) <= 1e-14 * mag), (t1 - t0) / mag
    whole = np.array([math.fsum((cn[v] * h.dx_coarse ** 3).ravel()) for v in range(5)])
    assert np.all(np.abs(whole - t1) <= 1e-14 * mag)


def _cut(u, c, wrap):
    """5^3 block around c = (x, y, z) of a [5][z][y][x] array."""
    if wrap:
        n = u.shape[1:]
        iz, iy, ix = [np.arange(c[a] - 2, c[a] + 3) % n[2 - a] for a in (2, 1, 0)]
        return u[:, iz][:, :, iy][:, :, :, ix]
    return u[:, c[2] - 2:c[2] + 3, c[1] - 2:c[1] + 3, c[0] - 2:c[0] + 3]


def _face_of_cell(block, d, upper, gamma, dx, dt):
    """Flux through the lower / upper d-face of the one-cell patch `block`."""
    _, fl, _ = oracle.step(block, gamma, dx, dt)
    return fl[10 * d + 5 * upper:10 * d + 5 * upper + 5]


def test_coarse_cells_at_the_interface_match_a_direct_update(run):
    h, dt, (cn, fin, _, _) = run
    nc, dxc = h.nc, h.dx_coarse
    cells = set()
    for z in range(nc):
        for y in range(nc):
            for x in range(nc):
                if _covering_patch(h, (x, y, z)) >= 0:
                    continue
                for d in range(3):
                    for s in (-1, 1):
                        o = [x, y, z]
                        o[d] += s
                        if _covering_patch(h, o) >= 0:
                            cells.add((x, y, z))
    assert len(cells) > 100
    worst = 0.0
    scale = np.abs(h.coarse).reshape(5, -1).max(axis=1)
    for c in sorted(cells):
        div = np.zeros(5)
        for d in range(3):
            for upper in (0, 1):
                o = list(c)
                o[d] += 1 if upper else -1
                q = _covering_patch(h, o)
                if q < 0:
                    F = _face_of_cell(_cut(h.coarse, c, True), d, upper, G, dxc, dt)
                else:
                    # the 2x2 fine cells of q that touch this face
                    nx, ny, nz = (int(v) for v in h.n[q])
                    off = h.fine.u_in_off[q]
                    fq = fin[off:off + 5 * (nx + 4) * (ny + 4) * (nz + 4)].reshape(
                        5, nz + 4, ny + 4, nx + 4)
                    base = [2 * o[a] - 2 * h.lo[q][a] for a in range(3)]
                    base[d] += 0 if upper else 1
                    t = [a for a in range(3) if a != d]
                    Fs = []
                    for i0 in (0, 1):
                        for i1 in (0, 1):
                            f = list(base)
                            f[t[0]] += i0
                            f[t[1]] += i1
                            blk = _cut(fq, [f[0] + 2, f[1] + 2, f[2] + 2], False)
                            Fs.append(_face_of_cell(blk, d, 1 - upper, G, dxc / 2, dt))
                    F = sum(Fs) / 4
                div += F if upper else -F
        want = h.coarse[:, c[2], c[1], c[0]] - dt / dxc * div
        worst = max(worst, float(np.max(np.abs(cn[:, c[2], c[1], c[0]] - want) / scale)))
    assert worst <= 1e-13, worst


def test_average_down_of_a_linear_field():
    h = inputs.amr_hierarchy(gamma=G)
    fout = np.zeros(h.fine.u_out_size)
    for p in range(len(h.lo)):
        nx, ny, nz = (int(v) for v in h.n[p])
        gx = 2 * h.lo[p][0] + np.arange(nx) + 0.5
        gy = 2 * h.lo[p][1] + np.arange(ny) + 0.5
        gz = 2 * h.lo[p][2] + np.arange(nz) + 0.5
        o = h.fine.patch_out(fout, p)
        for v, (a, b, c) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 2, 3), (3, -1, 2)]):
            o[v] = a * gx[None, None, :] + b * gy[None, :, None] + c * gz[:, None, None]
    cn = np.full_like(h.coarse, np.nan)
    amr.average_down(h, fout, cn)
    covered = 0
    for z in range(h.nc):
        for y in range(h.nc):
            for x in range(h.nc):
                if _covering_patch(h, (x, y, z)) < 0:
                    assert np.all(np.isnan(cn[:, z, y, x]))
                    continue
                X, Y, Z = 2 * x + 1, 2 * y + 1, 2 * z + 1
                want = [X, Y, Z, X + 2 * Y + 3 * Z, 3 * X - Y + 2 * Z]
                assert np.allclose(cn[:, z, y, x], want, rtol=0, atol=1e-12), (x, y, z)
                covered += 1
    assert covered == int(sum(np.prod(h.n // 2, axis=1)))
