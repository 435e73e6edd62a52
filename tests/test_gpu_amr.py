"""Two-level AMR seams on the GPU through the C ABI against the AMR oracle:
ghost fill bit for bit, the whole two-level step (ghost fill, coarse step,
batched fine step, refluxing, averaging down) to 1e-12 in FP64 and 1e-5 in
FP32 for every limiter / Riemann pair, the reflux launch alone, composite
conservation, a uniform state, device dt, hierarchies with patches at the
periodic boundary or spanning a whole axis, an empty hierarchy, and a 64^3
box with 48 patches; and the 128^3 box with 1024 patches the benchmark times,
checked everywhere by the ghost fill and by conservation and on samples
otherwise."""
import math

import numpy as np
import pytest

from oracle import amr
from helpers import bflux_err, parity_err, say
from paper_1412_0934_amd import inputs

pytestmark = pytest.mark.gpu
G = 1.4


@pytest.fixture(scope="module")
def gd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_0934_amd import godunov
    return godunov


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return t if dtype is None else t.to(dtype)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def plan_for(gd, h):
    f = h.fine
    t = gd.amr_patch_table(h.lo, h.n, f.u_in_off, f.u_out_off, f.flux_off)
    return gd.AmrPlan((h.nc,) * 3, h.dx_coarse, t)


def run_gpu(gd, h, dt, dtype=None, **kw):
    """One gd_amr_step; returns (coarse', filled fine input, fine out, fine flux)."""
    import torch
    plan = plan_for(gd, h)
    ci = dev(h.coarse, dtype)
    fi = dev(np.nan_to_num(h.fine.u_in, nan=-7.0), dtype)
    co = torch.empty_like(ci)
    fo = torch.full((max(h.fine.u_out_size, 1),), float("nan"), dtype=ci.dtype, device="cuda")
    ff = torch.full((max(h.fine.flux_size, 1),), float("nan"), dtype=ci.dtype, device="cuda")
    plan.step(ci, fi, G, dt, coarse_out=co, fine_out=fo, fine_flux=ff, **kw)
    return host(co), host(fi), host(fo)[:h.fine.u_out_size], host(ff)[:h.fine.flux_size]


def stable_dt(h, cfl=0.3):
    """CFL step of the fine level, from the coarse state (both sample one field)."""
    import oracle
    return oracle.cfl_dt(h.coarse, G, h.dx_coarse / 2, cfl, periodic=True)


def test_ghost_fill_is_bit_exact(gd):
    h = inputs.amr_hierarchy(gamma=G)
    say("amr ghost fill", len(h.lo), "patches")
    want = amr.fill_ghosts(h, h.coarse)
    plan = plan_for(gd, h)
    fi = dev(np.nan_to_num(h.fine.u_in, nan=-7.0))
    plan.fill_ghosts(dev(h.coarse), fi)
    assert np.array_equal(host(fi), want)


@pytest.mark.parametrize("lim,rs", [("minmod", "hllc"), ("mc", "hll"), ("none", "hllc"),
                                    ("minmod", "hll")])
def test_two_level_step_matches_oracle(gd, lim, rs):
    h = inputs.amr_hierarchy(gamma=G)
    dt = stable_dt(h)
    cn, fin, fo, ff = amr.step(h, G, dt, limiter=lim, riemann=rs)
    say("amr step", lim, rs)
    gc, gfi, gfo, gff = run_gpu(gd, h, dt, limiter=lim, riemann=rs)
    assert np.array_equal(gfi, fin)
    assert parity_err(gfo, fo) <= 1e-12
    assert parity_err(gff, ff) <= 1e-12
    assert parity_err(gc, cn) <= 1e-12


def test_reflux_launch_alone_matches_oracle(gd):
    """gd_amr_reflux on the oracle's own coarse step and fine fluxes."""
    import oracle
    h = inputs.amr_hierarchy(gamma=G, seed=12)
    dt = stable_dt(h)
    cn, _, fo, ff = amr.step(h, G, dt)
    pre, _, _ = oracle.step(h.coarse, G, h.dx_coarse, dt, periodic=True)
    say("amr reflux alone")
    plan = plan_for(gd, h)
    new = dev(pre)
    plan.reflux(dev(h.coarse), new, dev(fo), dev(ff), G, dt)
    assert parity_err(host(new), cn) <= 1e-12


def test_fp32_matches_oracle(gd):
    import torch
    h = inputs.amr_hierarchy(gamma=G, seed=13)
    dt = stable_dt(h)
    cn, _, fo, _ = amr.step(h, G, dt)
    say("amr fp32")
    gc, _, gfo, _ = run_gpu(gd, h, dt, dtype=torch.float32)
    assert parity_err(gfo, fo) <= 1e-5
    assert parity_err(gc, cn) <= 1e-5


def _totals(h, coarse, interiors):
    own = amr.owner_map(h).transpose(2, 1, 0)
    dv = h.dx_coarse ** 3
    tot, mag = [], []
    for v in range(5):
        terms = list(coarse[v][own < 0] * dv)
        for p in range(len(h.lo)):
            terms.extend((interiors(p)[v] * (dv / 8)).ravel())
        tot.append(math.fsum(terms))
        mag.append(math.fsum(abs(t) for t in terms))
    return np.array(tot), np.array(mag)


def test_composite_state_is_conserved(gd):
    h = inputs.amr_hierarchy(gamma=G, seed=14)
    dt = stable_dt(h)
    say("amr conservation")
    gc, _, gfo, _ = run_gpu(gd, h, dt)
    t0, mag = _totals(h, h.coarse, lambda p: h.fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2])
    t1, _ = _totals(h, gc, lambda p: h.fine.patch_out(gfo, p))
    assert np.all(np.abs(t1 - t0) <= 1e-14 * mag), (t1 - t0) / mag


def test_uniform_state_is_unchanged(gd):
    h = inputs.amr_hierarchy(gamma=G)
    U = np.array([float(x) for x in inputs.conserved(np.array(1.3), 0.4, -0.25, 0.15,
                                                       np.array(0.9), G)])
    h.coarse[...] = U[:, None, None, None]
    for p in range(len(h.lo)):
        h.fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2] = U[:, None, None, None]
    say("amr uniform")
    gc, _, gfo, _ = run_gpu(gd, h, 1e-3)
    assert np.array_equal(gc, h.coarse)
    for p in range(len(h.lo)):
        assert np.array_equal(h.fine.patch_out(gfo, p), h.fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2])


def test_device_dt_gives_the_same_step(gd):
    import torch
    h = inputs.amr_hierarchy(gamma=G, seed=15)
    dt = stable_dt(h)
    say("amr device dt")
    a = run_gpu(gd, h, dt)
    b = run_gpu(gd, h, None, dt_dev=torch.tensor([dt], dtype=torch.float64, device="cuda"))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("boxes", [
    [((0, 2, 2), (8, 2, 3)), ((2, 5, 0), (2, 3, 2))],          # full x span; z at 0
    [((0, 0, 0), (2, 2, 2)), ((6, 6, 6), (2, 2, 2)), ((2, 0, 0), (3, 1, 1))],   # box corners
    [((3, 3, 3), (1, 1, 1))],                                   # one coarse cell
    [],                                                          # no fine level
])
def test_edge_hierarchies(gd, boxes):
    h = inputs.amr_hierarchy(nc=8, gamma=G, boxes=boxes, seed=16)
    dt = stable_dt(h)
    cn, fin, fo, ff = amr.step(h, G, dt)
    say("amr edge hierarchy", boxes)
    gc, gfi, gfo, gff = run_gpu(gd, h, dt)
    assert parity_err(gc, cn) <= 1e-12
    if boxes:
        assert np.array_equal(gfi, fin)
        assert parity_err(gfo, fo) <= 1e-12
        assert parity_err(gff, ff) <= 1e-12


def test_64_box_with_48_patches(gd):
    h = inputs.amr_hierarchy(nc=64, nfine=48, max_size=8, seed=3, gamma=G)
    assert len(h.lo) == 48
    dt = stable_dt(h)
    cn, fin, fo, ff = amr.step(h, G, dt)
    say("amr 64^3 + 48 patches")
    gc, gfi, gfo, gff = run_gpu(gd, h, dt)
    assert np.array_equal(gfi, fin)
    assert parity_err(gfo, fo) <= 1e-12
    assert parity_err(gff, ff) <= 1e-12
    assert parity_err(gc, cn) <= 1e-12


def test_full_size_hierarchy_sampled(gd):
    """The two-level step at the size the benchmark times: a 128^3 periodic
    coarse box with 1024 fine patches (gamma 5/3, seed 21). The whole oracle
    step is too slow here (one coarse flux recomputed per interface face, in
    Python), so: the ghost fill bit for bit everywhere; 64 sampled fine
    patches against the oracle's step of their oracle-filled input; every
    coarse cell away from the interfaces against the oracle's coarse step;
    200 sampled uncovered interface cells against the oracle's coarse step
    plus all their reflux corrections (coarse flux recomputed, fine fluxes
    from the oracle's own fine steps); the covered cells of the sampled
    patches against the average of the oracle's fine outputs; and composite
    conservation over the whole hierarchy."""
    import torch
    import oracle
    g = 5.0 / 3.0
    h = inputs.amr_hierarchy(nc=128, nfine=1024, max_size=12, seed=21, gamma=g)
    dt = oracle.cfl_dt(h.coarse, g, h.dx_coarse / 2, 0.5, periodic=True)
    say("amr full size: gpu step")
    plan = plan_for(gd, h)
    ci = dev(h.coarse)
    fi = dev(np.nan_to_num(h.fine.u_in, nan=-7.0))
    co = torch.empty_like(ci)
    fo = torch.full((h.fine.u_out_size,), float("nan"), dtype=ci.dtype, device="cuda")
    ff = torch.full((h.fine.flux_size,), float("nan"), dtype=ci.dtype, device="cuda")
    plan.step(ci, fi, g, dt, coarse_out=co, fine_out=fo, fine_flux=ff)
    gc, gfi, gfo, gff = host(co), host(fi), host(fo), host(ff)
    say("amr full size: ghost fill")
    fin = amr.fill_ghosts(h, h.coarse)
    assert np.array_equal(gfi, fin)

    dxc = h.dx_coarse
    npatch = len(h.lo)

    def oracle_fine(p):
        nx, ny, nz = (int(v) for v in h.n[p])
        u = fin[h.fine.u_in_off[p]:h.fine.u_in_off[p] + 5 * (nx + 4) * (ny + 4) * (nz + 4)]
        out, fl, _ = oracle.step(u.reshape(5, nz + 4, ny + 4, nx + 4), g, dxc / 2, dt)
        flat = np.full(h.fine.flux_size, np.nan)
        flat[h.fine.flux_off[p]:h.fine.flux_off[p] + fl.size] = fl
        return out, flat

    rng = np.random.default_rng(5)
    say("amr full size: sampled fine patches and their covered cells")
    for p in rng.choice(npatch, size=64, replace=False):
        out, flat = oracle_fine(p)
        assert parity_err(h.fine.patch_out(gfo, p), out) <= 1e-12, p
        assert bflux_err(h.fine.patch_flux(gff, p), h.fine.patch_flux(flat, p), *h.fine.dims[p]) <= 1e-12, p
        avg = np.zeros_like(h.coarse)
        amr.average_down(_one_patch(h, p), out.ravel(), avg)
        sx, sy, sz = (int(v) for v in h.n[p] // 2)
        x, y, z = (int(v) for v in h.lo[p])
        blk = (slice(None), slice(z, z + sz), slice(y, y + sy), slice(x, x + sx))
        assert parity_err(gc[blk], avg[blk]) <= 1e-12, p

    say("amr full size: coarse cells")
    cref = oracle.step(h.coarse, g, dxc, dt, periodic=True)[0]
    faces = amr.interface_faces(h)
    own = amr.owner_map(h).transpose(2, 1, 0)
    touched = np.zeros(own.shape, dtype=bool)
    by_cell = {}
    for f in faces:
        x, y, z = f[4]
        touched[z, y, x] = True
        by_cell.setdefault((x, y, z), []).append(f)
    plain = (own < 0) & ~touched
    for v in range(5):
        scale = np.abs(cref[v]).max()
        assert np.abs(gc[v][plain] - cref[v][plain]).max() <= 1e-12 * scale, v
    cells = list(by_cell)
    fine_flux = {}
    for c in (cells[i] for i in rng.choice(len(cells), size=200, replace=False)):
        want = cref[:, c[2], c[1], c[0]].copy()
        for p, d, side, cell, out_cell in by_cell[c]:
            if p not in fine_flux:
                fine_flux[p] = oracle_fine(p)[1]
            right = out_cell if side else cell
            Fc = amr.coarse_face_flux(h.coarse, d, right, g, dxc, dt, "minmod", "hllc")
            Ff = amr.fine_face_mean(h, fine_flux[p], p, d, side, cell)
            want += dt / dxc * (Ff - Fc) if side else dt / dxc * (Fc - Ff)
        scale = np.abs(cref).reshape(5, -1).max(axis=1)
        assert np.all(np.abs(gc[:, c[2], c[1], c[0]] - want) <= 1e-12 * scale), c

    say("amr full size: composite conservation")
    t0, mag = _totals(h, h.coarse, lambda p: h.fine.patch_in(p)[:, 2:-2, 2:-2, 2:-2])
    t1, _ = _totals(h, gc, lambda p: h.fine.patch_out(gfo, p))
    assert np.all(np.abs(t1 - t0) <= 1e-13 * mag), (t1 - t0) / mag


def _one_patch(h, p):
    """A view of hierarchy h restricted to patch p whose fine output buffer
    is that patch's interior alone (for the oracle's averaging down)."""
    import types
    n = h.n[p]
    fine = types.SimpleNamespace(patch_out=lambda buf, q: buf.reshape(5, int(n[2]), int(n[1]),
                                                                      int(n[0])))
    return types.SimpleNamespace(lo=[h.lo[p]], n=[n], fine=fine)
