"""Pins of the PPM oracle (CPU only): the parabola against closed forms and its
defining properties, the step against the invariants the PLM step satisfies,
and the order of accuracy the parabola buys.

* unlimited interface values are exact for cell averages of any cubic;
* the limited parabola has no extremum inside a cell, is flat at a local
  extremum and keeps its edge values between the neighbouring cell values;
  on linear data it is the exact line;
* on data whose primitives are linear in x the unlimited PPM step equals the
  unlimited (central-slope) PLM step, whose face states are the same line;
* free stream bit for bit, conservation on a periodic box, the boundary-flux
  telescoping identity, mirror symmetry, axis permutation, one-dimensional
  reduction, corner and deep edge ghosts never read;
* the semi-discrete residual on exact cell averages of an advected sine is
  fourth-order accurate for the unlimited parabola, and for the limited one
  away from the sine's extrema (where PLM is second order);
* Sod: the same plateaus and L1 convergence as the PLM step.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact_riemann as er
from paper_1412_0934_amd import inputs

G = 5.0 / 3.0
PPM = ["ppm", "ppm_unlimited"]
SOLVERS = ["hllc", "hll"]


def rel_norm_err(a, b):
    a = np.asarray(a).reshape(5, -1)
    b = np.asarray(b).reshape(5, -1)
    den = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return float((np.abs(a - b).max(axis=1) / den).max())


def uniform_state(shape, rho, v, p, gamma=G):
    one = np.ones(shape)
    return inputs.conserved(rho * one, v[0] * one, v[1] * one, v[2] * one, p * one, gamma)


# ----------------------------------------------------------------- the parabola


def test_unlimited_interfaces_are_exact_for_cubics():
    rng = np.random.default_rng(0)
    for _ in range(100):
        c = rng.normal(size=4)
        # exact averages of c0 + c1 x + c2 x^2 + c3 x^3 over [i - 1/2, i + 1/2]
        F = lambda x: c[0] * x + c[1] * x ** 2 / 2 + c[2] * x ** 3 / 3 + c[3] * x ** 4 / 4
        f = lambda x: c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
        a = np.array([F(i + 0.5) - F(i - 0.5) for i in range(-2, 3)])
        aL, aR = oracle.ppm_edges(a, "ppm_unlimited")
        scale = np.abs(a).max()
        assert abs(aL - f(-0.5)) <= 1e-13 * scale and abs(aR - f(0.5)) <= 1e-13 * scale


def test_limited_parabola_properties():
    rng = np.random.default_rng(1)
    for _ in range(3000):
        a = rng.normal(size=5) * rng.choice([1e-3, 1.0, 1e3])
        aL, aR = oracle.ppm_edges(a, "ppm")
        a0 = a[2]
        if (a[3] - a0) * (a0 - a[1]) <= 0:
            continue       # the cell is a local extremum of the data: see below
        # edges between the neighbouring values (the interface interpolation
        # with MC slopes stays inside the data's range across each face)
        assert min(a[1], a0) - 1e-12 * abs(a0) <= aL <= max(a[1], a0) + 1e-12 * abs(a0)
        assert min(a0, a[3]) - 1e-12 * abs(a0) <= aR <= max(a0, a[3]) + 1e-12 * abs(a0)
        # the parabola a(s) = aL + s (D + a6 (1 - s)), s in [0, 1], is monotone:
        # its derivative D + a6 (1 - 2 s) keeps the sign of D at both ends
        D, a6 = aR - aL, 6.0 * (a0 - 0.5 * (aL + aR))
        tol = 1e-12 * max(abs(D), abs(a6), 1e-300)
        assert (D + a6) * D >= -tol * abs(D) and (D - a6) * D >= -tol * abs(D)


def test_limited_parabola_is_flat_at_extrema_and_exact_on_lines():
    rng = np.random.default_rng(2)
    for _ in range(500):
        a0 = rng.normal()
        up = np.abs(rng.normal(size=4)) + 0.1
        a = np.array([a0 - up[0], a0 - up[1], a0, a0 - up[2], a0 - up[3]])    # a maximum
        assert oracle.ppm_edges(a, "ppm") == (a0, a0)
        assert oracle.ppm_edges(-a, "ppm") == (-a0, -a0)
        s, b = rng.normal(), rng.normal()
        line = b + s * np.arange(-2, 3, dtype=float)
        aL, aR = oracle.ppm_edges(line, "ppm")
        assert abs(aL - (b - s / 2)) <= 1e-14 * (abs(b) + abs(s)) * 4
        assert abs(aR - (b + s / 2)) <= 1e-14 * (abs(b) + abs(s)) * 4


# ----------------------------------------------------------------- whole step


def test_linear_primitives_give_the_plm_step():
    n = 12
    x = np.arange(-3, n + 3, dtype=float) / n
    shape3 = (n + 6, n + 6, n + 6)

    def along_x(f):
        return np.broadcast_to(f[None, None, :], shape3)

    rng = np.random.default_rng(3)
    s = rng.uniform(-0.3, 0.3, 5)
    u3 = inputs.conserved(along_x(1 + s[0] * x), along_x(0.2 + s[1] * x), along_x(-0.1 + s[2] * x),
                          along_x(0.3 + s[3] * x), along_x(1 + s[4] * x), G)
    u2 = u3[:, 1:-1, 1:-1, 1:-1].copy()
    dx, dt = 1 / n, 0.2 / n
    a, ba, _ = oracle.step(u3, G, dx, dt, ng=3, limiter="ppm_unlimited")
    b, bb, _ = oracle.step(u2, G, dx, dt, ng=2, limiter="none")
    assert rel_norm_err(a, b) <= 1e-13
    assert np.allclose(ba, bb, rtol=0, atol=1e-13 * np.abs(bb).max())


@pytest.mark.parametrize("lim", PPM)
@pytest.mark.parametrize("rs", SOLVERS)
@pytest.mark.parametrize("periodic", [False, True])
def test_free_stream_is_bitwise(lim, rs, periodic):
    U = uniform_state((5, 6, 7), 1.3, (0.4, -0.7, 0.25), 0.8)
    u = U if periodic else inputs.outflow_fill(U, 3)
    out, _, hits = oracle.step(u, G, 0.01, 0.002, ng=3, periodic=periodic, limiter=lim, riemann=rs)
    assert hits == 0
    assert np.array_equal(out, U)


@pytest.mark.parametrize("lim", PPM)
@pytest.mark.parametrize("rs", SOLVERS)
def test_conservation_periodic(lim, rs):
    u = inputs.turbulent_box(16, mach=2.0)
    dx = 1 / 16
    dt = oracle.cfl_dt(u, G, dx, periodic=True)
    out, _, _ = oracle.step(u, G, dx, dt, periodic=True, limiter=lim, riemann=rs)
    assert np.all(np.isfinite(out))
    for v in range(5):
        before = math.fsum(u[v].ravel())
        after = math.fsum(out[v].ravel())
        scale = math.fsum(np.abs(u[v]).ravel())
        assert abs(after - before) <= 1e-13 * scale, v


@pytest.mark.parametrize("lim", PPM)
def test_bflux_telescoping_identity(lim):
    nx, ny, nz = 7, 5, 6
    u = inputs.random_patch(nx, ny, nz, ng=3, seed=4)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, ng=3)
    out, b, _ = oracle.step(u, G, dx, dt, ng=3, limiter=lim)
    sh = oracle.split_bflux(b, nx, ny, nz)
    inner = u[:, 3:-3, 3:-3, 3:-3]
    for v in range(5):
        lhs = math.fsum(out[v].ravel()) - math.fsum(inner[v].ravel())
        net = (math.fsum(sh["x+"][v].ravel()) - math.fsum(sh["x-"][v].ravel())
               + math.fsum(sh["y+"][v].ravel()) - math.fsum(sh["y-"][v].ravel())
               + math.fsum(sh["z+"][v].ravel()) - math.fsum(sh["z-"][v].ravel()))
        scale = math.fsum(np.abs(inner[v]).ravel())
        assert abs(lhs + dt / dx * net) <= 1e-13 * scale, v


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("lim", PPM)
def test_mirror_symmetry(axis, lim):
    u = inputs.random_patch(6, 5, 7, ng=3, seed=7)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, ng=3)
    flip = 3 - axis

    def reflect(a):
        r = np.flip(a, axis=flip).copy()
        r[1 + axis] *= -1.0
        return r

    out, _, _ = oracle.step(u, G, dx, dt, ng=3, limiter=lim)
    out_r, _, _ = oracle.step(reflect(u), G, dx, dt, ng=3, limiter=lim)
    assert rel_norm_err(out_r, reflect(out)) <= 1e-14


@pytest.mark.parametrize("lim", PPM)
@pytest.mark.parametrize("rs", SOLVERS)
def test_axis_permutation(lim, rs):
    u = inputs.random_patch(5, 6, 7, ng=3, seed=8)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, ng=3)

    def permute(a):
        b = np.transpose(a, (0, 3, 1, 2)).copy()
        return b[[0, 2, 3, 1, 4]]

    out, _, _ = oracle.step(u, G, dx, dt, ng=3, limiter=lim, riemann=rs)
    out_p, _, _ = oracle.step(permute(u), G, dx, dt, ng=3, limiter=lim, riemann=rs)
    assert rel_norm_err(out_p, permute(out)) <= 1e-14


@pytest.mark.parametrize("lim", PPM)
def test_one_dimensional_reduction(lim):
    n = 24
    x = (np.arange(n) + 0.5) / n
    rho = 1.0 + 0.5 * (x > 0.4) + 0.1 * np.sin(6 * x)
    p = 1.0 + 0.8 * (x < 0.6)
    ux = 0.3 * np.cos(5 * x)
    shape = (4, 3, n)
    zero = np.zeros(shape)
    U = inputs.conserved(np.broadcast_to(rho, shape), np.broadcast_to(ux, shape), zero, zero,
                         np.broadcast_to(p, shape), G)
    out, _, _ = oracle.step(inputs.outflow_fill(U, 3), G, 1 / n, 0.004, ng=3, limiter=lim)
    for v in range(5):
        assert np.array_equal(out[v], np.broadcast_to(out[v, :1, :1, :], out[v].shape))
    assert np.all(out[2] == 0.0) and np.all(out[3] == 0.0)


def test_only_the_stencil_is_read():
    """Face ghosts to depth 3 and edge ghosts at depths (1, <= 2) are read;
    poisoning every other ghost (corners, deeper edges) changes nothing. The
    unlimited parabola carries a NaN through (the MC slope maps a NaN
    difference to zero), so a read of a poisoned cell would show."""
    u = inputs.random_patch(5, 6, 4, ng=3, seed=9)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, ng=3)
    ref, bref, _ = oracle.step(u, G, dx, dt, ng=3, limiter="ppm_unlimited")
    poisoned = u.copy()
    gz, gy, gx = u.shape[1:]
    for k in range(gz):
        for j in range(gy):
            for i in range(gx):
                depth = sorted(max(3 - c, c - (n - 4), 0) for c, n in ((i, gx), (j, gy), (k, gz)))
                nout = sum(d > 0 for d in depth)
                if nout == 3 or (nout == 2 and not (depth[1] == 1 and depth[2] <= 2)):
                    poisoned[:, k, j, i] = np.nan
    out, b, _ = oracle.step(poisoned, G, dx, dt, ng=3, limiter="ppm_unlimited")
    assert np.array_equal(out, ref) and np.array_equal(b, bref)
    # and a deep edge ghost that the stencil does read does matter
    poisoned = u.copy()
    poisoned[:, 3, 1, 2] = np.nan           # x depth 1, y depth 2, z interior
    out, _, _ = oracle.step(poisoned, G, dx, dt, ng=3, limiter="ppm_unlimited")
    assert not np.all(np.isfinite(out))


def test_ghosted_ppm_needs_three_layers():
    u = inputs.random_patch(4, 4, 4, ng=2, seed=1)
    with pytest.raises(ValueError):
        oracle.step(u, G, 1 / 64, 1e-3, ng=2, limiter="ppm")


# ----------------------------------------------------------------- order of accuracy


def _sine_cell_averages(n):
    x = np.arange(n + 1) / n
    avg = 1 + 0.2 * (np.cos(2 * np.pi * x[:-1]) - np.cos(2 * np.pi * x[1:])) / (2 * np.pi / n)
    rho = avg.reshape(1, 1, n)
    one = np.ones_like(rho)
    return inputs.conserved(rho, one, 0 * one, 0 * one, one, 1.4)


def _residual_error(n, lim, mask_extrema=False):
    """Mean |R - R_exact| of the density residual R = d(rho_bar)/dt, from two
    tiny steps with Richardson extrapolation in dt (removing the Hancock
    predictor's O(dt) term), against the exact -(rho(x+) - rho(x-))/dx of unit
    speed advection."""
    U = _sine_cell_averages(n)
    dx = 1.0 / n
    dt = 1e-3 * dx
    a, _, _ = oracle.step(U, 1.4, dx, dt, periodic=True, limiter=lim)
    b, _, _ = oracle.step(U, 1.4, dx, 2 * dt, periodic=True, limiter=lim)
    R = ((4 * (a - U) - (b - U)) / (2 * dt))[0, 0, 0, :]
    x = np.arange(n + 1) / n
    f = 1 + 0.2 * np.sin(2 * np.pi * x)
    err = np.abs(R + (f[1:] - f[:-1]) / dx)
    if mask_extrema:
        xc = (np.arange(n) + 0.5) / n
        err = err[(np.abs(xc - 0.25) > 0.12) & (np.abs(xc - 0.75) > 0.12)]
    return err.mean()


@pytest.mark.parametrize("lim,mask,lo,hi", [("ppm_unlimited", False, 3.8, 4.2),
                                            ("ppm", True, 3.8, 4.2),
                                            ("none", False, 1.8, 2.2),
                                            ("mc", True, 1.8, 2.2)])
def test_semi_discrete_order_of_accuracy(lim, mask, lo, hi):
    errs = [_residual_error(n, lim, mask) for n in (32, 64, 128)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(lo <= r <= hi for r in rates), (errs, rates)


def _sod_run(n, gamma, t_end=0.2, cfl=0.4):
    x = (np.arange(n) + 0.5) / n
    rho = np.where(x < 0.5, 1.0, 0.125).reshape(1, 1, n)
    p = np.where(x < 0.5, 1.0, 0.1).reshape(1, 1, n)
    zero = np.zeros((1, 1, n))
    U = inputs.conserved(rho, zero, zero, zero, p, gamma)
    dx = 1.0 / n
    t = 0.0
    while t < t_end - 1e-14:
        u = inputs.outflow_fill(U, 3)
        dt = min(oracle.cfl_dt(u, gamma, dx, cfl, ng=3), t_end - t)
        U, _, _ = oracle.step(u, gamma, dx, dt, ng=3, limiter="ppm")
        t += dt
    return U[:, 0, 0, :]


def test_sod_converges_to_exact_solution():
    gamma = 1.4
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    errs = []
    for n in (128, 256, 512):
        U = _sod_run(n, gamma)
        assert np.all(U[0] > 0) and np.all(np.isfinite(U))
        rho_ex, _, _ = er.cell_averages(np.linspace(0, 1, n + 1), 0.2, 0.5, L, R, gamma)
        errs.append(np.abs(U[0] - rho_ex).mean())
        if n == 512:
            x = (np.arange(n) + 0.5) / n
            p_s, u_s = er.star_state(L, R, gamma)
            rl, rr = er.star_densities(L, R, gamma)
            _, S = er.wave_speeds(L, R, gamma)
            xc, xs = 0.5 + u_s * 0.2, 0.5 + S * 0.2
            tail = 0.5 + 0.2 * (u_s - math.sqrt(gamma * p_s / rl))
            plate_l = (x > tail + 0.02) & (x < xc - 0.02)
            plate_r = (x > xc + 0.02) & (x < xs - 0.02)
            assert abs(U[0][plate_l].mean() / rl - 1) < 0.01
            assert abs(U[0][plate_r].mean() / rr - 1) < 0.01
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    overall = 0.5 * math.log2(errs[0] / errs[2])
    assert min(orders) >= 0.6 and overall >= 0.7, (errs, orders)
    assert errs[2] < 2.5e-3
