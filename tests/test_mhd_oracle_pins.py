"""Pins of the ideal-MHD oracle (HLLD + GLM cleaning) to what the mathematics
fixes, independently of the oracle itself: reduction of HLLD to the Euler
oracle's HLLC without a field, flux consistency, closed forms of the fast
speed, free-stream preservation, conservation, mirror and axis symmetries,
second-order convergence on the exact circularly polarised Alfven wave, an
exactly preserved stationary contact and static tangential discontinuity, and
the decay of div B under the cleaning (and its persistence without it)."""
import math

import numpy as np
import pytest

import oracle
from oracle import mhd
from helpers import rel_norm_err
from paper_1412_0934_amd import inputs

G = 5.0 / 3.0
LIMS = ["minmod", "mc", "none"]


def _random_prim(rng, field=True):
    W = np.zeros(9)
    W[0] = rng.uniform(0.1, 2.0)
    W[1:4] = rng.normal(0.0, 1.0, 3)
    W[4] = rng.uniform(0.1, 2.0)
    if field:
        W[5:8] = rng.normal(0.0, 1.0, 3)
        W[8] = rng.normal(0.0, 0.1)
    return W


def test_hlld_reduces_to_hllc_without_a_field():
    """Miyoshi & Kusano's solver with B = 0 has the HLLC wave fan and star
    states, so its flux equals the Euler oracle's HLLC flux to rounding."""
    rng = np.random.default_rng(1)
    for t in range(600):
        WL, WR = _random_prim(rng, False), _random_prim(rng, False)
        d = t % 3
        F = mhd.face_flux(d, WL, WR, G, ch=1.0)
        Fe = oracle.face_flux(d, WL[:5], WR[:5], G, "hllc")
        assert np.all(F[5:] == 0.0)
        assert np.abs(F[:5] - Fe).max() <= 1e-13 * max(1.0, np.abs(Fe).max()), t


def test_face_flux_is_consistent():
    """F(W, W) is the physical GLM-MHD flux of W."""
    rng = np.random.default_rng(2)
    for t in range(600):
        W = _random_prim(rng)
        d = t % 3
        F = mhd.face_flux(d, W, W, G, ch=1.3)
        Fp = mhd.phys_flux(d, W, G, ch=1.3)
        assert np.abs(F - Fp).max() <= 1e-13 * np.abs(Fp).max(), t


def test_fast_speed_closed_forms():
    rng = np.random.default_rng(3)
    for _ in range(50):
        W = _random_prim(rng)
        a2 = G * W[4] / W[0]
        for d in range(3):
            Wp = W.copy()
            Wp[5 + d] = 0.0            # field normal to the direction: cf^2 = a^2 + b^2
            b2 = float(np.sum(Wp[5:8] ** 2)) / W[0]
            assert math.isclose(mhd.fast_speed(d, Wp, G) ** 2, a2 + b2, rel_tol=1e-13)
            Wa = W.copy()
            Wa[5:8] = 0.0
            Wa[5 + d] = W[5 + d]       # field along the direction: cf = max(a, b_n)
            bn = abs(W[5 + d]) / math.sqrt(W[0])
            assert math.isclose(mhd.fast_speed(d, Wa, G), max(math.sqrt(a2), bn), rel_tol=1e-13)


def test_free_stream_is_preserved_bit_for_bit():
    n = 6
    one = np.ones((n, n + 1, n + 2))
    u = inputs.mhd_conserved(1.3 * one, 0.4, -0.2, 0.3, 0.7 * one, 0.8, -0.5, 0.3, gamma=G)
    dt, ch = mhd.cfl(u, G, 1 / n)
    out, hits = mhd.step(u, G, 1 / n, dt, ch, alpha=0.1)
    assert hits == 0
    assert np.array_equal(out, u)


@pytest.mark.parametrize("lim", LIMS)
def test_conservation_on_a_periodic_box(lim):
    u = inputs.mhd_random_box(7, 6, 5, seed=4)
    dx = 1 / 7
    dt, ch = mhd.cfl(u, G, dx)
    out, _ = mhd.step(u, G, dx, dt, ch, alpha=0.0, limiter=lim)
    for v in range(9):
        before, after = math.fsum(u[v].ravel()), math.fsum(out[v].ravel())
        scale = math.fsum(np.abs(u[v]).ravel())
        assert abs(after - before) <= 1e-13 * scale, v


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("lim", LIMS)
def test_mirror_symmetry(axis, lim):
    """x_a -> -x_a with v_a and B_a negated (psi and div B unchanged)."""
    u = inputs.mhd_random_box(6, 5, 7, seed=5)
    dx = 1 / 7
    dt, ch = mhd.cfl(u, G, dx)
    flip = 3 - axis

    def reflect(a):
        r = np.flip(a, axis=flip).copy()
        r[1 + axis] *= -1.0
        r[5 + axis] *= -1.0
        return r

    out, _ = mhd.step(u, G, dx, dt, ch, alpha=0.1, limiter=lim)
    out_r, _ = mhd.step(reflect(u), G, dx, dt, ch, alpha=0.1, limiter=lim)
    assert rel_norm_err(out_r, reflect(out), 9) <= 1e-14


@pytest.mark.parametrize("lim", LIMS)
def test_axis_permutation(lim):
    u = inputs.mhd_random_box(5, 6, 7, seed=6)
    dx = 1 / 7
    dt, ch = mhd.cfl(u, G, dx)

    def permute(a):
        # new (x, y, z) = old (y, z, x); vector components follow their axes
        b = np.transpose(a, (0, 3, 1, 2)).copy()
        return b[[0, 2, 3, 1, 4, 6, 7, 5, 8]]

    out, _ = mhd.step(u, G, dx, dt, ch, alpha=0.1, limiter=lim)
    out_p, _ = mhd.step(permute(u), G, dx, dt, ch, alpha=0.1, limiter=lim)
    assert rel_norm_err(out_p, permute(out), 9) <= 1e-14


def _alfven_period(n, lim, axis=0):
    u0 = inputs.alfven_wave(n, axis=axis)
    u, t, dx = u0.copy(), 0.0, 1.0 / n
    while t < 1.0 - 1e-14:
        dt, ch = mhd.cfl(u, G, dx, 0.4)
        dt = min(dt, 1.0 - t)
        u, _ = mhd.step(u, G, dx, dt, ch, alpha=0.1, limiter=lim)
        t += dt
    return u0, u


def _alfven_error(n, lim):
    # after one period the exact solution is the initial state
    u0, u = _alfven_period(n, lim)
    return float(np.mean(np.abs(u[6] - u0[6])))


def test_alfven_wave_converges_at_second_order():
    errs = [_alfven_error(n, "none") for n in (16, 32, 64)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= 1.9, (errs, rates)
    errs = [_alfven_error(n, "minmod") for n in (32, 64, 128)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[0] >= 1.4 and rates[1] >= 1.6, (errs, rates)


def test_alfven_wave_along_each_axis_agrees():
    """The same wave along y and z gives the x result with the vector
    components permuted, to rounding (sums over vector components run in a
    fixed axis order; fixed dt, since the CFL sum over axes rounds too)."""
    n = 32
    dx = 1.0 / n
    dt = 0.4 * dx / 3.5

    def run(axis):
        u = inputs.alfven_wave(n, axis=axis)
        for _ in range(20):
            u, _ = mhd.step(u, G, dx, dt, 1.2, alpha=0.1, limiter="minmod")
        return u.reshape(9, n)

    line = run(0)
    for a in (1, 2):
        perm = [0] + [1 + (a + c) % 3 for c in range(3)] + [4] + [5 + (a + c) % 3 for c in range(3)] + [8]
        # the normal momentum and psi are zero up to rounding: compare
        # against the scale of the whole state
        assert np.abs(run(a)[perm] - line).max() <= 1e-14 * np.abs(line).max(), a


def test_stationary_contact_is_kept():
    """A density jump at rest in uniform pressure and field is an isolated
    contact; HLLD resolves it exactly, so a step leaves it in place."""
    n = 16
    x = (np.arange(n) + 0.5) / n
    rho = np.where((x > 0.25) & (x < 0.7), 2.5, 0.6)[None, None, :] * np.ones((2, 3, n))
    u = inputs.mhd_conserved(rho, 0.0, 0.0, 0.0, 1.0, 0.9, 0.5, -0.3, gamma=G)
    dt, ch = mhd.cfl(u, G, 1 / n)
    out, _ = mhd.step(u, G, 1 / n, dt, ch, alpha=0.1)
    assert rel_norm_err(out, u, 9) <= 1e-14


def test_static_tangential_discontinuity_is_kept():
    """No normal field, gas plus magnetic pressure p + |B|^2/2 equal on both
    sides, fluid at rest: a static tangential discontinuity, which a step
    leaves in place (the limited slopes vanish at a step profile, and HLLD
    then carries no momentum across it)."""
    n = 16
    x = (np.arange(n) + 0.5) / n
    left = ((x > 0.25) & (x < 0.7))[None, None, :] * np.ones((2, 3, n))
    by = np.where(left, 1.0, 0.3)
    bz = np.where(left, -0.2, 0.6)
    p = 1.0 + 0.5 * (1.0 + 0.04) - 0.5 * (by ** 2 + bz ** 2)
    rho = np.where(left, 0.8, 1.7)
    u = inputs.mhd_conserved(rho, 0.0, 0.0, 0.0, p, 0.0, by, bz, gamma=G)
    dt, ch = mhd.cfl(u, G, 1 / n)
    out, _ = mhd.step(u, G, 1 / n, dt, ch, alpha=0.1)
    # momentum is zero up to rounding: measure against the scale of the state
    assert np.abs(out - u).max() <= 1e-14 * np.abs(u).max()


def _div_b_norm(u, dx):
    bx = u[5]
    d = (np.roll(bx, -1, axis=2) - np.roll(bx, 1, axis=2)) / (2 * dx)
    return float(np.sqrt(np.mean(d * d)))


@pytest.mark.parametrize("clean", [True, False])
def test_glm_cleaning_removes_div_b(clean):
    """B_x = 1 + 0.1 sin(2 pi x) has div B != 0 and, in ideal MHD without
    cleaning, would stay; the GLM waves and the damping of psi carry it off."""
    n = 64
    x = (np.arange(n) + 0.5) / n
    bx = (1.0 + 0.1 * np.sin(2 * np.pi * x))[None, None, :]
    u = inputs.mhd_conserved(np.ones((1, 1, n)), 0.0, 0.0, 0.0, 1.0, bx, 0.2, 0.0, gamma=G)
    dx = 1.0 / n
    d0 = _div_b_norm(u, dx)
    t = 0.0
    while t < 2.0:
        dt, ch = mhd.cfl(u, G, dx, 0.4)
        u, _ = mhd.step(u, G, dx, dt, ch if clean else 1e-9, alpha=0.5 if clean else 0.0)
        t += dt
    d1 = _div_b_norm(u, dx)
    if clean:
        assert d1 <= 0.2 * d0, (d0, d1)
    else:
        assert abs(d1 - d0) <= 0.02 * d0, (d0, d1)


def test_one_dimensional_reduction():
    line = inputs.alfven_wave(24)
    box = np.broadcast_to(line, (9, 3, 2, 24)).copy()
    dt, ch = mhd.cfl(line, G, 1 / 24)
    out_l, _ = mhd.step(line, G, 1 / 24, dt, ch, alpha=0.1)
    out_b, _ = mhd.step(box, G, 1 / 24, dt, ch, alpha=0.1)
    assert np.array_equal(out_b, np.broadcast_to(out_l, out_b.shape))
