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

Characteristic tracing (ppm_ct, ppm_ct_unlimited) keeps every invariant above
and adds:
* on linear primitive profiles with every wave moving towards the upper
  faces (supersonic along x, y and z) it is the Hancock step, face for face
  where the flux depends on it;
* a contact (uniform velocity below the sound speed, uniform pressure) is
  carried by exactly the PPM advection scheme: the density flux through a
  face is u times the parabola's average over the last u dt/dx of the
  upwind cell;
* on an advected smooth contact the whole step converges at third order
  (unlimited parabola), where the Hancock step converges at second.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact_riemann as er
from paper_1412_0934_amd import inputs

G = 5.0 / 3.0
PPM = ["ppm", "ppm_unlimited", "ppm_ct", "ppm_ct_unlimited"]
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


# ----------------------------------------------------------------- characteristic tracing


@pytest.mark.parametrize("traced,hancock", [("ppm_ct_unlimited", "ppm_unlimited"),
                                            ("ppm_ct", "ppm")])
def test_tracing_is_the_hancock_step_when_every_wave_moves_towards_the_face(traced, hancock):
    """Linear primitives (the parabola is the line, a_6 = 0) moving at three
    times the sound speed along +x, +y and +z: every wave reaches the upper
    faces, where the traced state is a_R - dt/(2dx) A_d (a_R - a_L) plus the
    transverse terms, the Hancock state; the lower-face states differ, but
    every face's flux is the upwind one and never reads them."""
    n = 8
    idx = np.arange(-3, n + 3, dtype=float) / n
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    rng = np.random.default_rng(4)
    a = rng.uniform(-0.05, 0.05, (5, 3))
    lin = lambda c, k: c + a[k, 0] * X + a[k, 1] * Y + a[k, 2] * Z     # noqa: E731
    u = inputs.conserved(lin(1.0, 0), lin(4.0, 1), lin(4.2, 2), lin(3.9, 3), lin(1.0, 4), G)
    dx, dt = 1 / n, 0.1 / n
    for rs in SOLVERS:
        t, bt, _ = oracle.step(u, G, dx, dt, ng=3, limiter=traced, riemann=rs)
        h, bh, _ = oracle.step(u, G, dx, dt, ng=3, limiter=hancock, riemann=rs)
        assert rel_norm_err(t, h) <= 1e-14
        assert np.abs(bt - bh).max() <= 1e-14 * np.abs(bh).max()
    # and the steps do differ when some waves move away from a face
    a *= 6.0
    u2 = inputs.conserved(lin(1.0, 0), lin(0.2, 1), lin(0.1, 2), lin(-0.2, 3), lin(1.0, 4), G)
    t, _, _ = oracle.step(u2, G, dx, 4 * dt, ng=3, limiter=traced)
    h, _, _ = oracle.step(u2, G, dx, 4 * dt, ng=3, limiter=hancock)
    assert rel_norm_err(t, h) > 1e-6


def _contact(n, rho_of_x, u0=0.7, p0=1.0):
    """A periodic n x 2 x 2 box holding a contact: density rho_of_x(x) at the
    cell centres, velocity (u0, 0, 0) below the sound speed, pressure p0."""
    x = (np.arange(n) + 0.5) / n
    shape = (2, 2, n)
    zero = np.zeros(shape)
    rho = np.broadcast_to(rho_of_x(x), shape)
    return inputs.conserved(rho, u0 + zero, zero, zero, p0 + zero, G)


@pytest.mark.parametrize("lim", ["ppm_ct", "ppm_ct_unlimited"])
@pytest.mark.parametrize("u0", [0.7, -0.7])
def test_contact_is_carried_by_the_ppm_advection_scheme(lim, u0):
    """The density flux through a face is u times the parabola's average over
    the part of the upwind cell that crosses the face in dt: the last s of
    the cell on the left for u > 0, the first |s| of the cell on the right
    for u < 0 (s = u dt/dx), A = a_R - (s/2)(a_R - a_L - (1 - 2s/3) a_6) and
    B = a_L + (|s|/2)(a_R - a_L + (1 - 2|s|/3) a_6); rho' = rho - (dt/dx)
    (F_{i+1/2} - F_{i-1/2}). The edges come from the pinned parabola
    construction (oracle.ppm_edges)."""
    n = 40
    rng = np.random.default_rng(7)
    rho_c = 1.0 + 0.3 * rng.random(n)
    U = _contact(n, lambda x: rho_c, u0=u0)
    dx = 1.0 / n
    for t in (0.1, 0.45, 0.9):
        dt = t * dx / abs(u0)
        out, _, _ = oracle.step(U, G, dx, dt, periodic=True, limiter=lim)
        parab = "ppm" if lim == "ppm_ct" else "ppm_unlimited"
        face = np.empty(n)        # the upwind average through face i + 1/2
        for i in range(n):
            c = i if u0 > 0 else (i + 1) % n
            a5 = rho_c[[(c + m) % n for m in (-2, -1, 0, 1, 2)]]
            aL, aR = oracle.ppm_edges(a5, parab)
            a6 = 6.0 * (rho_c[c] - 0.5 * (aL + aR))
            if u0 > 0:
                face[i] = aR - 0.5 * t * (aR - aL - (1.0 - 2.0 * t / 3.0) * a6)
            else:
                face[i] = aL + 0.5 * t * (aR - aL + (1.0 - 2.0 * t / 3.0) * a6)
        F = u0 * face
        want = rho_c - dt / dx * (F - np.roll(F, 1))
        assert np.abs(out[0, 0, 0] - want).max() <= 1e-14 * np.abs(want).max(), t
        # the contact stays a contact: velocity and pressure unchanged
        vel = out[1] / out[0]
        pres = (G - 1.0) * (out[4] - 0.5 * out[1] * vel)
        assert np.abs(vel - u0).max() <= 1e-13 and np.abs(pres - 1.0).max() <= 1e-13




def _primitive_jacobian(W, d, gamma):
    """A_d of the primitive Euler system in (rho, u, v, w, p)."""
    rho, p, un = W[0], W[4], W[1 + d]
    A = np.eye(5) * un
    n = 1 + d
    A[0, n] = rho
    A[n, 4] = 1.0 / rho
    A[4, n] = gamma * p
    return A


def _parabola_average(aL, aR, a0, lo, hi):
    """Average over [lo, hi] (cell fractions) of the parabola with edges aL,
    aR and mean a0, by three-point Gauss quadrature (exact for quadratics)."""
    a6 = 6.0 * (a0 - 0.5 * (aL + aR))
    nodes = np.array([-math.sqrt(0.6), 0.0, math.sqrt(0.6)])
    weights = np.array([5.0, 8.0, 5.0]) / 18.0
    xi = lo + (hi - lo) * (nodes + 1.0) / 2.0
    vals = aL[:, None] + xi[None, :] * ((aR - aL)[:, None] + a6[:, None] * (1.0 - xi[None, :]))
    return vals @ weights


def test_trace_of_each_characteristic_family():
    """The traced state of a face, family by family: with P_mu the spectral
    projector of the primitive Jacobian onto the eigenvalue mu (from numpy's
    eigendecomposition, not the oracle's eigenvectors), the state is the
    edge value plus, for each eigenvalue whose wave moves towards the face,
    P_mu (average of the parabolas over the part of the cell that wave
    sweeps in dt - edge value)."""
    rng = np.random.default_rng(21)
    for trial in range(60):
        W = np.array([0.5 + rng.random(), *rng.normal(0, 1.2, 3), 0.5 + rng.random()])
        aL = W + rng.normal(0, 0.1, 5)
        aR = W + rng.normal(0, 0.1, 5)
        d = trial % 3
        dx = 0.1
        dt = rng.uniform(0.01, 0.9) * dx / (abs(W[1 + d]) + math.sqrt(G * W[4] / W[0]))
        A = _primitive_jacobian(W, d, G)
        lam, R = np.linalg.eig(A)
        lam, R = lam.real, R.real
        Linv = np.linalg.inv(R)
        for upper in (True, False):
            got = oracle.ppm_trace(W, aL, aR, d, upper, G, dx, dt)
            edge = aR if upper else aL
            want = edge.copy()
            for mu in np.unique(np.round(lam, 12)):
                pick = np.abs(lam - mu) < 1e-9
                proj = R[:, pick] @ Linv[pick, :]
                s = mu * dt / dx
                if upper and s > 0:
                    avg = _parabola_average(aL, aR, W, 1.0 - s, 1.0)
                elif not upper and s < 0:
                    avg = _parabola_average(aL, aR, W, 0.0, -s)
                else:
                    continue
                want += proj @ (avg - edge)
            assert np.abs(got - want).max() <= 1e-12 * (1 + np.abs(want).max()), (trial, upper)


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


def _sod_run(n, gamma, t_end=0.2, cfl=0.4, lim="ppm"):
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
        U, _, _ = oracle.step(u, gamma, dx, dt, ng=3, limiter=lim)
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


# ----------------------------------------------------------------- tracing: whole-step orders


def _advected_sine_error(n, lim, cfl=0.5):
    """L1 density error after one crossing of a smooth contact
    rho = 1 + 0.2 sin(2 pi x) at u = 0.7, pressure 1, against the exact cell
    averages."""
    u0 = 0.7
    dx = 1.0 / n
    avg = lambda x0: 1.0 + 0.2 * (np.cos(2 * np.pi * (x0 - dx / 2)) -              # noqa: E731
                                  np.cos(2 * np.pi * (x0 + dx / 2))) / (2 * np.pi * dx)
    x = (np.arange(n) + 0.5) / n
    U = _contact(n, avg)
    # one crossing in steps whose Courant number on the fastest wave
    # (u + c, c at the lowest density) is at most cfl
    smax = u0 + math.sqrt(G * 1.0 / 0.8)
    steps = int(math.ceil(smax / (u0 * cfl * dx)))
    dt = 1.0 / u0 / steps
    for _ in range(steps):
        U = oracle.step(U, G, dx, dt, periodic=True, limiter=lim)[0]
    return float(np.abs(U[0, 0, 0] - avg(x)).mean())


def test_traced_step_is_third_order_on_a_smooth_contact():
    """The whole step, not only the reconstruction: with tracing the time
    average over the domain of dependence is exact for a contact, so the
    unlimited parabola's spatial order shows (>= 2.8 measured between 32, 64
    and 128 cells at CFL 0.5 on u + c); the Hancock step on the same data is
    held to second order by its time discretisation."""
    errs = {lim: [_advected_sine_error(n, lim) for n in (32, 64, 128)]
            for lim in ("ppm_ct_unlimited", "ppm_unlimited")}
    ct = errs["ppm_ct_unlimited"]
    orders = [math.log2(ct[i] / ct[i + 1]) for i in range(2)]
    assert min(orders) >= 2.8, (ct, orders)
    hk = errs["ppm_unlimited"]
    hk_order = math.log2(hk[1] / hk[2])
    assert 1.7 <= hk_order <= 2.4, (hk, hk_order)
    assert ct[2] < hk[2]


def test_traced_sod_converges_to_exact_solution():
    gamma = 1.4
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    errs = []
    for n in (128, 256, 512):
        U = _sod_run(n, gamma, lim="ppm_ct")
        assert np.all(U[0] > 0) and np.all(np.isfinite(U))
        rho_ex, _, _ = er.cell_averages(np.linspace(0, 1, n + 1), 0.2, 0.5, L, R, gamma)
        errs.append(np.abs(U[0] - rho_ex).mean())
    # L1 convergence at a contact is about 2/3 for second-order TVD schemes;
    # measured with tracing: 1.23 then 0.57 (overall 0.90), at 512 cells an
    # error of 6.0e-4
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    overall = 0.5 * math.log2(errs[0] / errs[2])
    assert min(orders) >= 0.5 and overall >= 0.7, (errs, orders)
    assert errs[2] < 1e-3
