"""GPU step with piecewise-parabolic reconstruction through the C ABI against
the PPM oracle: single ghosted patches (ng = 3) and periodic boxes of ragged
shapes, both parabolas and both Riemann solvers, FP64 to 1e-12 and FP32 to
1e-5, outputs and boundary fluxes; free stream; device dt and the CFL step
of the new state; batches of uneven patches in one call (tiny ragged ones,
the 1024-patch batch of 8^3..32^3 every patch, bitwise equality with the
patches stepped one by one, and replays of a captured HIP graph); and the 256^3
periodic turbulent box at full size, checked cell by cell on a sample, each
sampled cell from a 7^3 ghosted cut-out that the oracle steps."""
import numpy as np
import pytest

import oracle
from helpers import bflux_err, parity_err, say
from paper_1412_0934_amd import inputs

pytestmark = pytest.mark.gpu
G = 5.0 / 3.0
# the Hancock half step and characteristic tracing, each with the limited and
# the unlimited parabola
ALL = ["ppm", "ppm_unlimited", "ppm_ct", "ppm_ct_unlimited"]


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


@pytest.mark.parametrize("shape", [(8, 8, 8), (5, 7, 3), (1, 4, 9), (17, 3, 2), (33, 9, 5)])
@pytest.mark.parametrize("lim", ALL)
@pytest.mark.parametrize("rs", ["hllc", "hll"])
def test_ghosted_patch_matches_oracle(gd, shape, lim, rs):
    nx, ny, nz = shape
    u = inputs.random_patch(nx, ny, nz, ng=3, seed=nx + 7 * ny + 31 * nz, generic=True)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, 0.4, ng=3)
    ref, bref, _ = oracle.step(u, G, dx, dt, ng=3, limiter=lim, riemann=rs)
    say("ppm ghosted", shape, lim, rs)
    out, b = gd.step(dev(u), G, dx, dt, ng=3, limiter=lim, riemann=rs)
    assert parity_err(host(out), ref) <= 1e-12
    assert bflux_err(host(b), bref, *shape) <= 1e-12


@pytest.mark.parametrize("shape", [(16, 16, 16), (6, 5, 7), (1, 1, 12), (2, 9, 4)])
@pytest.mark.parametrize("lim", ALL)
def test_periodic_box_matches_oracle(gd, shape, lim):
    nx, ny, nz = shape
    u = inputs.random_patch(nx, ny, nz, ng=3, seed=3 * nx + ny + 5 * nz, generic=True)
    u = u[:, 3:-3, 3:-3, 3:-3].copy()
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, 0.4, periodic=True)
    ref, bref, _ = oracle.step(u, G, dx, dt, periodic=True, limiter=lim)
    say("ppm periodic", shape, lim)
    out, b = gd.step(dev(u), G, dx, dt, periodic=True, limiter=lim)
    assert parity_err(host(out), ref) <= 1e-12
    assert bflux_err(host(b), bref, *shape) <= 1e-12


@pytest.mark.parametrize("shape", [(16384, 1, 1), (1, 3, 16384)])
@pytest.mark.parametrize("lim", ["ppm", "ppm_ct"])
def test_maximum_extents(gd, shape, lim):
    """The largest accepted extent along an axis: 16-bit tile coordinates of
    the staged box (one layer wider than the interior) at their last tile."""
    u = inputs.random_patch(*shape, ng=3, seed=sum(shape), generic=True)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, 0.4, ng=3)
    ref, bref, _ = oracle.step(u, G, dx, dt, ng=3, limiter=lim)
    say("ppm maximum extent", shape, lim)
    out, b = gd.step(dev(u), G, dx, dt, ng=3, limiter=lim)
    assert parity_err(host(out), ref) <= 1e-12
    assert bflux_err(host(b), bref, *shape) <= 1e-12


@pytest.mark.parametrize("lim", ["ppm", "ppm_ct"])
def test_fp32_matches_oracle(gd, lim):
    import torch
    u = inputs.random_patch(12, 10, 9, ng=3, seed=5, generic=True)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, 0.4, ng=3)
    ref, _, _ = oracle.step(u, G, dx, dt, ng=3, limiter=lim)
    say("ppm fp32", lim)
    out, _ = gd.step(dev(u, torch.float32), G, dx, dt, ng=3, limiter=lim)
    assert parity_err(host(out), ref) <= 1e-5


@pytest.mark.parametrize("lim", ALL)
def test_free_stream_is_bitwise(gd, lim):
    one = np.ones((6, 7, 8))
    U = inputs.conserved(1.3 * one, 0.4 * one, -0.7 * one, 0.25 * one, 0.8 * one, G)
    say("ppm free stream", lim)
    out, _ = gd.step(dev(inputs.outflow_fill(U, 3)), G, 0.01, 0.002, ng=3, limiter=lim)
    assert np.array_equal(host(out), U)


def test_ghosted_ppm_needs_three_layers(gd):
    u = inputs.random_patch(4, 4, 4, ng=2, seed=1)
    with pytest.raises(gd.GodunovError):
        gd.step(dev(u), G, 1 / 64, 1e-3, ng=2, limiter="ppm")


def test_device_dt_and_the_next_cfl_step(gd):
    import torch
    u = inputs.random_patch(9, 8, 7, ng=3, seed=6, generic=True)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, 0.4, ng=3)
    say("ppm device dt + cfl")
    ud = dev(u)
    a, _ = gd.step(ud, G, dx, dt, ng=3, limiter="ppm")
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    nxt = torch.empty_like(dtd)
    b, _ = gd.step(ud, G, dx, dt_dev=dtd, ng=3, limiter="ppm", cfl=0.4, dt_next=nxt)
    out = host(b)
    assert np.array_equal(host(a), out)
    want = oracle.cfl_dt(out, G, dx, 0.4, periodic=True)
    assert abs(float(host(nxt)[0]) - want) <= 1e-14 * want


@pytest.mark.parametrize("lim", ALL)
def test_batch_matches_oracle(gd, lim):
    import torch
    rng = np.random.default_rng(8)
    dims = [tuple(int(v) for v in rng.integers(1, 14, size=3)) for _ in range(40)]
    states = [inputs.random_patch(*d, ng=3, seed=100 + i, generic=True) for i, d in enumerate(dims)]
    batch = inputs.pack_batch(states, 3, 1 / 64, order_seed=3)
    dt = min(oracle.cfl_dt(s, G, 1 / 64, 0.4, ng=3) for s in states)
    table = gd.patch_table(batch.dims, 3, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    out = torch.full((batch.u_out_size,), float("nan"), dtype=torch.float64, device="cuda")
    fl = torch.full((batch.flux_size,), float("nan"), dtype=torch.float64, device="cuda")
    say("ppm batch", lim)
    dt_next = torch.empty(1, dtype=torch.float64, device="cuda")
    gd.step_batched(dev(batch.u_in), table, G, out=out, bflux=fl, limiter=lim, cfl=0.4,
                    dt_next=dt_next)
    o, f = host(out), host(fl)
    for p, s in enumerate(states):
        ref, bref, _ = oracle.step(s, G, 1 / 64, dt, ng=3, limiter=lim)
        assert parity_err(batch.patch_out(o, p), ref) <= 1e-12, p
        assert bflux_err(batch.patch_flux(f, p), bref, *batch.dims[p]) <= 1e-12, p
    want = min(oracle.cfl_dt(batch.patch_out(o, p), G, 1 / 64, 0.4, periodic=True)
               for p in range(len(states)))
    assert abs(float(host(dt_next)[0]) - want) <= 1e-14 * want


@pytest.mark.parametrize("lim", ["ppm", "ppm_ct"])
def test_batch_equals_its_patches_stepped_one_by_one(gd, lim):
    """The batched launch marches the same tiles as the single-patch launch
    (other z-ranges, another order): every patch bitwise equal, outputs and
    boundary fluxes, FP64 and FP32."""
    import torch
    rng = np.random.default_rng(12)
    dims = [tuple(int(v) for v in rng.integers(2, 31, size=3)) for _ in range(24)]
    states = [inputs.random_patch(*d, ng=3, seed=200 + i) for i, d in enumerate(dims)]
    batch = inputs.pack_batch(states, 3, 1 / 64, order_seed=5)
    dt = min(oracle.cfl_dt(s, G, 1 / 64, 0.4, ng=3) for s in states)
    table = gd.patch_table(batch.dims, 3, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    for dtype in (torch.float64, torch.float32):
        say("ppm batch vs patches", lim, dtype)
        out = torch.empty(batch.u_out_size, dtype=dtype, device="cuda")
        fl = torch.empty(batch.flux_size, dtype=dtype, device="cuda")
        gd.step_batched(dev(batch.u_in, dtype), table, G, out=out, bflux=fl, limiter=lim)
        o, f = host(out), host(fl)
        for p, st in enumerate(states):
            a, b = gd.step(dev(st, dtype), G, 1 / 64, dt, ng=3, limiter=lim)
            assert np.array_equal(batch.patch_out(o, p), host(a)), p
            assert np.array_equal(batch.patch_flux(f, p), host(b).ravel()), p


@pytest.mark.parametrize("lim", ["ppm", "ppm_ct"])
def test_batch_in_a_hip_graph(gd, lim):
    """Two chained batched steps with the fused CFL reduction (the second
    takes the first's next step from the device) captured in one HIP graph and
    replayed with eager work and synchronisations between the replays: every
    replay bitwise equal to the eager calls, whose first step matches the
    oracle. The persistent launch leaves its work counter at zero and the CFL
    finish leaves its accumulator cleared, so no replay needs a reset."""
    import torch
    rng = np.random.default_rng(21)
    dims = [tuple(int(v) for v in rng.integers(2, 27, size=3)) for _ in range(48)]
    states = [inputs.random_patch(*d, ng=3, seed=300 + i) for i, d in enumerate(dims)]
    batch = inputs.pack_batch(states, 3, 1 / 64, order_seed=6)
    dt = min(oracle.cfl_dt(s, G, 1 / 64, 0.4, ng=3) for s in states)
    table = gd.patch_table(batch.dims, 3, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    u_in = dev(batch.u_in)
    outs = [torch.empty(batch.u_out_size, dtype=torch.float64, device="cuda") for _ in range(2)]
    fls = [torch.empty(batch.flux_size, dtype=torch.float64, device="cuda") for _ in range(2)]
    dts = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in range(2)]

    def steps():
        gd.step_batched(u_in, table, G, out=outs[0], bflux=fls[0], limiter=lim, cfl=0.4,
                        dt_next=dts[0])
        gd.step_batched(u_in, table, G, out=outs[1], bflux=fls[1], dt_dev=dts[0], limiter=lim,
                        cfl=0.4, dt_next=dts[1])

    say("ppm graph: eager reference", lim)
    steps()
    ref = [host(t) for t in outs + fls + dts]
    for p in range(0, len(states), 12):
        want, _, _ = oracle.step(states[p], G, 1 / 64, dt, ng=3, limiter=lim)
        assert parity_err(batch.patch_out(ref[0], p), want) <= 1e-12, p
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        steps()                     # warm-up on another stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("ppm graph: capture", lim)
    with torch.cuda.graph(g):
        steps()
    for r in range(4):
        for t in outs + fls:
            t.fill_(float("nan"))
        for t in dts:
            t.fill_(0.0)
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()   # eager work
        torch.cuda.synchronize()
        say("ppm graph: replay", r)
        g.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        got = [host(t) for t in outs + fls + dts]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), r


@pytest.mark.parametrize("lim", ["ppm", "ppm_ct"])
def test_full_amr_batch_every_patch(gd, lim):
    """1024 ghosted patches of 8^3..32^3 (ng = 3) in one persistent launch,
    every patch against the oracle element by element, and the batch's next
    CFL step."""
    import torch
    batch = inputs.amr_batch(1024, seed=5, ng=3)
    dt = 0.4 * min(batch.dx[p] / oracle.max_signal(batch.patch_in(p), G, ng=3)
                   for p in range(batch.npatch))
    table = gd.patch_table(batch.dims, 3, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    out = torch.full((batch.u_out_size,), float("nan"), dtype=torch.float64, device="cuda")
    fl = torch.full((batch.flux_size,), float("nan"), dtype=torch.float64, device="cuda")
    dt_next = torch.empty(1, dtype=torch.float64, device="cuda")
    say("ppm amr batch", lim)
    gd.step_batched(dev(batch.u_in), table, G, out=out, bflux=fl, limiter=lim, cfl=0.4,
                    dt_next=dt_next)
    o, f = host(out), host(fl)
    worst = 0.0
    smax = 0.0
    for p in range(batch.npatch):
        ref, bref, _ = oracle.step(batch.patch_in(p), G, batch.dx[p], dt, ng=3, limiter=lim)
        e = max(parity_err(batch.patch_out(o, p), ref),
                bflux_err(batch.patch_flux(f, p), bref, *batch.dims[p]))
        assert e <= 1e-12, (p, e)
        worst = max(worst, e)
        smax = max(smax, oracle.max_signal(batch.patch_out(o, p), G, periodic=True) / batch.dx[p])
    say(f"ppm amr batch {lim}: worst patch parity {worst:.3e}")
    want = 0.4 / smax
    assert abs(float(host(dt_next)[0]) - want) <= 1e-14 * want


@pytest.mark.parametrize("lim", ["ppm", "ppm_ct"])
def test_turbulent_box_256_sampled_cells(gd, lim):
    """The PPM workload at full size: one step of the 256^3 periodic box;
    400 sampled cells, each compared with the oracle's step of the 7^3 block
    around it (ng = 3, wrapped), which reads exactly the cell's stencil."""
    import torch
    n = 256
    u = inputs.turbulent_box(n)
    dx = 1 / n
    dt = oracle.cfl_dt(u, G, dx, 0.5, periodic=True)
    say("ppm 256^3", lim)
    out, _ = gd.step(dev(u), G, dx, dt, periodic=True, limiter=lim, want_bflux=False)
    got = host(out)
    rng = np.random.default_rng(9)
    cells = rng.integers(0, n, size=(400, 3))
    cells[:8] = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 5], [n - 1, 0, 7],
                 [3, 0, n - 1], [1, 1, 1], [n - 2, 2, 128], [128, 128, 128]]
    scale = np.abs(got).reshape(5, -1).max(axis=1)
    worst = 0.0
    for x, y, z in cells:
        idx = [np.arange(c - 3, c + 4) % n for c in (z, y, x)]
        blk = u[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]
        ref, _, _ = oracle.step(blk, G, dx, dt, ng=3, limiter=lim)
        worst = max(worst, float(np.max(np.abs(got[:, z, y, x] - ref[:, 0, 0, 0]) / scale)))
    assert worst <= 1e-12, worst


@pytest.mark.parametrize("lim", ALL)
def test_ghost_cells_the_stencil_never_reads(gd, lim):
    """A ghosted patch's corner ghosts and its edge ghosts deeper than (1, 2)
    are never read: given a negative density (which any conversion of them
    would count as a floor hit) and a NaN energy (which any use of them would
    carry into the output), they leave the step's output, its boundary fluxes
    and the floor count exactly as with finite values. The
    one-launch single-patch path has interior, ring and halo columns that
    reach three cells past a tile, so this checks that its halo and ring
    windows stop where the reconstruction stops."""
    nx, ny, nz, ng = 30, 11, 19, 3
    u = inputs.random_patch(nx, ny, nz, ng=ng, seed=77, generic=True)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, 0.4, ng=ng)
    # depth outside the interior along each axis, per ghosted index
    def depth(n):
        i = np.arange(n + 2 * ng) - ng
        return np.where(i < 0, -i, np.where(i >= n, i - n + 1, 0))
    dz, dy, dx_ = np.meshgrid(depth(nz), depth(ny), depth(nx), indexing="ij")
    nout = (dz > 0).astype(int) + (dy > 0) + (dx_ > 0)
    d = np.stack([dz, dy, dx_])
    edge = nout == 2
    # read: faces to depth 3, edges with depths (1, <= 2)
    edge_read = edge & (np.sort(np.where(d > 0, d, 99), axis=0)[0] == 1) & \
        (np.sort(np.where(d > 0, d, 0), axis=0)[2] <= 2)
    never = (nout == 3) | (edge & ~edge_read)
    assert never.sum() > 0
    bad = u.copy()
    bad[0][never] = -1.0
    bad[4][never] = np.nan
    ctx = gd.context()
    say("ppm unread ghosts", lim)
    ctx.reset_stats()
    a, fa = gd.step(dev(u), G, dx, dt, ng=ng, limiter=lim)
    ha = ctx.floor_hits()
    ctx.reset_stats()
    b, fb = gd.step(dev(bad), G, dx, dt, ng=ng, limiter=lim)
    hb = ctx.floor_hits()
    assert np.array_equal(host(a), host(b))
    assert np.array_equal(host(fa), host(fb))
    assert ha == hb
