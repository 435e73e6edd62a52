"""Tiling choices never change results; the autotuner; HIP-graph capture of
the batched step (cfl_dt + godunov_step_batched) replayed several times."""
import numpy as np
import pytest

import oracle
from helpers import parity_err, say
from paper_1412_0934_amd import inputs

pytestmark = pytest.mark.gpu
G = 5.0 / 3.0


@pytest.fixture(scope="module")
def gd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_0934_amd import godunov
    return godunov


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_every_single_patch_configuration_gives_identical_bits(gd, dtype_name):
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    u = torch.from_numpy(inputs.random_patch(37, 29, 45, seed=41)).to("cuda", dtype)
    dt = 1e-3
    results = []
    try:
        for shape in gd.TILE_SHAPES:
            for zlen in (1, 2, 7, 32):
                say("config", shape, zlen, dtype_name)
                gd.set_config(dtype, shape_single=shape, zlen_single=zlen)
                out, flux = gd.step(u, G, 1 / 64, dt)
                results.append((host(out), host(flux)))
    finally:
        gd.set_config(dtype)
    for out, flux in results[1:]:
        assert np.array_equal(out, results[0][0]) and np.array_equal(flux, results[0][1])


def test_z_ranges_on_a_wide_patch_give_identical_bits(gd):
    """A patch wide enough that z-ranges of 3 and 8 planes keep their length
    (a small patch is cut into two-plane ranges whatever the setting); 48
    planes are cut to 16 by the four-workgroups-per-CU rule."""
    import torch
    u = torch.from_numpy(inputs.random_patch(256, 256, 48, seed=43)).to("cuda")
    results = []
    try:
        for shape in ("24x8", "16x16"):
            for zlen in (3, 8, 16, 48):
                say("wide config", shape, zlen)
                gd.set_config(torch.float64, shape_single=shape, zlen_single=zlen)
                out, flux = gd.step(u, G, 1 / 64, 1e-3)
                results.append((host(out), host(flux)))
    finally:
        gd.set_config(torch.float64)
    for out, flux in results[1:]:
        assert np.array_equal(out, results[0][0]) and np.array_equal(flux, results[0][1])


def test_every_batched_configuration_gives_identical_bits(gd):
    import torch
    rng = np.random.default_rng(42)
    states = [inputs.random_patch(*(int(v) for v in rng.integers(3, 30, size=3)), seed=100 + p)
              for p in range(30)]
    batch = inputs.pack_batch(states, 2, 1 / 64, order_seed=3)
    table = gd.patch_table(batch.dims, 2, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 1e-3)
    u_in = torch.from_numpy(batch.u_in).cuda()
    results = []
    try:
        for shape in gd.BATCHED_SHAPES:
            for pol in (0, 1, 2):
                say("batched config", shape, pol)
                gd.set_config(torch.float64, shape_batched=shape, zpolicy_batched=pol)
                out = torch.empty(batch.u_out_size, dtype=torch.float64, device="cuda")
                flux = torch.empty(batch.flux_size, dtype=torch.float64, device="cuda")
                gd.step_batched(u_in, table, G, out=out, bflux=flux)
                results.append((host(out), host(flux)))
    finally:
        gd.set_config(torch.float64)
    for out, flux in results[1:]:
        assert np.array_equal(out, results[0][0]) and np.array_equal(flux, results[0][1])


def test_the_tile_pair_is_a_batched_only_choice(gd):
    """gd_set_config takes the 16x8 + 24x8 pair (index 5) as a batched shape
    only; a single-patch shape 5 or a batched shape 6 is an argument error."""
    import torch
    ctx = gd.context()
    try:
        assert ctx.lib.gd_set_config(ctx.handle, 0, 5, 32, 3, 1) != 0
        assert ctx.lib.gd_set_config(ctx.handle, 0, 3, 32, 6, 1) != 0
        assert ctx.lib.gd_set_config(ctx.handle, 1, 3, 32, 5, 2) == 0
        assert gd.get_config(torch.float32)["shape_batched"] == "16x8+24x8"
    finally:
        gd.set_config(torch.float32)


def test_autotuner_picks_a_configuration_that_keeps_parity(gd):
    import torch
    u = inputs.turbulent_box(64, mach=2.0)
    dx = 1 / 64
    dt = oracle.cfl_dt(u, G, dx, periodic=True)
    ud = torch.from_numpy(u).cuda()
    try:
        say("autotune step")
        choice = gd.autotune_step(ud, G, dx, dt, periodic=True)
        assert 0 <= choice < 15
        say("tuned config", gd.get_config())
        out, _ = gd.step(ud, G, dx, dt, periodic=True)
        ref, _, _ = oracle.step(u, G, dx, dt, periodic=True)
        assert parity_err(host(out), ref) <= 1e-12
    finally:
        gd.set_config(torch.float64)


@pytest.mark.parametrize("dtype_name,shape,pol", [("f64", "16x16", 1), ("f64", "16x8", 2),
                                                   ("f32", "16x8+24x8", 2)])
def test_batched_step_in_a_hip_graph(gd, dtype_name, shape, pol):
    """Capture cfl_dt + godunov_step_batched in a graph; replay it several
    times with eager work and synchronisations between replays, each replay
    checked against the eager result. The default configuration and the two
    the autotuner picks for the AMR batch (16x8 tiles in FP64, the tile pair
    in FP32, whole-patch z-ranges)."""
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    rng = np.random.default_rng(43)
    states = [inputs.random_patch(*(int(v) for v in rng.integers(4, 26, size=3)), seed=200 + p)
              for p in range(40)]
    batch = inputs.pack_batch(states, 2, 1 / 128, order_seed=4)
    table = gd.patch_table(batch.dims, 2, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 0.0)
    u_in = torch.from_numpy(batch.u_in).cuda().to(dtype)
    out = torch.empty(batch.u_out_size, dtype=dtype, device="cuda")
    flux = torch.empty(batch.flux_size, dtype=dtype, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    gd.set_config(dtype, shape_batched=shape, zpolicy_batched=pol)
    try:
        _replay_batched_graph(gd, batch, table, u_in, out, flux, dt, (dtype_name, shape, pol))
    finally:
        gd.set_config(dtype)


def _replay_batched_graph(gd, batch, table, u_in, out, flux, dt, what):
    import torch

    def step():
        gd.cfl_dt_batched(u_in, table, G, 0.5, out=dt)
        gd.step_batched(u_in, table, G, out=out, bflux=flux, dt_dev=dt)

    say("graph: eager reference", *what)
    step()
    ref_out, ref_flux, ref_dt = host(out), host(flux), host(dt)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                      # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("graph: capture", *what)
    with torch.cuda.graph(g):
        step()
    for r in range(4):
        out.fill_(float("nan"))
        flux.fill_(float("nan"))
        dt.fill_(0.0)
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()   # eager work
        torch.cuda.synchronize()
        say("graph: replay", *what, r)
        g.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert np.array_equal(host(dt), ref_dt)
        assert np.array_equal(host(out), ref_out) and np.array_equal(host(flux), ref_flux)
