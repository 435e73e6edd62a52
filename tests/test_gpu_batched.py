"""Batched persistent step and batched CFL against the oracle and against the
single-patch entry point, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from helpers import bflux_err, parity_err, say
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


def small_batch(seed=21, npatch=40):
    rng = np.random.default_rng(seed)
    states, dxs = [], []
    for p in range(npatch):
        nx, ny, nz = (int(v) for v in rng.integers(1, 22, size=3))
        dx = float(rng.choice([1 / 64, 1 / 128, 1 / 256]))
        states.append(inputs.random_patch(nx, ny, nz, seed=seed * 1000 + p, dx=dx))
        dxs.append(dx)
    return inputs.pack_batch(states, 2, np.array(dxs), order_seed=seed)


def run_batched(gd, batch, dts, dtype, dt_dev=None, limiter="minmod", riemann="hllc"):
    import torch
    table = gd.patch_table(batch.dims, batch.ng, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dts)
    u_in = torch.from_numpy(batch.u_in).to("cuda", dtype)
    out = torch.full((batch.u_out_size,), float("nan"), dtype=dtype, device="cuda")
    flux = torch.full((batch.flux_size,), float("nan"), dtype=dtype, device="cuda")
    gd.step_batched(u_in, table, G, out=out, bflux=flux, dt_dev=dt_dev, limiter=limiter,
                    riemann=riemann)
    return host(out), host(flux)


def test_batch_with_maximum_extents(gd):
    """Patches 16384 cells long along each axis among small ones: the 16-bit
    tile coordinates of the work items at their last tile."""
    import torch
    dims = [(16384, 1, 1), (3, 4, 5), (1, 16384, 1), (2, 2, 2), (1, 1, 16384), (16384, 2, 3)]
    states = [inputs.random_patch(*d, seed=70 + i) for i, d in enumerate(dims)]
    batch = inputs.pack_batch(states, 2, 1 / 64, order_seed=4)
    dts = np.array([0.4 * oracle.cfl_dt(s, G, 1 / 64) for s in states])
    say("batch with maximum extents")
    out, flux = run_batched(gd, batch, dts, torch.float64)
    for p, u in enumerate(states):
        ref, rflux, _ = oracle.step(u, G, 1 / 64, dts[p])
        assert parity_err(batch.patch_out(out, p), ref) <= 1e-12, p
        assert bflux_err(batch.patch_flux(flux, p), rflux, *batch.dims[p]) <= 1e-12, p


@pytest.mark.parametrize("lim,rs", [("minmod", "hllc"), ("mc", "hll"), ("none", "hllc")])
def test_small_batch_matches_oracle_and_single_patch(gd, lim, rs):
    import torch
    batch = small_batch()
    dts = np.array([0.4 * oracle.cfl_dt(batch.patch_in(p), G, batch.dx[p])
                    for p in range(batch.npatch)])
    say("small batch", lim, rs)
    out, flux = run_batched(gd, batch, dts, torch.float64, limiter=lim, riemann=rs)
    assert np.all(np.isfinite(out)) and np.all(np.isfinite(flux))
    for p in range(batch.npatch):
        u = batch.patch_in(p)
        ref, rflux, _ = oracle.step(u, G, batch.dx[p], dts[p], limiter=lim, riemann=rs)
        assert parity_err(batch.patch_out(out, p), ref) <= 1e-12, p
        assert bflux_err(batch.patch_flux(flux, p), rflux, *batch.dims[p]) <= 1e-12, p
        single, sflux = gd.step(torch.from_numpy(u).cuda(), G, batch.dx[p], dts[p], limiter=lim,
                                riemann=rs)
        assert np.array_equal(batch.patch_out(out, p), host(single)), p
        assert np.array_equal(batch.patch_flux(flux, p), host(sflux)), p


def test_small_batch_fp32(gd):
    import torch
    batch = small_batch(seed=22)
    dts = np.array([0.4 * oracle.cfl_dt(batch.patch_in(p), G, batch.dx[p])
                    for p in range(batch.npatch)])
    say("small batch fp32")
    out, flux = run_batched(gd, batch, dts, torch.float32)
    for p in range(batch.npatch):
        ref, rflux, _ = oracle.step(batch.patch_in(p), G, batch.dx[p], dts[p])
        assert parity_err(batch.patch_out(out, p), ref) <= 1e-5, p
        assert bflux_err(batch.patch_flux(flux, p), rflux, *batch.dims[p]) <= 1e-5, p


def test_batched_cfl_and_device_dt(gd):
    import torch
    batch = small_batch(seed=23)
    ref_dt = oracle.cfl_dt_batched([(batch.patch_in(p), batch.dx[p]) for p in range(batch.npatch)],
                                   G, 0.5)
    table = gd.patch_table(batch.dims, batch.ng, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 0.0)
    u_in = torch.from_numpy(batch.u_in).cuda()
    say("batched cfl")
    dt_dev = gd.cfl_dt_batched(u_in, table, G, 0.5)
    got = float(host(dt_dev)[0])
    assert abs(got - ref_dt) <= 1e-14 * ref_dt
    say("batched with device dt")
    out, _ = run_batched(gd, batch, np.zeros(batch.npatch), torch.float64, dt_dev=dt_dev)
    for p in range(0, batch.npatch, 5):
        ref, _, _ = oracle.step(batch.patch_in(p), G, batch.dx[p], got)
        assert parity_err(batch.patch_out(out, p), ref) <= 1e-12, p


def test_repeated_calls_reuse_tables_and_agree(gd):
    import torch
    batch = small_batch(seed=24, npatch=12)
    dts = np.full(batch.npatch, 1e-4)
    say("repeat 1")
    a, fa = run_batched(gd, batch, dts, torch.float64)
    say("repeat 2")
    b, fb = run_batched(gd, batch, dts, torch.float64)
    assert np.array_equal(a, b) and np.array_equal(fa, fb)


@pytest.fixture(scope="module")
def amr():
    """The 4096-patch batch, its CFL dt, and the oracle's step of every patch
    (outputs and boundary fluxes in the batch's flat layouts)."""
    batch = inputs.amr_batch(4096, seed=5)
    dt = 0.5 * min(batch.dx[p] / oracle.max_signal(batch.patch_in(p), G)
                   for p in range(batch.npatch))
    say("amr batch: oracle step of every patch")
    ref_out = np.empty(batch.u_out_size)
    ref_flux = np.empty(batch.flux_size)
    for p in range(batch.npatch):
        o, f, _ = oracle.step(batch.patch_in(p), G, batch.dx[p], dt)
        batch.patch_out(ref_out, p)[...] = o
        batch.patch_flux(ref_flux, p)[...] = f
    return batch, dt, ref_out, ref_flux


def check_every_patch(batch, out, flux, ref_out, ref_flux, tol):
    worst = 0.0
    for p in range(batch.npatch):
        e = max(parity_err(batch.patch_out(out, p), batch.patch_out(ref_out, p)),
                bflux_err(batch.patch_flux(flux, p), batch.patch_flux(ref_flux, p), *batch.dims[p]))
        assert e <= tol, (p, e)
        worst = max(worst, e)
    return worst


def check_telescoping(batch, out, flux, dt):
    for p in range(batch.npatch):
        nx, ny, nz = (int(v) for v in batch.dims[p])
        sh = oracle.split_bflux(batch.patch_flux(flux, p), nx, ny, nz)
        before = batch.patch_in(p)[:, 2:-2, 2:-2, 2:-2]
        after = batch.patch_out(out, p)
        for v in (0, 4):
            lhs = math.fsum(after[v].ravel()) - math.fsum(before[v].ravel())
            net = sum(math.fsum(sh[s][v].ravel()) * sg for s, sg in
                      (("x+", 1), ("x-", -1), ("y+", 1), ("y-", -1), ("z+", 1), ("z-", -1)))
            scale = math.fsum(np.abs(before[v]).ravel())
            assert abs(lhs + dt / batch.dx[p] * net) <= 1e-12 * scale, (p, v)


@pytest.mark.parametrize("dtype_name,shape,policy", [
    ("f64", "16x16", 1), ("f64", "16x8", 2), ("f64", "24x8", 2), ("f64", "16x8+24x8", 2),
    ("f32", "16x16", 1), ("f32", "24x8", 2), ("f32", "16x8", 2), ("f32", "16x8+24x8", 2)])
def test_full_amr_batch(gd, amr, dtype_name, shape, policy):
    """4096 patches 8^3..32^3 in one persistent launch, in the default
    configuration and in the ones the autotuner picks for this batch on one
    MI355X (FP64: 16x8 tiles, FP32: the 16x8 + 24x8 pair, whole-patch
    z-ranges, which the benchmark times), every patch against the oracle
    element by element, and (FP64) the boundary-flux telescoping identity on
    every patch."""
    import torch
    batch, dt, ref_out, ref_flux = amr
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    tol = 1e-12 if dtype_name == "f64" else 1e-5
    say("amr batch", dtype_name, shape, policy)
    try:
        gd.set_config(dtype, shape_batched=shape, zpolicy_batched=policy)
        out, flux = run_batched(gd, batch, np.full(batch.npatch, dt), dtype)
    finally:
        gd.set_config(dtype)
    assert np.all(np.isfinite(out)) and np.all(np.isfinite(flux))
    worst = check_every_patch(batch, out, flux, ref_out, ref_flux, tol)
    say(f"amr batch {dtype_name} {shape}/{policy}: worst patch parity {worst:.3e}")
    if dtype_name == "f64":
        check_telescoping(batch, out, flux, dt)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_full_amr_batch_in_the_autotuned_configuration(gd, amr, dtype_name):
    """Whatever configuration the autotuner picks on this machine (as the
    benchmark does before timing): every patch against the oracle."""
    import torch
    batch, dt, ref_out, ref_flux = amr
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    tol = 1e-12 if dtype_name == "f64" else 1e-5
    table = gd.patch_table(batch.dims, batch.ng, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    u_in = torch.from_numpy(batch.u_in).to("cuda", dtype)
    out = torch.full((batch.u_out_size,), float("nan"), dtype=dtype, device="cuda")
    flux = torch.full((batch.flux_size,), float("nan"), dtype=dtype, device="cuda")
    try:
        say("amr batch autotune", dtype_name)
        gd.autotune_batched(u_in, table, G, out=out, bflux=flux)
        say("amr batch autotuned config", gd.get_config(dtype))
        out.fill_(float("nan"))
        flux.fill_(float("nan"))
        gd.step_batched(u_in, table, G, out=out, bflux=flux)
        o, f = host(out), host(flux)
    finally:
        gd.set_config(dtype)
    worst = check_every_patch(batch, o, f, ref_out, ref_flux, tol)
    say(f"amr batch {dtype_name} autotuned: worst patch parity {worst:.3e}")


@pytest.mark.parametrize("shape", ["16x16", "16x8+24x8"])
def test_fused_cfl_batched_step(gd, shape):
    """godunov_step_batched_cfl writes the same states as the plain batched
    step and dt_next = min over patches of C dx_p / s_p of the new states,
    with one tile shape and with the per-patch pair."""
    import torch
    batch = small_batch(seed=25)
    table = gd.patch_table(batch.dims, batch.ng, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 0.0)
    u_in = torch.from_numpy(batch.u_in).cuda()
    dt = gd.cfl_dt_batched(u_in, table, G, 0.5)
    out1 = torch.empty(batch.u_out_size, dtype=torch.float64, device="cuda")
    out2 = torch.empty_like(out1)
    nxt = torch.empty(1, dtype=torch.float64, device="cuda")
    try:
        gd.set_config(torch.float64, shape_batched=shape, zpolicy_batched=2)
        say("fused batched: plain", shape)
        gd.step_batched(u_in, table, G, out=out1, dt_dev=dt)
        say("fused batched: with cfl", shape)
        gd.step_batched(u_in, table, G, out=out2, dt_dev=dt, cfl=0.5, dt_next=nxt)
        o1, o2 = host(out1), host(out2)
    finally:
        gd.set_config(torch.float64)
    assert np.array_equal(o1, o2)
    ref = min(0.5 * batch.dx[p] / oracle.max_signal(batch.patch_out(o1, p), G, periodic=True)
              for p in range(batch.npatch))
    assert abs(float(host(nxt)[0]) - ref) <= 1e-14 * ref
