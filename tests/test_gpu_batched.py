"""Batched persistent step and batched CFL against the oracle and against the
single-patch entry point, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from helpers import rel_norm_err, say
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
        assert rel_norm_err(batch.patch_out(out, p), ref) <= 1e-12, p
        assert rel_norm_err(batch.patch_flux(flux, p), rflux) <= 1e-12, p


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
        assert rel_norm_err(batch.patch_out(out, p), ref) <= 1e-12, p
        assert rel_norm_err(batch.patch_flux(flux, p), rflux) <= 1e-12, p
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
        assert rel_norm_err(batch.patch_out(out, p), ref) <= 1e-5, p
        assert rel_norm_err(batch.patch_flux(flux, p), rflux) <= 1e-5, p


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
        assert rel_norm_err(batch.patch_out(out, p), ref) <= 1e-12, p


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
    return inputs.amr_batch(4096, seed=5)


@pytest.mark.parametrize("dtype_name,shape,policy", [("f64", "16x16", 1), ("f64", "24x8", 2),
                                                     ("f32", "16x16", 1), ("f32", "24x8", 2)])
def test_full_amr_batch(gd, amr, dtype_name, shape, policy):
    """4096 patches 8^3..32^3 in one persistent launch, in the default
    configuration and in the one the autotuner picks for this batch (24x8
    tiles, whole-patch z-ranges): oracle parity on a seeded sample of
    patches, and the boundary-flux telescoping identity on every patch."""
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    tol = 1e-12 if dtype_name == "f64" else 1e-5
    rng = np.random.default_rng(77)
    sample = rng.choice(amr.npatch, size=48, replace=False)
    dt = 0.5 * min(amr.dx[p] / oracle.max_signal(amr.patch_in(p), G) for p in range(amr.npatch))
    say("amr batch", dtype_name, shape, policy)
    try:
        gd.set_config(dtype, shape_batched=shape, zpolicy_batched=policy)
        out, flux = run_batched(gd, amr, np.full(amr.npatch, dt), dtype)
    finally:
        gd.set_config(dtype)
    assert np.all(np.isfinite(out)) and np.all(np.isfinite(flux))
    for p in sample:
        ref, rflux, _ = oracle.step(amr.patch_in(p), G, amr.dx[p], dt)
        assert rel_norm_err(amr.patch_out(out, p), ref) <= tol, p
        assert rel_norm_err(amr.patch_flux(flux, p), rflux) <= tol, p
    if dtype_name == "f32":
        return
    for p in range(amr.npatch):
        nx, ny, nz = (int(v) for v in amr.dims[p])
        sh = oracle.split_bflux(amr.patch_flux(flux, p), nx, ny, nz)
        before = amr.patch_in(p)[:, 2:-2, 2:-2, 2:-2]
        after = amr.patch_out(out, p)
        for v in (0, 4):
            lhs = math.fsum(after[v].ravel()) - math.fsum(before[v].ravel())
            net = sum(math.fsum(sh[s][v].ravel()) * sg for s, sg in
                      (("x+", 1), ("x-", -1), ("y+", 1), ("y-", -1), ("z+", 1), ("z-", -1)))
            scale = math.fsum(np.abs(before[v]).ravel())
            assert abs(lhs + dt / amr.dx[p] * net) <= 1e-12 * scale, (p, v)


def test_fused_cfl_batched_step(gd):
    """godunov_step_batched_cfl writes the same states as the plain batched
    step and dt_next = min over patches of C dx_p / s_p of the new states."""
    import torch
    batch = small_batch(seed=25)
    table = gd.patch_table(batch.dims, batch.ng, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 0.0)
    u_in = torch.from_numpy(batch.u_in).cuda()
    dt = gd.cfl_dt_batched(u_in, table, G, 0.5)
    out1 = torch.empty(batch.u_out_size, dtype=torch.float64, device="cuda")
    out2 = torch.empty_like(out1)
    say("fused batched: plain")
    gd.step_batched(u_in, table, G, out=out1, dt_dev=dt)
    nxt = torch.empty(1, dtype=torch.float64, device="cuda")
    say("fused batched: with cfl")
    gd.step_batched(u_in, table, G, out=out2, dt_dev=dt, cfl=0.5, dt_next=nxt)
    o1, o2 = host(out1), host(out2)
    assert np.array_equal(o1, o2)
    ref = min(0.5 * batch.dx[p] / oracle.max_signal(batch.patch_out(o1, p), G, periodic=True)
              for p in range(batch.npatch))
    assert abs(float(host(nxt)[0]) - ref) <= 1e-14 * ref
