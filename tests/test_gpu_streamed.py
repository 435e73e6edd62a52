"""Streamed batches (godunov_step_batched_streamed): a batch held in host
memory, stepped chunk by chunk through three device staging slots with the
copies overlapping the steps. Results must be bitwise those of the resident
batched step on the same data -- for chunk sizes from a few patches to the
whole batch, pinned and pageable host memory, FP64 and FP32, device dt, with
and without boundary fluxes, patches in a shuffled memory order -- and match
the oracle; the 4096-patch batch at full size is streamed in 64 MB chunks.
Patches here are at most 19^3 (about 0.85 MB of blocks in FP64), so 1 MB
chunks hold one to a few patches."""
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


def small_batch(n=120, seed=4, order_seed=7):
    rng = np.random.default_rng(seed)
    dims = [tuple(int(v) for v in rng.integers(3, 20, size=3)) for _ in range(n)]
    states = [inputs.random_patch(*d, seed=200 + i) for i, d in enumerate(dims)]
    return inputs.pack_batch(states, 2, 1 / 64, order_seed=order_seed), states


def host_tensor(a, dtype, pinned):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dtype)
    return t.pin_memory() if pinned else t


def resident(gd, batch, table, dtype, dt_dev=None):
    import torch
    out = torch.empty(batch.u_out_size, dtype=dtype, device="cuda")
    fl = torch.empty(batch.flux_size, dtype=dtype, device="cuda")
    gd.step_batched(torch.from_numpy(batch.u_in).to("cuda", dtype), table, G, out=out, bflux=fl,
                    dt_dev=dt_dev)
    torch.cuda.synchronize()
    return out.cpu(), fl.cpu()


def streamed(gd, batch, table, dtype, chunk, pinned, with_flux=True, dt_dev=None):
    import torch
    u = host_tensor(batch.u_in, dtype, pinned)
    out = torch.full((batch.u_out_size,), float("nan"), dtype=dtype)
    fl = torch.full((batch.flux_size,), float("nan"), dtype=dtype) if with_flux else None
    if pinned:
        out = out.pin_memory()
        fl = fl.pin_memory() if fl is not None else None
    gd.step_batched_streamed(u, table, G, out=out, bflux=fl, chunk_bytes=chunk, dt_dev=dt_dev)
    torch.cuda.synchronize()
    return out, fl


@pytest.mark.parametrize("chunk", [1 << 20, 4 << 20, 1 << 30])
@pytest.mark.parametrize("pinned", [True, False])
def test_streamed_equals_resident_fp64(gd, chunk, pinned):
    import torch
    batch, _ = small_batch()
    dt = 2e-4
    table = gd.patch_table(batch.dims, 2, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    ro, rf = resident(gd, batch, table, torch.float64)
    say("streamed fp64", chunk, pinned)
    so, sf = streamed(gd, batch, table, torch.float64, chunk, pinned)
    assert torch.equal(so, ro) and torch.equal(sf, rf)


@pytest.mark.parametrize("shape", ["16x8+24x8", "16x8"])
def test_streamed_in_the_tuned_tile_configurations(gd, shape):
    """The streamed pipeline builds its chunks' work items in the batched
    tile configuration of the context, including the per-patch 16x8 + 24x8
    pair (the one the autotuner picks for FP32): bitwise the resident step."""
    import torch
    batch, _ = small_batch(n=80, seed=9)
    table = gd.patch_table(batch.dims, 2, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 2e-4)
    try:
        for dtype in (torch.float32, torch.float64):
            gd.set_config(dtype, shape_batched=shape, zpolicy_batched=2)
            ro, rf = resident(gd, batch, table, dtype)
            say("streamed", shape, dtype)
            so, sf = streamed(gd, batch, table, dtype, 2 << 20, True)
            assert torch.equal(so, ro) and torch.equal(sf, rf)
    finally:
        gd.set_config(torch.float32)
        gd.set_config(torch.float64)


def test_streamed_fp32_and_device_dt_without_fluxes(gd):
    import torch
    batch, _ = small_batch(seed=5, order_seed=None)
    table = gd.patch_table(batch.dims, 2, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 0.0)
    dt = torch.tensor([3e-4], dtype=torch.float64, device="cuda")
    ro, _ = resident(gd, batch, table, torch.float32, dt_dev=dt)
    say("streamed fp32, device dt, no fluxes")
    so, _ = streamed(gd, batch, table, torch.float32, 1 << 20, True, with_flux=False, dt_dev=dt)
    assert torch.equal(so, ro)


def test_streamed_matches_oracle(gd):
    import torch
    batch, states = small_batch(n=30, seed=6)
    dt = 2e-4
    table = gd.patch_table(batch.dims, 2, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    say("streamed vs oracle")
    so, sf = streamed(gd, batch, table, torch.float64, 1 << 20, True)
    o, f = so.numpy(), sf.numpy()
    for p, s in enumerate(states):
        ref, bref, _ = oracle.step(s, G, 1 / 64, dt)
        assert parity_err(batch.patch_out(o, p), ref) <= 1e-12, p
        assert bflux_err(batch.patch_flux(f, p), bref, *batch.dims[p]) <= 1e-12, p


def test_repeated_and_interleaved_calls(gd):
    import torch
    a, _ = small_batch(n=60, seed=8)
    b, _ = small_batch(n=40, seed=9)
    ta = gd.patch_table(a.dims, 2, a.u_in_off, a.u_out_off, a.flux_off, a.dx, 1e-4)
    tb = gd.patch_table(b.dims, 2, b.u_in_off, b.u_out_off, b.flux_off, b.dx, 1e-4)
    ra, rb = resident(gd, a, ta, torch.float64), resident(gd, b, tb, torch.float64)
    say("streamed repeated / interleaved")
    for _ in range(2):
        for batch, table, ref in ((a, ta, ra), (b, tb, rb)):
            so, sf = streamed(gd, batch, table, torch.float64, 1536 << 10, True)
            assert torch.equal(so, ref[0]) and torch.equal(sf, ref[1])


def test_chunk_smaller_than_a_patch_is_rejected(gd):
    import torch
    batch, _ = small_batch(n=10)
    table = gd.patch_table(batch.dims, 2, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 1e-4)
    with pytest.raises(gd.GodunovError):
        streamed(gd, batch, table, torch.float64, 8 << 10, False)


def test_full_batch_streamed_in_64mb_chunks(gd):
    import torch
    batch = inputs.amr_batch(4096, seed=5)
    dt = 1e-4
    table = gd.patch_table(batch.dims, batch.ng, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    ro, rf = resident(gd, batch, table, torch.float64)
    say("streamed 4096 patches")
    so, sf = streamed(gd, batch, table, torch.float64, 64 << 20, True)
    assert torch.equal(so, ro) and torch.equal(sf, rf)
