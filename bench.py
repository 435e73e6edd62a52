"""Benchmark of the Godunov hot path on one MI355X.

Workload (one "step"): one unsplit MUSCL-Hancock + HLLC Godunov step
(minmod slopes) of a periodic 256^3 FP64 Euler box with log-normal density
(sigma_ln = 1, k^-11/3 Gaussian random field) and Gaussian random velocities
at rms Mach 2, including the CFL reduction (C = 0.5): each step launch reads
dt from a device scalar and reduces the next dt from the state it writes
(godunov_step_cfl), so a step is one launch and nothing returns to the host.

Prints one JSON line:
  value     Mcell-updates/s of the whole step (step + CFL reduction)
  roofline  the step kernel's algorithmic HBM bytes per launch / its average
            launch time (HIP events on the launch stream) against 8 TB/s;
            traffic = measured HBM bytes per launch from rocprofv3 counters
            (profiles/), or null when the kernel source changed since
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload
  also      the batched AMR workload (4096 ghost-zoned patches 8^3..32^3,
            FP64 and FP32, one persistent launch per step) for the
            plain-vs-batched comparison

  also.adjoint  one adjoint step against one forward step (128^3), and the
            backward pass of a checkpointed 20-step rollout against its forward

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batched]
                       [--no-adjoint] [--no-mhd] [--tile 8x8 --zlen 16] [--calibrate-copy]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GAMMA = 5.0 / 3.0
HBM_PEAK_GBS = 8000.0
METRIC = "Mcell-updates/s per Godunov step (plain vs batched), % HBM roofline; adjoint/fwd"
# the step kernel's own code (its launch interface lives in godunov_internal.h,
# whose other declarations do not change the kernel)
KERNEL_SRC = [os.path.join(ROOT, "paper_1412_0934_amd", "csrc", f)
              for f in ("godunov_kernels.hip", "godunov_tile.h", "godunov_cell.h",
                        "godunov_math.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_periodic256_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "step_kernel_periodic256_valu.txt")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _summary_blocks(path):
    """The "key: value" blocks of a committed counter summary, each opened
    by its tile_config line."""
    if not os.path.exists(path):
        return []
    blocks, cur = [], None
    for line in open(path):
        if ":" not in line or line.startswith("#"):
            continue
        k, v = (x.strip() for x in line.split(":", 1))
        if k == "tile_config":
            cur = {}
            blocks.append(cur)
        if cur is not None:
            cur[k] = v.split("  (")[0].strip()
    return blocks


def _current_block(path, tile_config):
    """The summary block for this tile configuration taken on the current
    kernel source, or None (the figures then describe another kernel)."""
    for b in _summary_blocks(path):
        if (b.get("tile_config") == tile_config and
                b.get("kernel_source_sha256_16") == kernel_source_hash()):
            return b
    return None


def measured_traffic(tile_config):
    """HBM bytes per launch of the step kernel from the committed counter
    summary, if it was taken on the current kernel source and holds a
    measurement for this tile configuration; else None."""
    b = _current_block(TRAFFIC_FILE, tile_config)
    try:
        return float(b["hbm_bytes_per_launch"]) if b else None
    except (KeyError, ValueError):
        return None


def measured_valu(tile_config):
    """VALU wave-instructions per cell and the fraction of SIMD cycles that
    issue VALU work, from the committed counter summary of the current
    kernel source and tile configuration; else None."""
    b = _current_block(VALU_FILE, tile_config)
    if not b:
        return None
    try:
        return {"valu_wave_instructions_per_cell": float(b["valu_wave_instructions_per_cell"]),
                "fp64_valu_wave_instructions_per_cell":
                    float(b["fp64_valu_wave_instructions_per_cell"]),
                "simd_valu_issue_fraction": float(b["simd_valu_issue_fraction"]),
                "source": os.path.relpath(VALU_FILE, ROOT)}
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bench_periodic(torch, gd, steps, warmup, n=256, tile=None, zlen=None):
    from paper_1412_0934_amd import inputs
    log(f"bench: generating the {n}^3 periodic box")
    u0 = inputs.turbulent_box(n, mach=2.0)
    dx = 1.0 / n
    u0_dev = torch.from_numpy(u0).cuda()
    ua = u0_dev.clone()
    ub = torch.empty_like(ua)
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    # One launch per step: the step kernel reads dt from the device scalar and,
    # from the state it writes, reduces the CFL step for the next step into
    # the same scalar; the first dt comes from one cfl_dt call.
    def one_step(src, dst, ev=None):
        if ev is not None:
            ev[0].record(stream)
        gd.step(src, GAMMA, dx, dt_dev=dt, periodic=True, want_bflux=False, out=dst,
                cfl=0.5, dt_next=dt)
        if ev is not None:
            ev[1].record(stream)

    if tile is None:
        log("bench: autotuning the step kernel")
        dt_host = 0.5 * dx / 8.0
        gd.autotune_step(ua, GAMMA, dx, dt_host, periodic=True, out=ub)
    else:
        cfg = gd.get_config(torch.float64)
        cfg.update(shape_single=tile, zlen_single=zlen or 16)
        gd.set_config(torch.float64, **cfg)
    log(f"bench: config {gd.get_config(torch.float64)}")
    log(f"bench: {warmup} warmup steps")
    gd.cfl_dt(ua, GAMMA, dx, 0.5, periodic=True, out=dt)
    for i in range(warmup):
        one_step(ua, ub) if i % 2 == 0 else one_step(ub, ua)
    # restart from the initial state so that every run times the same data
    # (a device copy: no idle gap between the warm-up and the timed steps)
    ua.copy_(u0_dev)
    gd.cfl_dt(ua, GAMMA, dx, 0.5, periodic=True, out=dt)
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
    torch.cuda.synchronize()
    ctx = gd.context()
    ctx.reset_stats()
    log(f"bench: timing {steps} steps")
    t0 = time.perf_counter()
    for i in range(steps):
        if i % 2 == 0:
            one_step(ua, ub, events[i])
        else:
            one_step(ub, ua, events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    floor_hits = ctx.floor_hits()
    per_step = [a.elapsed_time(b) for a, b in events]
    kernel_ms = sum(per_step) / steps
    log("bench: step kernel ms, first 5 / min / median / max: "
        f"{[round(x, 3) for x in per_step[:5]]} / {min(per_step):.3f} / "
        f"{sorted(per_step)[steps // 2]:.3f} / {max(per_step):.3f}")
    cells = n ** 3
    return {
        "cells": cells, "wall_s": wall, "ms_per_step": 1e3 * wall / steps,
        "step_kernel_ms": kernel_ms, "bytes_per_launch": 80.0 * cells, "u0": u0,
        "floor_hits": floor_hits,
    }


def bench_batched(torch, gd, steps, warmup, dtype_name, config=None, plain=True):
    import numpy as np
    from paper_1412_0934_amd import inputs
    log(f"bench: batched AMR workload ({dtype_name})")
    batch = bench_batched.cache
    if batch is None:
        batch = inputs.amr_batch(4096, seed=5)
        bench_batched.cache = batch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    es = 8 if dtype == torch.float64 else 4
    table = gd.patch_table(batch.dims, batch.ng, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 0.0)
    u_in = torch.from_numpy(batch.u_in).to("cuda", dtype)
    out = torch.empty(batch.u_out_size, dtype=dtype, device="cuda")
    flux = torch.empty(batch.flux_size, dtype=dtype, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    gd.cfl_dt_batched(u_in, table, GAMMA, 0.5, out=dt)
    if config is None:
        gd.autotune_batched(u_in, table, GAMMA, out=out, bflux=flux)
    else:
        cfg = gd.get_config(dtype)
        cfg.update(shape_batched=config[0], zpolicy_batched=config[1])
        gd.set_config(dtype, **cfg)
    log(f"bench: batched config {gd.get_config(dtype)}")
    # the batched step writes the batch's next CFL step into a second scalar
    # (the input state is the same every repetition, so dt stays the same)
    dt_next = torch.empty_like(dt)
    for _ in range(warmup):
        gd.step_batched(u_in, table, GAMMA, out=out, bflux=flux, dt_dev=dt, cfl=0.5,
                        dt_next=dt_next)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    stream = torch.cuda.current_stream()
    for i in range(steps):
        ev[i][0].record(stream)
        gd.step_batched(u_in, table, GAMMA, out=out, bflux=flux, dt_dev=dt, cfl=0.5,
                        dt_next=dt_next)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    cells = batch.interior_cells
    # minimal traffic: the cells the stencil reads once, the interior written
    # once, and the boundary-flux sheets written once
    d = batch.dims.astype(np.int64)
    read_cells = (np.prod(d, axis=1) + 4 * (d[:, 0] * d[:, 1] + d[:, 1] * d[:, 2] + d[:, 0] * d[:, 2])
                  + 4 * (d[:, 0] + d[:, 1] + d[:, 2])).sum()
    nbytes = es * (5 * read_cells + 5 * cells + batch.flux_size)
    gbs = nbytes / (ms * 1e-3) / 1e9
    res = {"workload": "4096 ghost-zoned patches 8^3..32^3 (p=.5/.3/.15/.05), ng=2, "
                       "sine background + Mach-3 shock, minmod+HLLC, bflux returned",
           "config": gd.get_config(dtype),
           "dtype": dtype_name, "cells": int(cells), "ms_per_step": ms,
           "mcell_per_s": cells / (ms * 1e-3) / 1e6, "bytes_per_step": int(nbytes),
           "achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    if dtype == torch.float64 and plain:
        res["plain"] = bench_plain(torch, gd, batch, u_in, out, flux, dt, cells, steps)
    return res


def bench_plain(torch, gd, batch, u_in, out, flux, dt, cells, steps):
    """The same batch as 4096 separate godunov_step launches per step: issued
    from the host one by one, and captured once into a HIP graph that is
    replayed (the paper's per-patch GPU calls, against one persistent launch)."""
    import ctypes
    log("bench: plain per-patch launches (eager, then one captured graph)")
    ctx = gd.context()
    o = gd._opts(torch.float64, False, "minmod", "hllc", gd.RHO_FLOOR, gd.P_FLOOR)
    es = 8
    calls = []
    for p in range(batch.npatch):
        nx, ny, nz = (int(v) for v in batch.dims[p])
        calls.append((nx, ny, nz, ctypes.c_void_p(u_in.data_ptr() + es * int(batch.u_in_off[p])),
                      ctypes.c_void_p(out.data_ptr() + es * int(batch.u_out_off[p])),
                      ctypes.c_void_p(flux.data_ptr() + es * int(batch.flux_off[p])),
                      float(batch.dx[p])))
    dtp = ctypes.c_void_p(dt.data_ptr())
    lib, h, ob = ctx.lib, ctx.handle, ctypes.byref(o)

    def issue(stream):
        s = ctypes.c_void_p(stream.cuda_stream)
        for nx, ny, nz, a, b, c, dx in calls:
            r = lib.godunov_step(h, ob, nx, ny, nz, 2, a, b, c, GAMMA, dx, 0.0, dtp, s)
            if r:
                ctx.check(r)

    stream = torch.cuda.current_stream()
    issue(stream)
    torch.cuda.synchronize()
    n_eager = max(2, steps // 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n_eager):
        issue(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / n_eager
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        issue(side)                       # warm the capture stream once
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        issue(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    return {"launches_per_step": batch.npatch,
            "eager_ms_per_step": round(eager_ms, 3),
            "eager_mcell_per_s": cells / (eager_ms * 1e-3) / 1e6,
            "graph_ms_per_step": round(graph_ms, 3),
            "graph_mcell_per_s": cells / (graph_ms * 1e-3) / 1e6}


bench_batched.cache = None


def bench_mhd(torch, gd, steps=10, warmup=2, n=128):
    """Ideal MHD (HLLD + GLM cleaning) on the 128^3 periodic turbulent box
    (log-normal density, rms Mach 1, Gaussian random B at plasma beta 100):
    per step one godunov_step_mhd_cfl, which reads dt and the cleaning speed
    from device scalars and writes the next step's there. Minimal traffic: the
    9 FP64 conserved values read and written once, 144 B per cell."""
    from paper_1412_0934_amd import inputs
    log(f"bench: MHD, {n}^3 turbulent box")
    u0 = inputs.mhd_turbulent_box(n)
    a = torch.from_numpy(u0).cuda()
    b = torch.empty_like(a)
    dx = 1.0 / n
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    ch = torch.empty(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def one(src, dst):
        gd.step_mhd(src, GAMMA, dx, dt_dev=dt, ch_dev=ch, alpha=0.1, out=dst, cfl=0.4,
                    dt_next=dt, ch_next=ch)

    gd.cfl_dt_mhd(a, GAMMA, dx, 0.4, out_dt=dt, out_ch=ch)
    for i in range(warmup):
        one(a, b) if i % 2 == 0 else one(b, a)
    a.copy_(torch.from_numpy(u0))
    gd.cfl_dt_mhd(a, GAMMA, dx, 0.4, out_dt=dt, out_ch=ch)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        one(a, b) if i % 2 == 0 else one(b, a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    last = (b if steps % 2 == 1 else a).cpu().numpy()

    def div_b(u):
        d = 0.0
        for c, ax in ((5, 2), (6, 1), (7, 0)):
            d = d + (np.roll(u[c], -1, axis=ax) - np.roll(u[c], 1, axis=ax)) / (2 * dx)
        return float(np.sqrt(np.mean(d * d)))

    cells = n ** 3
    return {"workload": f"ideal MHD {n}^3 periodic, log-normal density, rms Mach 1, Gaussian "
                        "random B at plasma beta 100, HLLD + GLM cleaning (alpha 0.1), minmod, "
                        "FP64; per step one godunov_step_mhd_cfl (step + the next dt and ch), on the device",
            "ms_per_step": ms, "mcell_per_s": cells / (ms * 1e-3) / 1e6,
            "bytes_per_step": 144 * cells, "achieved_gbs": 144 * cells / (ms * 1e-3) / 1e9,
            "hbm_frac": 144 * cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "div_b_rms_start": div_b(u0), f"div_b_rms_after_{steps}_steps": div_b(last)}



def bench_amr(torch, gd, steps=10, warmup=2, nc=128, nfine=1024, max_size=12):
    """One two-level AMR step (gd_amr_step: ghost fill, periodic coarse step,
    batched fine step with boundary fluxes, refluxing + averaging down) on a
    periodic coarse box with fine patches refined by 2, all FP64; plus the
    time of each stage from its own entry point, so the seams' share shows."""
    import numpy as np
    from paper_1412_0934_amd import inputs
    log(f"bench: two-level AMR, {nc}^3 coarse + up to {nfine} fine patches")
    h = inputs.amr_hierarchy(nc=nc, nfine=nfine, max_size=max_size, seed=21, gamma=GAMMA)
    f = h.fine
    table = gd.amr_patch_table(h.lo, h.n, f.u_in_off, f.u_out_off, f.flux_off)
    plan = gd.AmrPlan((nc,) * 3, h.dx_coarse, table)
    ci = torch.from_numpy(h.coarse).cuda()
    co = torch.empty_like(ci)
    fi = torch.from_numpy(np.nan_to_num(f.u_in)).cuda()
    fo = torch.empty(f.u_out_size, dtype=torch.float64, device="cuda")
    ff = torch.empty(f.flux_size, dtype=torch.float64, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    gd.cfl_dt(ci, GAMMA, h.dx_coarse / 2, 0.5, periodic=True, out=dt)
    fine_table = gd.patch_table(h.n, 2, f.u_in_off, f.u_out_off, f.flux_off, h.dx_coarse / 2, 0.0)
    stream = torch.cuda.current_stream()
    # the fine level's patches (4..24 cells per axis) are smaller than the
    # 4096-patch batch's: tune the batched step on them, as a user of the
    # hierarchy would, and restore the batch's configuration afterwards
    keep = gd.get_config(torch.float64)
    gd.autotune_batched(fi, fine_table, GAMMA, out=fo, bflux=ff)
    fine_config = gd.get_config(torch.float64)
    log(f"bench: AMR fine level config {fine_config}")

    def step():
        plan.step(ci, fi, GAMMA, dt_dev=dt, coarse_out=co, fine_out=fo, fine_flux=ff)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # stage by stage, same work
    stages = {"ghost_fill": lambda: plan.fill_ghosts(ci, fi),
              "coarse_step": lambda: gd.step(ci, GAMMA, h.dx_coarse, dt_dev=dt, periodic=True,
                                             out=co, want_bflux=False),
              "fine_batched_step": lambda: gd.step_batched(fi, fine_table, GAMMA, out=fo, bflux=ff,
                                                           dt_dev=dt),
              "reflux_and_average": lambda: plan.reflux(ci, co, fo, ff, GAMMA, dt_dev=dt)}
    stage_ms = {}
    for name, fn in stages.items():
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        stage_ms[name] = round(a.elapsed_time(b) / steps, 4)
    d = h.n.astype(np.int64)
    fine_cells = int(np.prod(d, axis=1).sum())
    ghosts = int((np.prod(d + 4, axis=1) - np.prod(d, axis=1)).sum())
    cells = nc ** 3 + fine_cells
    fill_bytes = 2 * 5 * 8 * ghosts
    gd.set_config(torch.float64, **keep)
    return {"workload": f"two-level AMR: periodic {nc}^3 coarse box + {len(h.lo)} disjoint fine "
                        f"patches refined by 2 (2..{max_size} coarse cells per axis, {fine_cells} "
                        "fine cells), smooth random Fourier state, minmod + HLLC, FP64, one "
                        "gd_amr_step per step (5 launches, dt on the device)",
            "fine_config": {"shape_batched": fine_config["shape_batched"],
                            "zpolicy_batched": fine_config["zpolicy_batched"]},
            "patches": int(len(h.lo)), "coarse_cells": nc ** 3, "fine_cells": fine_cells,
            "ghost_cells": ghosts, "ms_per_step": round(ms, 4),
            "mcell_per_s": cells / (ms * 1e-3) / 1e6, "stage_ms": stage_ms,
            "seam_share": round((stage_ms["ghost_fill"] + stage_ms["reflux_and_average"]) /
                                sum(stage_ms.values()), 4),
            "ghost_fill_gbs": round(fill_bytes / (stage_ms["ghost_fill"] * 1e-3) / 1e9, 1)}


def bench_ppm(torch, gd, u0, steps=10, warmup=2, limiter="ppm"):
    """The 256^3 periodic box with the PPM reconstruction (limited parabola,
    HLLC): per step one godunov_step_cfl (one launch: the tile march with the
    parabola, the update and the CFL reduction of the new state), dt in a
    device scalar; with the Hancock half step (limiter "ppm") or
    characteristic tracing ("ppm_ct")."""
    n = u0.shape[1]
    log(f"bench: PPM ({limiter}), {n}^3 periodic box")
    dx = 1.0 / n
    a = torch.from_numpy(u0).cuda()
    b = torch.empty_like(a)
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def one(src, dst):
        gd.step(src, GAMMA, dx, dt_dev=dt, periodic=True, limiter=limiter, out=dst,
                want_bflux=False, cfl=0.5, dt_next=dt)

    gd.cfl_dt(a, GAMMA, dx, 0.5, periodic=True, out=dt)
    for i in range(warmup):
        one(a, b) if i % 2 == 0 else one(b, a)
    a.copy_(torch.from_numpy(u0))
    gd.cfl_dt(a, GAMMA, dx, 0.5, periodic=True, out=dt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        one(a, b) if i % 2 == 0 else one(b, a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    cells = n ** 3
    half = "characteristic tracing" if limiter == "ppm_ct" else "Hancock half step"
    return {"workload": f"periodic Euler box {n}^3 FP64 (the turbulent box of the main line), "
                        f"PPM reconstruction (limited parabola) + {half} + HLLC; per step "
                        "one godunov_step_cfl (one launch: reconstruction, update, CFL reduction), "
                        "dt on the device",
            "ms_per_step": round(ms, 4), "mcell_per_s": cells / (ms * 1e-3) / 1e6,
            "bytes_per_step": 80 * cells, "achieved_gbs": 80 * cells / (ms * 1e-3) / 1e9,
            "hbm_frac": 80 * cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def bench_ppm_batched(torch, gd, limiter, steps=10, warmup=2):
    """1024 ghost-zoned patches of 8^3..32^3 (ng = 3) with the PPM
    reconstruction, FP64: per step one godunov_step_batched_cfl (one
    persistent launch and the CFL finish), boundary fluxes returned."""
    import numpy as np
    from paper_1412_0934_amd import inputs
    log(f"bench: PPM ({limiter}) batch of 1024 patches")
    batch = bench_ppm_batched.cache
    if batch is None:
        batch = inputs.amr_batch(1024, seed=5, ng=3)
        bench_ppm_batched.cache = batch
    table = gd.patch_table(batch.dims, 3, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, 0.0)
    u_in = torch.from_numpy(batch.u_in).cuda()
    out = torch.empty(batch.u_out_size, dtype=torch.float64, device="cuda")
    flux = torch.empty(batch.flux_size, dtype=torch.float64, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    gd.cfl_dt_batched(u_in, table, GAMMA, 0.4, out=dt)
    dt_next = torch.empty_like(dt)

    def one():
        gd.step_batched(u_in, table, GAMMA, out=out, bflux=flux, dt_dev=dt, limiter=limiter,
                        cfl=0.4, dt_next=dt_next)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        one()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    cells = batch.interior_cells
    # minimal traffic: the cells the stencils read once (the interior, face
    # ghosts to depth 3, edge ghosts at depths (1, 1), (1, 2) and (2, 1)), the
    # interior written once and the boundary-flux sheets written once
    d = batch.dims.astype(np.int64)
    read_cells = (np.prod(d, axis=1) + 6 * (d[:, 0] * d[:, 1] + d[:, 1] * d[:, 2] + d[:, 0] * d[:, 2])
                  + 12 * (d[:, 0] + d[:, 1] + d[:, 2])).sum()
    nbytes = 8 * (5 * read_cells + 5 * cells + batch.flux_size)
    gbs = nbytes / (ms * 1e-3) / 1e9
    half = "characteristic tracing" if limiter == "ppm_ct" else "Hancock half step"
    return {"workload": "1024 ghost-zoned patches 8^3..32^3 (p=.5/.3/.15/.05), ng=3, FP64, PPM "
                        f"(limited parabola) + {half} + HLLC, bflux returned; one persistent launch",
            "cells": int(cells), "ms_per_step": round(ms, 4),
            "mcell_per_s": cells / (ms * 1e-3) / 1e6, "bytes_per_step": int(nbytes),
            "achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}


bench_ppm_batched.cache = None


def bench_streamed(torch, gd, steps=5, chunks=(64 << 20, 128 << 20, 256 << 20)):
    """The 4096-patch FP64 batch held in pinned host memory: one
    godunov_step_batched_streamed per step (chunks copied in, stepped and
    copied back on three streams, the copies overlapping the steps), against
    the serial path (copy the whole batch in, one resident batched step, copy
    it back) and the host<->device bandwidth of one large copy each way."""
    from paper_1412_0934_amd import inputs
    log("bench: streamed batch (pinned host memory)")
    batch = bench_batched.cache
    if batch is None:
        batch = inputs.amr_batch(4096, seed=5)
        bench_batched.cache = batch
    dt = 1e-4
    table = gd.patch_table(batch.dims, batch.ng, batch.u_in_off, batch.u_out_off, batch.flux_off,
                           batch.dx, dt)
    u_h = torch.from_numpy(batch.u_in).pin_memory()
    out_h = torch.empty(batch.u_out_size, dtype=torch.float64).pin_memory()
    fl_h = torch.empty(batch.flux_size, dtype=torch.float64).pin_memory()
    u_d = torch.empty(len(batch.u_in), dtype=torch.float64, device="cuda")
    out_d = torch.empty(batch.u_out_size, dtype=torch.float64, device="cuda")
    fl_d = torch.empty(batch.flux_size, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    def serial():
        u_d.copy_(u_h, non_blocking=True)
        gd.step_batched(u_d, table, GAMMA, out=out_d, bflux=fl_d)
        out_h.copy_(out_d, non_blocking=True)
        fl_h.copy_(fl_d, non_blocking=True)

    h2d_ms = timed(lambda: u_d.copy_(u_h, non_blocking=True), steps)
    d2h_ms = timed(lambda: out_h.copy_(out_d, non_blocking=True), steps)
    step_ms = timed(lambda: gd.step_batched(u_d, table, GAMMA, out=out_d, bflux=fl_d), steps)
    serial_ms = timed(serial, steps)
    cells = batch.interior_cells
    res = {"workload": "the 4096-patch FP64 batch in pinned host memory, minmod + HLLC, bflux "
                       "returned; per step one godunov_step_batched_streamed",
           "h2d_gbs": round(u_h.numel() * 8 / (h2d_ms * 1e-3) / 1e9, 1),
           "d2h_gbs": round(out_h.numel() * 8 / (d2h_ms * 1e-3) / 1e9, 1),
           "resident_step_ms": round(step_ms, 3),
           "serial_ms_per_step": round(serial_ms, 3),
           "serial_mcell_per_s": cells / (serial_ms * 1e-3) / 1e6,
           "streamed": []}
    for chunk in chunks:
        ms = timed(lambda: gd.step_batched_streamed(u_h, table, GAMMA, out=out_h, bflux=fl_h,
                                                    chunk_bytes=chunk), steps)
        res["streamed"].append({"chunk_bytes": chunk, "ms_per_step": round(ms, 3),
                                "mcell_per_s": cells / (ms * 1e-3) / 1e6,
                                "speedup_over_serial": round(serial_ms / ms, 3)})
    return res


def bench_periodic_f32(torch, gd, u0, steps=10, warmup=2):
    """The 256^3 periodic box in FP32 (the same values rounded once), tile
    configuration autotuned for FP32, one godunov_step_cfl per step. Minimal
    traffic 40 B per cell."""
    n = u0.shape[1]
    log(f"bench: FP32 {n}^3 periodic box")
    dx = 1.0 / n
    a = torch.from_numpy(u0).to("cuda", torch.float32)
    b = torch.empty_like(a)
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    gd.autotune_step(a, GAMMA, dx, 0.5 * dx / 8.0, periodic=True, out=b)
    stream = torch.cuda.current_stream()

    def one(src, dst):
        gd.step(src, GAMMA, dx, dt_dev=dt, periodic=True, want_bflux=False, out=dst, cfl=0.5,
                dt_next=dt)

    gd.cfl_dt(a, GAMMA, dx, 0.5, periodic=True, out=dt)
    for i in range(warmup):
        one(a, b) if i % 2 == 0 else one(b, a)
    a.copy_(torch.from_numpy(u0))
    gd.cfl_dt(a, GAMMA, dx, 0.5, periodic=True, out=dt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        one(a, b) if i % 2 == 0 else one(b, a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    cells = n ** 3
    return {"workload": f"the periodic {n}^3 turbulent box in FP32, minmod + HLLC, one "
                        "godunov_step_cfl per step",
            "config": gd.get_config(torch.float32), "ms_per_step": round(ms, 4),
            "mcell_per_s": cells / (ms * 1e-3) / 1e6, "bytes_per_step": 40 * cells,
            "hbm_frac": 40 * cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def bench_sod32(torch, gd, reps=200):
    """The 32^3 Sod patch (2 ghost layers, outflow ghosts, 1% density noise):
    the latency of one godunov_step call with boundary fluxes -- far below any
    bandwidth limit (3.4 MB), so microseconds per call, not a roofline."""
    import time
    from paper_1412_0934_amd import inputs
    log("bench: 32^3 Sod patch latency")
    u, dx = inputs.sod_patch(32)
    ud = torch.from_numpy(u).cuda()
    out = torch.empty((5, 32, 32, 32), dtype=torch.float64, device="cuda")
    fl = torch.empty(gd.bflux_size(32, 32, 32), dtype=torch.float64, device="cuda")
    dt = gd.cfl_dt(ud, GAMMA, dx, 0.5)
    for _ in range(10):
        gd.step(ud, GAMMA, dx, dt_dev=dt, out=out, bflux=fl)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        gd.step(ud, GAMMA, dx, dt_dev=dt, out=out, bflux=fl)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    return {"workload": "32^3 Sod patch + 2 ghost layers, FP64, minmod + HLLC, boundary fluxes, "
                        "dt on the device; back-to-back godunov_step calls",
            "us_per_call_gpu": round(e0.elapsed_time(e1) * 1e3 / reps, 2),
            "us_per_call_host": round(wall * 1e6, 2),
            "mcell_per_s": 32 ** 3 / (e0.elapsed_time(e1) * 1e-3 / reps) / 1e6}

def bench_adjoint(torch, gd, steps=10, n=128, nsteps=20, every=5):
    """Adjoint cost on the 128^3 smooth periodic box (8 random Fourier modes,
    5% amplitude), fixed dt: one adjoint step against one forward step, and
    the backward pass of a 20-step rollout with checkpoints every 5 steps
    (segments recomputed) against its forward pass."""
    from paper_1412_0934_amd import inputs
    log(f"bench: adjoint, {n}^3 smooth box")
    U0, target = inputs.smooth_box(n)
    u0 = torch.from_numpy(U0).cuda()
    dx = 1.0 / n
    dt = float(gd.cfl_dt(u0, GAMMA, dx, 0.5, periodic=True).item())
    lam = torch.randn_like(u0)
    out = torch.empty_like(u0)
    lin = torch.empty_like(u0)
    stream = torch.cuda.current_stream()

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    # the forward step it is compared with runs in the configuration the
    # autotuner picks for this box
    gd.autotune_step(u0, GAMMA, dx, dt, periodic=True, out=out)
    fwd_cfg = gd.get_config(torch.float64)
    fwd = timed(lambda: gd.step(u0, GAMMA, dx, dt, periodic=True, want_bflux=False, out=out), steps)
    adj = timed(lambda: gd.step_adjoint(u0, lam, GAMMA, dx, dt, periodic=True, out=lin), steps)
    tgt = torch.from_numpy(target).cuda()

    def rollout_fwd():
        return gd.rollout(u0.requires_grad_(True), GAMMA, dx, dt, nsteps, every)

    def loss_of(uT):
        return ((uT[0] - tgt) ** 2).sum()

    # one untimed forward + backward: the first backward pays one-off costs
    # (autograd worker start-up, first launches of torch's elementwise kernels)
    loss_of(rollout_fwd()).backward()
    torch.cuda.synchronize()
    t_fwd = t_bwd = 0.0
    reps = 3
    for _ in range(reps):
        u0.grad = None
        t0 = time.perf_counter()
        uT = rollout_fwd()
        torch.cuda.synchronize()
        t_fwd += time.perf_counter() - t0
        loss = loss_of(uT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t_bwd += time.perf_counter() - t0
    t_fwd /= reps
    t_bwd /= reps
    u0.requires_grad_(False)
    return {"workload": f"{n}^3 periodic smooth box, fixed dt, minmod + HLLC, FP64",
            "forward_step_ms": fwd, "forward_config": f"{fwd_cfg['shape_single']}/"
                                                      f"{fwd_cfg['zlen_single']}",
            "adjoint_step_ms": adj, "adjoint_over_forward": adj / fwd,
            "rollout": f"{nsteps} steps, checkpoint every {every}",
            "rollout_forward_ms": 1e3 * t_fwd, "rollout_backward_ms": 1e3 * t_bwd,
            "rollout_backward_over_forward": t_bwd / t_fwd}


# Ramses hydro solver in one cosmological AMR run (256^3 base mesh, 8 levels),
# whole-run seconds as printed in Sec. 3 (Table 1); the paper gives neither the
# cell count nor the step count, so none converts to Mcell-updates/s.
PAPER_CONTEXT = {
    "source": "Sec. 3, Table 1: Ramses hydro solver (OpenACC) in a cosmological AMR run, "
              "256^3 base mesh + 8 levels, Piz Daint (Cray XC30)",
    "hydro_seconds": {"1 CPU core (Xeon E5-2670)": 56218, "16 CPU cores": 2918,
                      "1 GPU (Tesla K20X)": 3009, "16 GPUs (K20X)": 179},
    "gpu_copy_seconds": {"1 GPU": 739, "16 GPUs": 64},
    "note": "context, not a target: no cell or step counts are given, so no Mcell-updates/s",
}


def cpu_single_thread(u0):
    """One full step (cfl + step) of the oracle on one host thread, in a child
    process started with OMP_NUM_THREADS=1."""
    import subprocess
    import tempfile
    import numpy as np
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "u0.npy")
        np.save(path, u0)
        code = ("import sys, time, numpy as np; sys.path.insert(0, %r); import oracle; "
                "u = np.load(%r); n = u.shape[1]; t0 = time.perf_counter(); "
                "dt = oracle.cfl_dt(u, %r, 1.0 / n, 0.5, periodic=True); "
                "oracle.step(u, %r, 1.0 / n, dt, periodic=True); "
                "print(time.perf_counter() - t0)" % (ROOT, path, GAMMA, GAMMA))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        log("bench: CPU oracle on 1 thread")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                           text=True, timeout=300)
    if r.returncode != 0:
        return None
    el = float(r.stdout.strip().splitlines()[-1])
    n = u0.shape[1]
    return {"value": round(n ** 3 / el / 1e6, 3), "unit": "Mcell-updates/s", "cores": 1,
            "sample": f"1 full step (cfl + step) of the same {n}^3 box, {el:.1f} s"}


def cpu_description():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(u0, budget_s=12.0, max_steps=40):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = u0.shape[1]
    dx = 1.0 / n
    log(f"bench: CPU oracle on {threads} threads")
    u = u0
    steps = 0
    floor_hits = None
    t0 = time.perf_counter()
    while steps < max_steps:
        dt = oracle.cfl_dt(u, GAMMA, dx, 0.5, periodic=True)
        u, _, hits = oracle.step(u, GAMMA, dx, dt, periodic=True)
        if floor_hits is None:
            floor_hits = int(hits)
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": round(steps * n ** 3 / el / 1e6, 3), "unit": "Mcell-updates/s",
            "cores": threads, "kind": "oracle", **cpu_description(),
            "sample": f"{steps} full steps (cfl + step) of the same {n}^3 periodic box, "
                      f"{el:.1f} s",
            "oracle_floor_hits_first_step": floor_hits}


def _in_child(code, threads, timeout=300):
    """Run `code` in a fresh interpreter with OMP_NUM_THREADS = threads and
    return the float it prints last (or None)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=timeout)
    if r.returncode != 0:
        log(r.stderr[-2000:])
        return None
    return float(r.stdout.strip().splitlines()[-1])


_BATCH_CODE = """
import sys, time
import numpy as np
sys.path.insert(0, %r)
import oracle
z = np.load(%r)
u_in, dims, off, dx = z["u_in"], z["dims"], z["u_in_off"], z["dx"]
npatch, g = %d, %r
def patch(p):
    nx, ny, nz = (int(v) for v in dims[p])
    n = 5 * (nz + 4) * (ny + 4) * (nx + 4)
    return u_in[off[p]:off[p] + n].reshape(5, nz + 4, ny + 4, nx + 4)
dt = 0.5 * min(dx[p] / oracle.max_signal(patch(p), g) for p in range(len(dims)))
t0 = time.perf_counter()
for p in range(npatch):
    oracle.step(patch(p), g, dx[p], dt)
print(time.perf_counter() - t0)
"""


def cpu_batched(threads_all):
    """The oracle's step of the 4096-patch batch (its patches one after
    another, each with the oracle's OpenMP loops): the whole batch on all
    host threads, the first 512 patches on one thread."""
    import tempfile
    from paper_1412_0934_amd import inputs
    b = bench_batched.cache or inputs.amr_batch(4096, seed=5)
    cells = np.prod(b.dims, axis=1)
    out = {"workload": "4096 ghost-zoned patches 8^3..32^3, one step (cfl dt, minmod + HLLC, "
                       "bflux)", "unit": "Mcell-updates/s", "kind": "oracle"}
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "batch.npz")
        np.savez(path, u_in=b.u_in, dims=b.dims, u_in_off=b.u_in_off, dx=b.dx)
        for key, threads, npatch in (("all_threads", threads_all, b.npatch),
                                     ("single_thread", 1, 512)):
            log(f"bench: CPU oracle, batched, {npatch} patches on {threads} threads")
            el = _in_child(_BATCH_CODE % (ROOT, path, npatch, GAMMA), threads)
            if el is not None:
                c = int(cells[:npatch].sum())
                out[key] = {"value": round(c / el / 1e6, 3), "cores": threads,
                            "sample": f"{npatch} patches, {c} cells, {el:.2f} s"}
    return out


_GRAD_CODE = """
import sys, time
import numpy as np
sys.path.insert(0, %r)
import oracle
from paper_1412_0934_amd import inputs
n, nsteps, every = %d, 20, 5
U0, target = inputs.smooth_box(n)
dx = 1.0 / n
dt = oracle.cfl_dt(U0, %r, dx, 0.5, periodic=True)
t0 = time.perf_counter()
ckpt, u = [U0], U0
for k in range(nsteps):
    u = oracle.step(u, %r, dx, dt, periodic=True)[0]
    if (k + 1) %% every == 0 and k + 1 < nsteps:
        ckpt.append(u)
lam = np.zeros_like(U0)
lam[0] = 2 * (u[0] - target)
for seg in reversed(range(len(ckpt))):
    states = [ckpt[seg]]
    for _ in range(every - 1):
        states.append(oracle.step(states[-1], %r, dx, dt, periodic=True)[0])
    for s in reversed(states):
        lam = oracle.step_adjoint(s, lam, %r, dx, dt, periodic=True)
print(time.perf_counter() - t0)
"""


def cpu_gradient(threads_all):
    """The oracle's gradient of the 20-step rollout (checkpoints every 5,
    segments recomputed, loss sum (rho_T - rho_target)^2) on the smooth
    periodic box: 64^3 on all host threads, 32^3 on one thread (the GPU
    figure, also.adjoint, is for 128^3: 8 times the cells of 64^3)."""
    out = {"workload": "gradient of a 20-step rollout of the smooth periodic box (checkpoints "
                       "every 5): 20 forward + 16 recomputed + 20 adjoint steps",
           "unit": "s per gradient", "kind": "oracle"}
    for key, threads, n in (("all_threads", threads_all, 64), ("single_thread", 1, 32)):
        log(f"bench: CPU oracle gradient, {n}^3 on {threads} threads")
        el = _in_child(_GRAD_CODE % (ROOT, n, GAMMA, GAMMA, GAMMA, GAMMA), threads)
        if el is not None:
            out[key] = {"value": round(el, 3), "cores": threads, "box": f"{n}^3"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-mhd", action="store_true")
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--no-ppm", action="store_true")
    ap.add_argument("--no-streamed", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--no-sod", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the 4096 separate launches of the batched leg")
    ap.add_argument("--batched-config", default=None,
                    help="SHAPE/POLICY for the batched leg instead of autotuning, e.g. 24x8/2")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (for counter scaling)")
    ap.add_argument("--tile", choices=["16x16", "8x8", "32x8", "16x8", "24x8"], default=None,
                    help="fix the step kernel's tile shape instead of autotuning")
    ap.add_argument("--zlen", type=int, default=None, help="z-range length with --tile")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU; multi-GPU runs are not implemented "
              "(the periodic box would shard as bricks with halo exchange)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU available", file=sys.stderr)
        sys.exit(1)
    from paper_1412_0934_amd import godunov as gd
    gd.context()

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    torch.cuda.synchronize()
    r = bench_periodic(torch, gd, args.steps, args.warmup, tile=args.tile, zlen=args.zlen)
    value = r["cells"] / (r["ms_per_step"] * 1e-3) / 1e6
    achieved = r["bytes_per_launch"] / (r["step_kernel_ms"] * 1e-3) / 1e9
    cfg = gd.get_config(torch.float64)
    traffic = measured_traffic(f"{cfg['shape_single']}/{cfg['zlen_single']}")
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "periodic Euler box 256^3 FP64: log-normal density (sigma_ln=1, "
                        "k^-11/3 GRF), rms Mach 2, p = 0.6 rho/gamma, gamma=5/3; per step one "
                        "godunov_step_cfl launch (step + CFL reduction of the new state, C=0.5, "
                        "dt in a device scalar), minmod + HLLC",
            "cells": r["cells"], "global_batch": 1, "parallelism": "none (1 GPU)",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "step_kernel<double, minmod, HLLC>", "step_kernel_ms": round(r["step_kernel_ms"], 4),
            "tile_config": gd.get_config(torch.float64),
            "algorithmic_bytes_per_launch": r["bytes_per_launch"],
            "valu": measured_valu(f"{cfg['shape_single']}/{cfg['zlen_single']}"),
        },
        "floor_hits_per_step": r["floor_hits"] / args.steps,
    }
    also = {}
    if not args.no_sod:
        also["sod32"] = bench_sod32(torch, gd)
    if not args.no_f32:
        also["periodic_f32"] = bench_periodic_f32(torch, gd, r["u0"])
    if not args.no_batched:
        bcfg = None
        if args.batched_config:
            shape, pol = args.batched_config.split("/")
            bcfg = (shape, int(pol))
        also["batched"] = [bench_batched(torch, gd, max(5, args.steps // 2), 2, "f64", bcfg,
                                         not args.no_plain),
                           bench_batched(torch, gd, max(5, args.steps // 2), 2, "f32", bcfg)]
    if not args.no_mhd:
        also["mhd"] = bench_mhd(torch, gd)
    if not args.no_amr:
        also["amr"] = bench_amr(torch, gd)
    if not args.no_ppm:
        also["ppm"] = bench_ppm(torch, gd, r["u0"])
        also["ppm_ct"] = bench_ppm(torch, gd, r["u0"], limiter="ppm_ct")
        also["ppm_batched"] = [bench_ppm_batched(torch, gd, lim) for lim in ("ppm", "ppm_ct")]
    if not args.no_streamed:
        also["streamed"] = bench_streamed(torch, gd)
    if not args.no_adjoint:
        also["adjoint"] = bench_adjoint(torch, gd)
    if also:
        line["also"] = also
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(r["u0"])
        single = cpu_single_thread(r["u0"])
        if single is not None:
            line["cpu_baseline"]["single_thread"] = single
        threads = line["cpu_baseline"]["cores"]
        line["cpu_baseline"]["batched"] = cpu_batched(threads)
        line["cpu_baseline"]["gradient"] = cpu_gradient(threads)
    line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
