"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects bad arguments on the host before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "godunov.h")
LIB = os.environ.get("GODUNOV_LIB", os.path.join(ROOT, "paper_1412_0934_amd", "libgodunov.so"))


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libgodunov.so is not built (run __graft_entry__.build())")
    from paper_1412_0934_amd import godunov
    return godunov.load_library(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("godunov_step", "godunov_step_batched", "godunov_step_adjoint", "cfl_dt",
              "gd_create", "gd_destroy", "gd_last_error", "gd_get_stats", "gd_reset_stats"):
        assert n in names


def test_library_exports_every_declared_function(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _opts(**kw):
    from paper_1412_0934_amd import godunov
    o = godunov.gd_opts(0, 0, 0, 0, 1e-10, 1e-10)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _step(lib, opts, nx=4, ny=4, nz=4, ng=2, u_in=0x1000, u_out=0x100000, bflux=None,
          gamma=5 / 3, dx=0.1, dt=0.01):
    return lib.godunov_step(None, ctypes.byref(opts), nx, ny, nz, ng, ctypes.c_void_p(u_in),
                            ctypes.c_void_p(u_out), ctypes.c_void_p(bflux), gamma, dx, dt, None,
                            None)


@pytest.mark.parametrize("case,kw", [
    ("bad dtype", dict(opts=dict(dtype=7))),
    ("bad bc", dict(opts=dict(bc=3))),
    ("bad limiter", dict(opts=dict(limiter=9))),
    ("bad riemann", dict(opts=dict(riemann=5))),
    ("negative floor", dict(opts=dict(rho_floor=-1.0))),
    ("ng < 2", dict(ng=1)),
    ("ng > 64", dict(ng=65)),
    ("extent above 16384", dict(nx=16385)),
    ("z extent above 16384", dict(nz=16385)),
    ("zero extent", dict(nx=0)),
    ("gamma <= 1", dict(gamma=1.0)),
    ("dx <= 0", dict(dx=0.0)),
    ("dt < 0", dict(dt=-1e-3)),
    ("null input", dict(u_in=0)),
    ("aliased output", dict(u_out=0x1000 + 64)),
    ("bflux aliasing", dict(bflux=0x1000)),
])
def test_bad_arguments_are_rejected_before_launch(lib, case, kw):
    opts = _opts(**kw.pop("opts", {}))
    r = _step(lib, opts, **kw)
    assert r == -1, case
    assert lib.gd_last_error(None)


def test_null_context_is_rejected(lib):
    r = _step(lib, _opts())
    assert r == -1
    assert b"ctx" in lib.gd_last_error(None)


def test_batched_rejects_periodic_and_empty(lib):
    from paper_1412_0934_amd import godunov
    o = _opts(bc=1)
    r = lib.godunov_step_batched(None, ctypes.byref(o), 1, None, ctypes.c_void_p(16),
                                 ctypes.c_void_p(1 << 20), None, None, 5 / 3, None)
    assert r == -4
    o = _opts()
    r = lib.godunov_step_batched(None, ctypes.byref(o), 0, None, ctypes.c_void_p(16),
                                 ctypes.c_void_p(1 << 20), None, None, 5 / 3, None)
    assert r == -1


def test_adjoint_rejects_fp32(lib):
    o = _opts(dtype=1)
    r = lib.godunov_step_adjoint(None, ctypes.byref(o), 4, 4, 4, 2, ctypes.c_void_p(16),
                                 ctypes.c_void_p(1 << 20), None, ctypes.c_void_p(1 << 24),
                                 5 / 3, 0.1, 0.01, None)
    assert r == -4


@pytest.mark.parametrize("n,expect", [(600, -4), (400, -1)])
def test_adjoint_rejects_boxes_beyond_32bit_indexing(lib, n, expect):
    """The 20 n^3 doubles of a scratch record array must stay below 2^31
    entries: 600^3 is refused on the host; 400^3 passes that check and stops
    at the NULL context."""
    o = _opts(bc=1)
    r = lib.godunov_step_adjoint(None, ctypes.byref(o), n, n, n, 0, ctypes.c_void_p(1 << 40),
                                 ctypes.c_void_p(2 << 40), None, ctypes.c_void_p(3 << 40),
                                 5 / 3, 0.1, 0.01, None)
    assert r == expect


@pytest.mark.parametrize("case,kw,expect", [
    ("ghosted box", dict(bc=0), -4),
    ("fp32 ok until the context", dict(dtype=1), -1),
    ("bad dx", dict(dx=0.0), -1),
    ("ch <= 0", dict(ch=0.0), -1),
    ("negative alpha", dict(alpha=-1.0), -1),
    ("aliased output", dict(u_out=0x1000 + 8), -1),
])
def test_mhd_step_rejects_bad_arguments(lib, case, kw, expect):
    o = _opts(bc=kw.pop("bc", 1), dtype=kw.pop("dtype", 0))
    a = dict(dx=0.1, ch=1.0, alpha=0.1, u_out=1 << 24)
    a.update(kw)
    r = lib.godunov_step_mhd(None, ctypes.byref(o), 4, 4, 4, ctypes.c_void_p(0x1000),
                             ctypes.c_void_p(a["u_out"]), 5 / 3, a["dx"], 0.01, None, a["ch"],
                             None, a["alpha"], None)
    assert r == expect, case


def test_fused_mhd_step_needs_an_output_and_a_cfl(lib):
    o = _opts(bc=1)
    args = [None, ctypes.byref(o), 4, 4, 4, ctypes.c_void_p(0x1000), ctypes.c_void_p(1 << 24),
            5 / 3, 0.1, 0.01, None, 1.0, None, 0.1]
    assert lib.godunov_step_mhd_cfl(*args, 0.4, None, None, None) == -1
    assert lib.godunov_step_mhd_cfl(*args, 0.0, ctypes.c_void_p(1 << 26), None, None) == -1


def test_cfl_dt_mhd_needs_an_output(lib):
    o = _opts(bc=1)
    r = lib.cfl_dt_mhd(None, ctypes.byref(o), 4, 4, 4, ctypes.c_void_p(0x1000), 5 / 3, 0.1, 0.4,
                       None, None, None)
    assert r == -1


def test_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    r = lib.gd_create(ctypes.byref(h), 0)
    assert r == -2 and not h.value
    assert b"device" in lib.gd_last_error(None)


def _amr_table(rows):
    from paper_1412_0934_amd import godunov
    lo = [r[0] for r in rows]
    n = [r[1] for r in rows]
    return godunov.amr_patch_table(lo, n, 0, 0, [r[2] if len(r) > 2 else 0 for r in rows])


@pytest.mark.parametrize("case,rows,nc,msg", [
    ("odd extent", [((2, 2, 2), (4, 3, 4))], 16, b"even"),
    ("extent below 2", [((2, 2, 2), (0, 4, 4))], 16, b"even"),
    ("outside the box", [((14, 2, 2), (6, 4, 4))], 16, b"inside"),
    ("negative corner", [((-1, 2, 2), (4, 4, 4))], 16, b"inside"),
    ("overlapping patches", [((2, 2, 2), (4, 4, 4)), ((3, 3, 3), (4, 4, 4))], 16, b"overlap"),
    ("no flux sheets", [((2, 2, 2), (4, 4, 4), -1)], 16, b"negative"),
    ("coarse box too large", [], 9000, b"coarse extents"),
    ("valid, stops at the NULL context", [((2, 2, 2), (4, 4, 4)), ((4, 2, 2), (4, 4, 4))], 16,
     b"ctx"),
])
def test_amr_create_validates_the_hierarchy(lib, case, rows, nc, msg):
    t = _amr_table(rows)
    plan = ctypes.c_void_p()
    r = lib.gd_amr_create(None, nc, nc, nc, 1.0 / nc, len(t), t.ctypes.data if len(t) else None,
                          ctypes.byref(plan))
    assert r == -1, case
    assert not plan.value
    assert msg in lib.gd_last_error(None), lib.gd_last_error(None)


def test_amr_calls_reject_a_null_plan(lib):
    o = _opts(bc=1)
    vp = ctypes.c_void_p
    assert lib.gd_amr_fill_ghosts(None, None, 0, vp(16), vp(1 << 20), None) == -1
    assert lib.gd_amr_reflux(None, None, ctypes.byref(o), vp(16), vp(1 << 20), vp(1 << 24),
                             vp(1 << 28), 1.4, 0.01, None, None) == -1
    assert lib.gd_amr_step(None, None, ctypes.byref(o), vp(16), vp(1 << 20), vp(1 << 24),
                           vp(1 << 26), vp(1 << 28), 1.4, 0.01, None, None) == -1
    assert lib.gd_amr_destroy(None) == 0


def test_ppm_options_are_checked(lib):
    """limiters 3 to 6 select the PPM reconstructions (with and without
    characteristic tracing): a ghosted patch needs three ghost layers, limiter
    7 does not exist, and the adjoint and the MHD step refuse PPM
    (GD_E_UNSUPPORTED) before anything else."""
    for lim in (3, 4, 5, 6):
        assert _step(lib, _opts(limiter=lim), ng=2) == -1
        assert b"ng >= 3" in lib.gd_last_error(None)
        assert _step(lib, _opts(limiter=lim), ng=3) == -1    # valid: stops at the NULL ctx
        assert b"ctx" in lib.gd_last_error(None)
    assert _step(lib, _opts(limiter=7), ng=3) == -1
    assert b"limiter" in lib.gd_last_error(None)
    o = _opts(limiter=5, bc=1)
    r = lib.godunov_step_adjoint(None, ctypes.byref(o), 4, 4, 4, 0, ctypes.c_void_p(16),
                                 ctypes.c_void_p(1 << 20), None, ctypes.c_void_p(1 << 24),
                                 5 / 3, 0.1, 0.01, None)
    assert r == -4
    r = lib.godunov_step_mhd(None, ctypes.byref(o), 4, 4, 4, ctypes.c_void_p(0x1000),
                             ctypes.c_void_p(1 << 24), 5 / 3, 0.1, 0.01, None, 1.0, None, 0.1, None)
    assert r == -4


def test_streamed_batch_rejects_bad_arguments(lib):
    from paper_1412_0934_amd import godunov
    t = godunov.patch_table([[4, 4, 4], [6, 5, 4]], 2, [0, 2000], [0, 400], [0, 600], 1 / 64, 1e-3)
    o = _opts()
    vp = ctypes.c_void_p
    args = lambda chunk, out=1 << 24, fl=None: (None, ctypes.byref(o), 2, t.ctypes.data, vp(1 << 20),
                                               vp(out), fl, None, 5 / 3, chunk, None)
    assert lib.godunov_step_batched_streamed(*args(1 << 20)) == -1          # NULL ctx
    assert b"ctx" in lib.gd_last_error(None)
    assert lib.godunov_step_batched_streamed(*args(1024)) == -1
    assert b"chunk_bytes" in lib.gd_last_error(None)
    assert lib.godunov_step_batched_streamed(*args(1 << 20, out=(1 << 20) + 64)) == -1
    assert b"overlaps" in lib.gd_last_error(None)
    o3 = _opts(limiter=3)
    r = lib.godunov_step_batched_streamed(None, ctypes.byref(o3), 2, t.ctypes.data, vp(1 << 20),
                                          vp(1 << 24), None, None, 5 / 3, 1 << 20, None)
    assert r == -4


def _fresh_python(code):
    import subprocess
    import sys
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                          timeout=300)


def test_missing_library_fails_loudly():
    """No fallback: without the built library the binding raises."""
    r = _fresh_python("from paper_1412_0934_amd import godunov\n"
                      "try:\n"
                      "    godunov.load_library('/nonexistent/libgodunov.so')\n"
                      "except RuntimeError as e:\n"
                      "    print('raised:', e)\n")
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "not built" in r.stdout


def test_step_without_a_gpu_raises():
    """On a machine without a GPU the step raises instead of computing on the CPU."""
    r = _fresh_python("import torch, numpy as np\n"
                      "assert not torch.cuda.is_available()\n"
                      "from paper_1412_0934_amd import godunov, inputs\n"
                      "u = torch.from_numpy(inputs.random_patch(4, 4, 4))\n"
                      "try:\n"
                      "    godunov.step(u, 5 / 3, 0.1, 1e-3)\n"
                      "except TypeError as e:\n"
                      "    print('raised:', e)\n"
                      "try:\n"
                      "    godunov.context()\n"
                      "except RuntimeError as e:\n"
                      "    print('raised:', e)\n")
    if "AssertionError" in r.stderr:
        pytest.skip("a GPU is present")
    assert r.returncode == 0, r.stderr
    assert "must be a CUDA tensor" in r.stdout and "no CPU path" in r.stdout


def test_batch_extents_cover_the_packed_layout():
    """The binding's buffer-size check for batched calls: the extents it
    derives from the descriptors equal the packed buffers' sizes, and any
    shorter buffer is refused."""
    import numpy as np
    import torch
    from paper_1412_0934_amd import godunov, inputs
    batch = inputs.batch_layout([(3, 4, 5), (8, 8, 8), (1, 1, 1), (2, 7, 3)], 2, 0.1, order_seed=3)
    t = godunov.patch_table(batch.dims, 2, batch.u_in_off, batch.u_out_off, batch.flux_off,
                            batch.dx)
    assert godunov.batch_extents(t) == (batch.u_in.size, batch.u_out_size, batch.flux_size)
    full = [torch.empty(n) for n in (batch.u_in.size, batch.u_out_size, batch.flux_size)]
    godunov._check_batch(t, *full)
    for i in range(3):
        args = list(full)
        args[i] = args[i][:-1]
        with pytest.raises(ValueError):
            godunov._check_batch(t, *args)
    t["flux_off"] = -1
    assert godunov.batch_extents(t)[2] == 0
    assert godunov.batch_extents(t[:0]) == (0, 0, 0)
    with pytest.raises(ValueError):
        godunov._check_size(torch.empty(3), "x", 0, (4,))
    assert np.all(t["nx"] >= 1)


def test_noalloc_step_checks_its_arguments_on_the_host(lib):
    """The allocation-free batched step rejects bad options, a patch count
    beyond its static scratch and NULL pointers before touching a device."""
    cases = [(_opts(), 0, 1, 1, -1), (_opts(), 65537, 1, 1, -1), (_opts(), 4, 0, 1, -1),
             (_opts(), 4, 1, 0, -1), (_opts(bc=1), 4, 1, 1, -4), (_opts(limiter=3), 4, 1, 1, -4),
             (_opts(limiter=6), 4, 1, 1, -4), (_opts(limiter=7), 4, 1, 1, -1),
             (_opts(dtype=5), 4, 1, 1, -1)]
    for opts, npatch, pd, u, expect in cases:
        r = lib.godunov_step_batched_noalloc(ctypes.byref(opts), npatch, ctypes.c_void_p(pd),
                                             ctypes.c_void_p(u), ctypes.c_void_p(u + 0x10000 if u else 0),
                                             None, None, 5 / 3, None)
        assert r == expect, (npatch, pd, u, r)
        assert lib.gd_last_error(None)
    r = lib.godunov_step_batched_noalloc(None, 4, ctypes.c_void_p(1), ctypes.c_void_p(1),
                                         ctypes.c_void_p(2), None, None, 5 / 3, None)
    assert r == -1
