"""How far two valid roundings of the oracle drift apart over a rollout.

The oracle is built twice: as always (x86-64-v2, no fused multiply-add) and
with FMA contraction (-mfma -ffp-contract=fast). Both are correct binary64
evaluations of the same scheme that differ only in rounding. Each runs the
same seeded rollout in a subprocess of its own (the library directory is
fixed at import), and the per-variable parity norm between the two final
states is printed. This is the scale against which a GPU tolerance over
several steps is set: a GPU result may not differ from the oracle by more
than the arithmetic's own rounding can explain.

    python tests/rounding_drift.py mhd 128 10
    python tests/rounding_drift.py euler 256 10
"""
import os
import subprocess
import sys
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
G = 5.0 / 3.0


def _rollout(kind, n, steps, out):
    sys.path.insert(0, ROOT)
    import oracle
    from oracle import mhd
    from paper_1412_0934_amd import inputs
    dx = 1.0 / n
    if kind == "mhd":
        u = inputs.mhd_turbulent_box(n)
        for _ in range(steps):
            dt, ch = mhd.cfl(u, G, dx, 0.4)
            u = mhd.step(u, G, dx, dt, ch, alpha=0.1)[0]
    else:
        u = inputs.turbulent_box(n, mach=2.0)
        for _ in range(steps):
            u = oracle.step(u, G, dx, oracle.cfl_dt(u, G, dx, 0.5, periodic=True),
                            periodic=True)[0]
    np.save(out, u)


def drift(kind, n, steps):
    """Per-variable max |a - b| / max |a| between the two builds' states."""
    sys.path.insert(0, ROOT)
    import oracle
    with tempfile.TemporaryDirectory() as tmp:
        fma_dir = os.path.join(tmp, "fma")
        os.makedirs(fma_dir)
        oracle.build(out_dir=fma_dir, extra_flags=("-mfma", "-ffp-contract=fast"))
        states = []
        for lib_dir in (None, fma_dir):
            env = dict(os.environ)
            if lib_dir:
                env["ORACLE_LIB_DIR"] = lib_dir
            else:
                env.pop("ORACLE_LIB_DIR", None)
            out = os.path.join(tmp, f"state_{len(states)}.npy")
            subprocess.run([sys.executable, os.path.abspath(__file__), "--worker", kind, str(n),
                            str(steps), out], check=True, env=env)
            states.append(np.load(out))
    a, b = states
    nvar = a.shape[0]
    a2, b2 = a.reshape(nvar, -1), b.reshape(nvar, -1)
    per_var = np.abs(a2 - b2).max(axis=1) / np.abs(a2).max(axis=1)
    return per_var, bool(np.array_equal(a, b))


if __name__ == "__main__":
    if sys.argv[1] == "--worker":
        _rollout(sys.argv[2], int(sys.argv[3]), int(sys.argv[4]), sys.argv[5])
    else:
        kind, n, steps = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
        per_var, same = drift(kind, n, steps)
        print(f"{kind} {n}^3, {steps} steps: max drift {per_var.max():.3e} "
              f"(per variable {' '.join(f'{v:.2e}' for v in per_var)}; bitwise equal: {same})")
