"""Shared test utilities (no method arithmetic)."""
import numpy as np


def rel_norm_err(a, b, nvar=5):
    """Parity norm: per variable max |a-b| / max |b|, maximised over variables
    (arrays hold nvar variables, variable-major)."""
    a = np.asarray(a, dtype=np.float64).reshape(nvar, -1)
    b = np.asarray(b, dtype=np.float64).reshape(nvar, -1)
    den = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return float((np.abs(a - b).max(axis=1) / den).max())


def say(*args):
    """Name the case before a GPU step, flushed, so a crash log shows it."""
    print(*args, flush=True)
