"""Shared test utilities (no method arithmetic)."""
import numpy as np

# Components of a state measured together as one quantity: mass, momentum (a
# vector), energy; for ideal MHD also the magnetic field (a vector) and psi.
GROUPS = {5: ((0,), (1, 2, 3), (4,)),
          9: ((0,), (1, 2, 3), (4,), (5, 6, 7), (8,))}


def rel_norm_err(a, b, nvar=5):
    """Per variable max |a-b| / max |b|, maximised over variables (arrays hold
    nvar variables, variable-major). The strict form, used by the oracle's
    own pins (symmetries, reductions)."""
    a = np.asarray(a, dtype=np.float64).reshape(nvar, -1)
    b = np.asarray(b, dtype=np.float64).reshape(nvar, -1)
    den = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return float((np.abs(a - b).max(axis=1) / den).max())


def parity_err(a, b, nvar=5):
    """The parity norm of a GPU state against the oracle's: per conserved
    quantity, max |a-b| over its components and cells divided by max |b|
    over the same, maximised over the quantities. Vector quantities
    (momentum, magnetic field) are measured as vectors, so the bound does
    not depend on the orientation of the flow relative to the grid: a
    momentum component that is small throughout a patch carries rounding
    errors of the size of the whole momentum (and of the pressure that acts
    on it), not of itself."""
    a = np.asarray(a, dtype=np.float64).reshape(nvar, -1)
    b = np.asarray(b, dtype=np.float64).reshape(nvar, -1)
    worst = 0.0
    for g in GROUPS[nvar]:
        den = max(float(np.abs(b[list(g)]).max()), 1e-300)
        worst = max(worst, float(np.abs(a[list(g)] - b[list(g)]).max()) / den)
    return worst


def bflux_vars(flat, nx, ny, nz):
    """The boundary-flux buffer (six sheets x-, x+, y-, y+, z-, z+, each
    [5][slow][fast]) as [5][all sheet faces]: one row per flux variable."""
    flat = np.asarray(flat, dtype=np.float64).ravel()
    rows, off = [[] for _ in range(5)], 0
    for n in (nz * ny, nz * ny, nz * nx, nz * nx, ny * nx, ny * nx):
        sheet = flat[off:off + 5 * n].reshape(5, n)
        for v in range(5):
            rows[v].append(sheet[v])
        off += 5 * n
    assert off == flat.size
    return np.stack([np.concatenate(r) for r in rows])


def bflux_err(a, b, nx, ny, nz):
    """Parity of two boundary-flux buffers: max |a-b| over every value of
    every sheet divided by max |b| over the same. The buffer is normed as a
    whole: fluxes of different quantities can vanish on every sheet at once
    (the mass flux out of a patch at rest is rounding noise), so no
    per-variable scale exists for them; the momentum flux carries the
    pressure and sets the scale. The sheets' layout is checked."""
    a = bflux_vars(a, nx, ny, nz)
    b = bflux_vars(b, nx, ny, nz)
    return float(np.abs(a - b).max()) / max(float(np.abs(b).max()), 1e-300)


def say(*args):
    """Name the case before a GPU step, flushed, so a crash log shows it."""
    print(*args, flush=True)
