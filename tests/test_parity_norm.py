"""The parity norm used by the GPU tests: boundary-flux buffers split into
sheets and variables as the ABI lays them out, and vector quantities
measured as vectors."""
import numpy as np

import oracle
from helpers import GROUPS, bflux_err, bflux_vars, parity_err, rel_norm_err


def test_bflux_vars_follows_the_sheet_layout():
    nx, ny, nz = 3, 4, 5
    flat = np.arange(oracle.bflux_size(nx, ny, nz), dtype=np.float64)
    rows = bflux_vars(flat, nx, ny, nz)
    sh = oracle.split_bflux(flat, nx, ny, nz)
    for v in range(5):
        want = np.concatenate([sh[s][v].ravel() for s in ("x-", "x+", "y-", "y+", "z-", "z+")])
        assert np.array_equal(rows[v], want)


def test_vectors_are_measured_as_vectors():
    rng = np.random.default_rng(0)
    b = rng.normal(size=(5, 100))
    b[2] *= 1e-3                          # a momentum component small everywhere
    a = b.copy()
    a[2, 7] += 1e-9                       # an error of 1e-9 in it
    assert np.isclose(rel_norm_err(a, b), 1e-9 / np.abs(b[2]).max(), rtol=1e-6)
    assert np.isclose(parity_err(a, b), 1e-9 / np.abs(b[1:4]).max(), rtol=1e-6)
    # a scalar quantity keeps its own scale
    a = b.copy()
    a[0, 3] += 1e-9
    assert np.isclose(parity_err(a, b), 1e-9 / np.abs(b[0]).max(), rtol=1e-6)
    assert GROUPS[9][3] == (5, 6, 7)
    f = rng.normal(size=oracle.bflux_size(2, 3, 4))
    g = f.copy()
    g[0] += 1e-9                          # mass flux of the x- sheet
    rows = bflux_vars(f, 2, 3, 4)
    assert np.isclose(bflux_err(g, f, 2, 3, 4), 1e-9 / np.abs(rows).max(), rtol=1e-6)
