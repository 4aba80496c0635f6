"""Shared test helpers.  The oracle side of every comparison is computed from
the seeded layout by the oracle's own encoding (never from GPU output)."""

import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def oracle_view(ora, x, v, rho, rho0, grid_tuple, lo, hi):
    """FP64 state the device holds after encoding (x, v, rho): positions
    quantised to (cell, FP32 offset), velocity and rho - rho0 rounded to FP32.
    Returns (x, v, rho, excl, cidx, off)."""
    org, cell, nc = grid_tuple
    cidx, off = ora.encode(x, org, cell, nc, lo, hi)
    xq = ora.decode(cidx, off, org, cell, nc)
    excl = (cidx == ora.EXCLUDED).astype(np.uint8)
    xq[excl == 1] = np.asarray(x)[excl == 1]
    vq = np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)
    rq = (np.asarray(rho, dtype=np.float64) - rho0).astype(np.float32).astype(np.float64) + rho0
    return xq, vq, rq, excl, cidx, off


def grid_tuple(sim):
    return (np.array(list(sim.grid.origin)), float(sim.grid.cell), [int(c) for c in sim.grid.nc])


def compress(lay, factor):
    """Positions pulled toward the domain's lower corner by `factor` (< 1): the
    density rises by factor**-3, so a cell's stencil spans several staging
    tiles and boundary cells hold more targets than are staged in LDS."""
    lay.x = lay.lo + factor * (lay.x - lay.lo)
    return lay
