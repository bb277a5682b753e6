"""Index bookkeeping shared by the parity tests (no method arithmetic)."""
import numpy as np


def cell_to_ijk(cell, grid):
    nx, ny, _ = grid
    cell = np.asarray(cell, dtype=np.int64)
    return np.stack([cell % nx, (cell // nx) % ny, cell // (nx * ny)], axis=1)


def gpu_xi(cell, off, grid):
    """Grid-unit positions from (cell, offset) pairs."""
    return cell_to_ijk(cell, grid).astype(np.float64) + off


def xi_to_cell_off(xi, grid):
    nx, ny, _ = grid
    f = np.floor(xi)
    cell = (f[:, 0] + nx * (f[:, 1] + ny * f[:, 2])).astype(np.uint32)
    return cell, xi - f


def by_id(ids, *arrays):
    o = np.argsort(ids, kind="stable")
    return (ids[o],) + tuple(a[o] for a in arrays)
