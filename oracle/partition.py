"""Gaussian partition into blocks, plain FP64 NumPy: TEST INFRASTRUCTURE ONLY.

Follows Sec. 3.2.2 ("Primitives and Data Division") of the paper:
  1. foreground normalisation: p_hat = 2 (p - p_min) / (p_max - p_min) - 1, so the
     foreground box maps to [-1, 1] per axis;
  2. contraction (Eq. 2): identity where the infinity norm of p_hat is <= 1,
     otherwise (2 - 1/|p_hat|_inf) * p_hat / |p_hat|_inf, so all space lands in
     the open cube (-2, 2)^3;
  3. uniform grid over the contracted cube along x and y (z is not divided):
     block (ix, iy) holds the Gaussians with b_min <= contract(p_hat) < b_max,
     b = -2 + 4 k / n per axis;
  4. the Gaussians are grouped by block, keeping their original order inside a
     block (the block table the level-of-detail selection works on).

Readings of points the paper leaves open (also listed in the design notes):
  * operation order: p_hat_i = (2 (p_i - min_i)) / (max_i - min_i) - 1 and
    c_i = (2 - 1/n) * (p_hat_i / n) with n = max_i |p_hat_i|, all FP64;
  * the z extent of the foreground box is the min and max z of all Gaussians;
  * an axis whose printed max is below its min is taken as the interval
    between the two values;
  * block id = iy * nx + ix; the grid index along an axis counts the interior
    boundaries -2 + 4 k / n (k = 1 .. n-1) that are <= the contracted coordinate,
    so a coordinate that rounds to exactly 2 falls in the last block.
"""
from __future__ import annotations

import numpy as np


def foreground_box(means, xy_min, xy_max):
    """p_min, p_max [3]: the given xy rectangle (ends in either order) and the
    z range of all centres."""
    p = np.asarray(means, np.float64)
    lo = np.array([min(xy_min[0], xy_max[0]), min(xy_min[1], xy_max[1]), float(p[2].min())])
    hi = np.array([max(xy_min[0], xy_max[0]), max(xy_min[1], xy_max[1]), float(p[2].max())])
    return lo, hi


def normalise(means, p_min, p_max):
    p = np.asarray(means, np.float64)
    out = np.empty_like(p)
    for ax in range(3):
        out[ax] = (2.0 * (p[ax] - p_min[ax])) / (p_max[ax] - p_min[ax]) - 1.0
    return out


def contract(p_hat):
    """Eq. 2, per column of p_hat [3, n]."""
    q = np.asarray(p_hat, np.float64)
    n = np.max(np.abs(q), axis=0)
    out = q.copy()
    far = n > 1.0
    s = 2.0 - 1.0 / n[far]
    for ax in range(3):
        out[ax, far] = s * (q[ax, far] / n[far])
    return out


def grid_index(c, n_cells):
    """Number of interior boundaries -2 + 4 k / n_cells (k = 1 .. n_cells-1) <= c."""
    idx = np.zeros(c.shape, np.int64)
    for k in range(1, n_cells):
        idx += (c >= (-2.0 + (4.0 * k) / n_cells)).astype(np.int64)
    return idx


def block_ids(means, p_min, p_max, nx, ny):
    c = contract(normalise(means, p_min, p_max))
    return grid_index(c[1], ny) * nx + grid_index(c[0], nx)


def partition(means, p_min, p_max, nx, ny):
    """(block id per Gaussian, perm, block_off [nx*ny + 1]): perm lists the
    Gaussians block by block, ascending original index inside each block."""
    b = block_ids(means, p_min, p_max, nx, ny)
    perm = np.argsort(b, kind="stable").astype(np.int64)
    counts = np.bincount(b, minlength=nx * ny)
    off = np.zeros(nx * ny + 1, np.int64)
    off[1:] = np.cumsum(counts)
    return b, perm, off


def contracted_cells(nx, ny):
    """Cells [nx*ny, 4] (x0, x1, y0, y1) of the grid in contracted coordinates,
    block id iy * nx + ix; the outermost ends are open (-inf / +inf) so the cell
    test gives every point the block grid_index gives it."""
    def edges(n):
        e = [-np.inf] + [-2.0 + (4.0 * k) / n for k in range(1, n)] + [np.inf]
        return e
    ex, ey = edges(nx), edges(ny)
    cells = np.zeros((nx * ny, 4))
    for iy in range(ny):
        for ix in range(nx):
            cells[iy * nx + ix] = (ex[ix], ex[ix + 1], ey[iy], ey[iy + 1])
    return cells
