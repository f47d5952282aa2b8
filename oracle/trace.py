"""Field-line and current-line tracing through the DBIE field (FP64, CPU).

TEST INFRASTRUCTURE (see the package docstring). The paper draws field lines of the reconstructed
field (its AR 11158 figures); the line is the curve whose tangent is B/|B| (or J/|J| for a current
line), here integrated in arc length s by the classical fourth-order Runge-Kutta method:
  k1 = d(x), k2 = d(x + ds/2 k1), k3 = d(x + ds/2 k2), k4 = d(x + ds k3),
  x <- x + ds/6 (k1 + 2 k2 + 2 k3 + k4),
with d the unit direction (times +1 or -1 for the sense along the line).

Readings (the paper gives no tracing scheme): lambda at a stage point comes from trilinear
interpolation of a given lambda grid (clamped to its edges); a line stops, keeping its last point,
when a step would place any of its four stage points outside the box [lo, hi] or the direction is
undefined (|B| or |J| zero or not finite), and after `n_steps` steps.
"""
from __future__ import annotations

import numpy as np

from .dbie_oracle import curl_div, field


def trilinear(grid, origin, spacing, xyz):
    """Trilinear interpolation of grid [C][nz][ny][nx] at points xyz [3, n], clamped to the grid."""
    grid = np.asarray(grid, np.float64)
    C, nz, ny, nx = grid.shape
    out = np.empty((C, xyz.shape[1]))
    idx, frac = [], []
    for d, n in zip(range(3), (nx, ny, nz)):
        t = (xyz[d] - origin[d]) / spacing[d]
        t = np.clip(t, 0.0, n - 1.0)
        i0 = np.minimum(np.floor(t).astype(np.int64), max(n - 2, 0))
        idx.append(i0)
        frac.append(t - i0 if n > 1 else np.zeros_like(t))
    (ix, iy, iz), (fx, fy, fz) = idx, frac
    for c in range(C):
        g = grid[c]

        def at(dz, dy, dx):
            return g[np.minimum(iz + dz, nz - 1), np.minimum(iy + dy, ny - 1), np.minimum(ix + dx, nx - 1)]

        c00 = at(0, 0, 0) * (1 - fx) + at(0, 0, 1) * fx
        c01 = at(0, 1, 0) * (1 - fx) + at(0, 1, 1) * fx
        c10 = at(1, 0, 0) * (1 - fx) + at(1, 0, 1) * fx
        c11 = at(1, 1, 0) * (1 - fx) + at(1, 1, 1) * fx
        out[c] = ((c00 * (1 - fy) + c01 * fy) * (1 - fz) + (c10 * (1 - fy) + c11 * fy) * fz)
    return out


def dbie_direction(B0, x0, y0, h, lam_grid, lam_origin, lam_spacing, current=False):
    """Unit direction of B (or of J = curl B at frozen lambda, Eq. 14) of the nodal DBIE field with
    lambda interpolated from the grid; returns a function xyz [3, n] -> [3, n] (NaN where undefined)."""

    def d(xyz):
        lam = trilinear(lam_grid, lam_origin, lam_spacing, xyz)
        B, dB = field(B0, x0, y0, h, xyz, lam)
        v = curl_div(dB)[0] if current else B
        n = np.sqrt(np.sum(v * v, axis=0))
        with np.errstate(invalid="ignore", divide="ignore"):
            return v / n

    return d


def rk4_trace(direction, seeds, ds, n_steps, lo, hi, sense=1.0):
    """Trace from each seed [3, n]; returns (points [n_steps + 1, 3, n], count [n]): points[k] is the
    k-th point of each line for k < count, NaN after."""
    seeds = np.asarray(seeds, np.float64)
    n = seeds.shape[1]
    lo = np.asarray(lo, np.float64).reshape(3, 1)
    hi = np.asarray(hi, np.float64).reshape(3, 1)
    pts = np.full((n_steps + 1, 3, n), np.nan)
    pts[0] = seeds
    count = np.ones(n, np.int64)
    x = seeds.copy()
    alive = np.ones(n, bool)

    def inside(y):
        return np.all((y >= lo) & (y <= hi), axis=0)

    for k in range(1, n_steps + 1):
        if not alive.any():
            break
        ok = alive & inside(x)
        k1 = sense * direction(x)
        y2 = x + 0.5 * ds * k1
        ok &= inside(y2)
        k2 = sense * direction(np.where(ok, y2, x))
        y3 = x + 0.5 * ds * k2
        ok &= inside(y3)
        k3 = sense * direction(np.where(ok, y3, x))
        y4 = x + ds * k3
        ok &= inside(y4)
        k4 = sense * direction(np.where(ok, y4, x))
        xn = x + ds / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        ok &= np.all(np.isfinite(xn), axis=0)
        alive = ok
        x = np.where(alive, xn, x)
        pts[k][:, alive] = x[:, alive]
        count[alive] += 1
    return pts, count
