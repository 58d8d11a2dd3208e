"""Seeded synthetic magnetization states.

This module holds input generators only -- no stray-field arithmetic -- so
that the product path and the CPU oracle can be fed the very same arrays.
Every generator returns a float64 numpy array in SoA layout [3][nz][ny][nx].

Cell centres: x_i = (i + 1/2 - nx/2) dx (and likewise y, z), i.e. the body is
centred at the origin, as the paper places its cube (Sec. 5.2).
"""
from __future__ import annotations

import numpy as np


def cell_centres(shape, cell):
    nx, ny, nz = shape
    dx, dy, dz = cell
    x = (np.arange(nx) + 0.5 - nx / 2.0) * dx
    y = (np.arange(ny) + 0.5 - ny / 2.0) * dy
    z = (np.arange(nz) + 0.5 - nz / 2.0) * dz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def _normalise(m):
    n = np.sqrt(np.sum(m * m, axis=0, keepdims=True))
    return m / n


def random_unit(shape, seed):
    """i.i.d. directions uniform on the unit sphere (normalised Gaussians)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return _normalise(rng.standard_normal((3, nz, ny, nx)))


def uniform(shape, direction=(1.0, 1.0, 1.0)):
    nx, ny, nz = shape
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    m = np.empty((3, nz, ny, nx))
    for c in range(3):
        m[c] = d[c]
    return m


def gaussian_vortex(shape, cell, r0, c=1.0):
    """m = normalise(-y, x, c exp(-r^2/r0^2)), r^2 = x^2 + y^2 (in-plane)."""
    X, Y, _ = cell_centres(shape, cell)
    r2 = X * X + Y * Y
    return _normalise(np.stack([-Y, X, c * np.exp(-r2 / (r0 * r0))]))


def flower_xyl(shape, cell, L=None):
    """m = normalise(x, y, L), L defaulting to the half-width nx dx / 2."""
    X, Y, _ = cell_centres(shape, cell)
    if L is None:
        L = shape[0] * cell[0] / 2.0
    return _normalise(np.stack([X, Y, np.full_like(X, L)]))


def paper_flower(shape, cell, a=1.0, b=2.0, c=1.0):
    """Flower state of Sec. 5.2, eq. (flower_mag), normalised:
    m ~ (xz/a, yz/c + y^3 z^3 / b^3, 1), body centred at the origin."""
    X, Y, Z = cell_centres(shape, cell)
    m = np.stack([X * Z / a, Y * Z / c + (Y ** 3) * (Z ** 3) / b ** 3, np.ones_like(X)])
    return _normalise(m)


def paper_vortex(shape, cell, rc=0.14):
    """Vortex of Sec. 5.2, eq. (config1) (Feldtkeller profile), axis along z:
    m = (-y/r s, x/r s, exp(-2 r^2/rc^2)), s = sqrt(1 - exp(-4 r^2/rc^2))."""
    X, Y, _ = cell_centres(shape, cell)
    r2 = X * X + Y * Y
    r = np.sqrt(r2)
    s = np.sqrt(1.0 - np.exp(-4.0 * r2 / (rc * rc)))
    with np.errstate(invalid="ignore", divide="ignore"):
        mx = np.where(r > 0, -Y / r * s, 0.0)
        my = np.where(r > 0, X / r * s, 0.0)
    mz = np.exp(-2.0 * r2 / (rc * rc))
    return np.stack([mx, my, mz])


def noisy_strip(shape, seed, base=(1.0, 0.1, 0.0), sigma=0.2):
    """normalise(base + sigma * xi), xi i.i.d. standard normal per component."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    m = np.asarray(base, dtype=np.float64).reshape(3, 1, 1, 1) + sigma * rng.standard_normal((3, nz, ny, nx))
    return _normalise(m)


def sample_targets(shape, count, seed):
    """Seeded flat target indices: `count` random cells, the 8 corners and the
    column through the centre (all z at the central x, y), sorted, unique."""
    nx, ny, nz = shape
    N = nx * ny * nz
    rng = np.random.default_rng(seed)
    t = set(int(v) for v in rng.integers(0, N, size=min(count, N)))
    for z in (0, nz - 1):
        for y in (0, ny - 1):
            for x in (0, nx - 1):
                t.add((z * ny + y) * nx + x)
    cx, cy = nx // 2, ny // 2
    for z in range(nz):
        t.add((z * ny + cy) * nx + cx)
    return np.array(sorted(t), dtype=np.int64)


def lowrank(shape, fmt, rank, seed, smooth=False):
    """Seeded compressed magnetization for the low-rank tensor-grid calls.

    Returns (core, factors): core [3][r][r][r] (Tucker, fmt 0; indexed
    [p][s3][s2][s1]) or [3][r] (CP, fmt 1); factors a list of three arrays
    (3, r, n_q), factor s of component p along axis q at [p][s].  smooth=True
    takes the first r cosine modes cos(pi s (i + 1/2) / n_q) as factors (a
    smooth state of rank r); otherwise the factors are standard normal.  The
    core / weights are standard normal, scaled by r^(-3/2) (Tucker) or r^(-1/2)
    (CP) so that the expanded components stay of order one."""
    rng = np.random.default_rng(seed)
    r = int(rank)
    factors = []
    for n in shape:
        if smooth:
            i = np.arange(n) + 0.5
            base = np.stack([np.cos(np.pi * s * i / n) for s in range(r)])
            f = np.broadcast_to(base, (3, r, n)).copy()
        else:
            f = rng.standard_normal((3, r, n))
        factors.append(f)
    if fmt == 0:
        core = rng.standard_normal((3, r, r, r)) * r ** -1.5
    else:
        core = rng.standard_normal((3, r)) * r ** -0.5
    return core, factors
