"""Seeded absorber phantoms on the confocal voxel grid.

The paper's scenes are discs, lines, pillars and vasculature embedded in a
homogeneous scattering background (section "Additional Image
Reconstructions"); its data are not available, so phantoms here are spheres
and 1 mm x 8 mm bars with a uniform absorption perturbation, voxelised by a
centre-inside test.  Voxel (k, j, i) has its centre at
(x, y, z) = (i * pitch, j * pitch, z_k); arrays are laid out [nz][ny][nx].
Overlapping absorbers add.
"""

from __future__ import annotations

import numpy as np

from .workloads import Geometry


def _sphere(mu, g: Geometry, rng, radius, dmua):
    n_x, n_y = g.nx, g.ny
    p = g.pitch_mm
    z = np.asarray(g.z_mm)
    # centre uniform over [r, (N-1) p - r] laterally, [z_1, z_Nz] in depth
    cx = rng.uniform(radius, max(radius, (n_x - 1) * p - radius))
    cy = rng.uniform(radius, max(radius, (n_y - 1) * p - radius))
    cz = rng.uniform(z[0], z[-1])
    xs = np.arange(n_x) * p
    ys = np.arange(n_y) * p
    d2 = ((z[:, None, None] - cz) ** 2 + (ys[None, :, None] - cy) ** 2
          + (xs[None, None, :] - cx) ** 2)
    inside = d2 <= radius * radius
    if not inside.any():
        # the nearest voxel centre always lies inside for the recipes used;
        # keep the absorber non-empty for any other grid as well
        k, j, i = np.unravel_index(np.argmin(d2), d2.shape)
        inside[k, j, i] = True
    mu[inside] += dmua


def _bar(mu, g: Geometry, rng, dmua, width=1.0, length=8.0):
    n_x, n_y = g.nx, g.ny
    p = g.pitch_mm
    z = np.asarray(g.z_mm)
    along_x = bool(rng.integers(0, 2))
    hx, hy = (length / 2, width / 2) if along_x else (width / 2, length / 2)
    cx = rng.uniform(min(hx, (n_x - 1) * p / 2), max(hx, (n_x - 1) * p - hx))
    cy = rng.uniform(min(hy, (n_y - 1) * p / 2), max(hy, (n_y - 1) * p - hy))
    cz = rng.uniform(z[0], z[-1])
    k = int(np.argmin(np.abs(z - cz)))
    xs = np.arange(n_x) * p
    ys = np.arange(n_y) * p
    inside = (np.abs(xs[None, :] - cx) <= hx) & (np.abs(ys[:, None] - cy) <= hy)
    if not inside.any():
        j = int(np.argmin(np.abs(ys - cy)))
        i = int(np.argmin(np.abs(xs - cx)))
        inside[j, i] = True
    mu[k][inside] += dmua


def phantom(g: Geometry, seed: int, n_abs=(1, 1), radius=(1.5, 1.5),
            dmua=(0.02, 0.02), kinds=("sphere",)) -> np.ndarray:
    """Absorption perturbation delta-mu_a [nz][ny][nx] (FP64, per mm, >= 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = np.zeros((g.nz, g.ny, g.nx), dtype=np.float64)
    count = int(rng.integers(n_abs[0], n_abs[1] + 1))
    for _ in range(count):
        kind = kinds[int(rng.integers(0, len(kinds)))] if len(kinds) > 1 else kinds[0]
        da = float(rng.uniform(dmua[0], dmua[1])) if dmua[0] != dmua[1] else float(dmua[0])
        if kind == "sphere":
            r = float(rng.uniform(radius[0], radius[1])) if radius[0] != radius[1] else float(radius[0])
            _sphere(mu, g, rng, r, da)
        else:
            _bar(mu, g, rng, da)
    return mu


def workload_phantom(w: dict, g: Geometry, seed: int) -> np.ndarray:
    return phantom(g, seed, n_abs=w["n_abs"], radius=w["radius"], dmua=w["dmua"],
                   kinds=w["kinds"])
