"""Scan geometries and workload recipes (numbers only, no method arithmetic).

The paper scans a collocated source/detector pair over a square grid
(section "Confocal ToF-DOT"), bins photon arrival times (time bins of
50-200 ps in its examples) and reconstructs absorption perturbations on a
voxel grid aligned with the scan grid (Eqs. 9-11).  Its own scenes and
Monte-Carlo data are not available, so every workload here is synthetic:

* ``tiny``      16x16 scan, 1 mm pitch, 8 layers 2..16 mm, 64 bins of 50 ps
* ``mid``       64x64 scan, 0.5 mm pitch, 32 layers 1..20 mm, 256 bins of 25 ps
* ``precision`` 128x128 scan, 0.5 mm pitch, 64 layers 1..30 mm, 512 bins of 20 ps
                (mu_s' drawn per scan from U[0.8, 1.2]/mm)
* ``batching``  64 scans, N in {32,48,64,96,128}, Nz in {16,32,64} over
                1..20 mm, 256 bins of 25 ps
* ``learned``   64x64, 32 layers 1..20 mm, 256 bins of 25 ps
* ``2d32``      32x32 scan at 1 mm, one plane at 6.5 mm, 256 bins of 25 ps
* ``2d128``     128x128 scan at 0.25 mm, one plane at 6.5 mm, 256 bins

All share mu_a = 0.01/mm and n = 1.4 for the homogeneous background
(section "Transient Light Transport: Forward Model": homogeneous background
plus sparse heterogeneity).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Confocal scan geometry and homogeneous background optics.

    Lateral voxel grid == scan grid (nx x ny points, square pitch, aligned);
    layer centres ``z_mm`` (strictly increasing, > 0) with voxel thickness
    ``dz_mm``; time bin k covers [t0 + k dt, t0 + (k+1) dt) picoseconds.
    """

    nx: int
    ny: int
    pitch_mm: float
    z_mm: Tuple[float, ...]
    dz_mm: float
    nt: int
    dt_ps: float
    t0_ps: float = 0.0
    mus_prime_per_mm: float = 1.0
    mua_per_mm: float = 0.01
    n_medium: float = 1.4

    @property
    def nz(self) -> int:
        return len(self.z_mm)

    def with_optics(self, mus_prime_per_mm: float) -> "Geometry":
        return dataclasses.replace(self, mus_prime_per_mm=float(mus_prime_per_mm))


def even_layers(z_min: float, z_max: float, nz: int) -> Tuple[Tuple[float, ...], float]:
    """Layer centres z_k = z_min + k (z_max - z_min)/(nz - 1) and their spacing."""
    if nz == 1:
        return (float(z_min),), 1.0
    dz = (z_max - z_min) / (nz - 1)
    return tuple(float(z_min + k * dz) for k in range(nz)), float(dz)


def _geom(n: int, pitch: float, z_min: float, z_max: float, nz: int, nt: int,
          dt: float, mus: float = 1.0) -> Geometry:
    z, dz = even_layers(z_min, z_max, nz)
    return Geometry(nx=n, ny=n, pitch_mm=pitch, z_mm=z, dz_mm=dz, nt=nt, dt_ps=dt,
                    mus_prime_per_mm=mus)


# Phantom recipe fields: n_abs (min, max), sphere radius (min, max) mm,
# delta mu_a (min, max) /mm, allowed kinds, peak counts (fixed or log-uniform).
WORKLOADS: Dict[str, dict] = {
    "tiny": dict(
        geometry=_geom(16, 1.0, 2.0, 16.0, 8, 64, 50.0),
        n_abs=(1, 1), radius=(1.5, 1.5), dmua=(0.02, 0.02), kinds=("sphere",),
        peak=(1e5, 1e5), iters=50, precision="fp64"),
    "mid": dict(
        geometry=_geom(64, 0.5, 1.0, 20.0, 32, 256, 25.0),
        n_abs=(1, 3), radius=(0.5, 2.0), dmua=(0.01, 0.05), kinds=("sphere", "bar"),
        peak=(1e4, 1e6), iters=200, precision="fp32"),
    "precision": dict(
        geometry=_geom(128, 0.5, 1.0, 30.0, 64, 512, 20.0),
        mus_range=(0.8, 1.2),
        n_abs=(1, 3), radius=(0.5, 2.0), dmua=(0.01, 0.05), kinds=("sphere", "bar"),
        peak=(1e5, 1e5), iters=200, precision="fp32"),
    "learned": dict(
        geometry=_geom(64, 0.5, 1.0, 20.0, 32, 256, 25.0),
        n_abs=(1, 4), radius=(0.5, 2.0), dmua=(0.01, 0.05), kinds=("sphere", "bar"),
        peak=(1e4, 1e6), iters=200, precision="fp32"),
    # 2D single-plane settings: a 32 x 32 mm field behind 6.5 mm of tissue
    # (mu_s = 9/mm read with anisotropy 0.9 as mu_s' = 0.9/mm), one absorbing
    # plane 0.5 mm thick, 256 bins of 25 ps
    "2d32": dict(
        geometry=Geometry(nx=32, ny=32, pitch_mm=1.0, z_mm=(6.5,), dz_mm=0.5, nt=256, dt_ps=25.0,
                          mus_prime_per_mm=0.9),
        n_abs=(1, 3), radius=(1.0, 3.0), dmua=(0.01, 0.05), kinds=("sphere", "bar"),
        peak=(1e5, 1e5), iters=200, precision="fp32"),
    "2d128": dict(
        geometry=Geometry(nx=128, ny=128, pitch_mm=0.25, z_mm=(6.5,), dz_mm=0.5, nt=256, dt_ps=25.0,
                          mus_prime_per_mm=0.9),
        n_abs=(1, 3), radius=(1.0, 3.0), dmua=(0.01, 0.05), kinds=("sphere", "bar"),
        peak=(1e5, 1e5), iters=200, precision="fp32"),
}

BATCH_SIZES = (32, 48, 64, 96, 128)
BATCH_NZ = (16, 32, 64)


def workload(name: str) -> dict:
    return WORKLOADS[name]


def geometry_for(name: str, seed: int = 0) -> Geometry:
    """The workload's geometry; per-scan optics are drawn from ``seed``."""
    w = WORKLOADS[name]
    g = w["geometry"]
    if "mus_range" in w:
        rng = np.random.Generator(np.random.PCG64(seed))
        lo, hi = w["mus_range"]
        g = g.with_optics(float(rng.uniform(lo, hi)))
    return g


def geometry_with_layers(name: str, nz: int, seed: int = 0) -> Geometry:
    """The workload's geometry with nz layers evenly spaced over the same
    depth range (the layer counts of the batching workload)."""
    g = geometry_for(name, seed)
    z, dz = even_layers(g.z_mm[0], g.z_mm[-1], nz)
    return Geometry(nx=g.nx, ny=g.ny, pitch_mm=g.pitch_mm, z_mm=z, dz_mm=dz, nt=g.nt, dt_ps=g.dt_ps,
                    t0_ps=g.t0_ps, mus_prime_per_mm=g.mus_prime_per_mm, mua_per_mm=g.mua_per_mm,
                    n_medium=g.n_medium)


def batching_scans(n_scans: int = 64, seed: int = 0):
    """The batching workload's list of (geometry, phantom seed, peak) triples.

    Scan sizes and layer counts are drawn once from ``seed``; a shape class
    is a distinct (N, Nz) pair and scans of one class share one geometry.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in range(n_scans):
        n = int(rng.choice(BATCH_SIZES))
        nz = int(rng.choice(BATCH_NZ))
        g = _geom(n, 0.5, 1.0, 20.0, nz, 256, 25.0)
        peak = float(10.0 ** rng.uniform(4.0, 6.0))
        out.append((g, 1000 + s, peak))
    return out


def draw_peak(w: dict, rng: np.random.Generator) -> float:
    lo, hi = w["peak"]
    if lo == hi:
        return float(lo)
    return float(10.0 ** rng.uniform(math.log10(lo), math.log10(hi)))
