"""The confocal blur kernel rho_z(x, y, t) tabulated on the scan grid (FP64).

Test infrastructure (see the package header).

Paper: the convolutional approximation (Eq. 9) and its 3D extension
(Eq. 11) use a depth-dependent kernel rho_z(x, y, t), obtained as the
measurement of a single point feature (section "Confocal ToF-DOT"); with
the analytic model it is the time-resolved Jacobian of Eq. 5 with source
and detector collocated.  Readings:

* voxel grid == scan grid: same N x N, same pitch, aligned; a voxel at
  lateral offset (dy, dx) grid steps from the scan point sits at
  rho = pitch * sqrt(dy^2 + dx^2), computed from integers so that the
  kernel is exactly symmetric under dy <-> dx and sign changes;
* time bin k is [t0 + k dt, t0 + (k+1) dt), no instrument response;
* K_z[dy, dx, k] = dV * integral over bin k of (Phi0 (*)_t R), with
  dV = pitch^2 * dz the voxel volume (detector area 1 mm^2 implicit);
* the source-to-voxel distance is floored at r_min = (3 dV / 4 pi)^(1/3);
* fluorescence mode (section "Materials and Methods"): the geometry's
  reduced scattering is the excitation one, ``mus_em`` the emission one,
  both share mu_a and n, and ``tau`` is the lifetime (ps, 0 = none); the
  bins are those of Phi0_ex (*) E_tau (*) R_em (``physics.fluorescence_bins``).
"""

from __future__ import annotations

import math

import numpy as np

from . import physics


def voxel_volume(g) -> float:
    return g.pitch_mm * g.pitch_mm * g.dz_mm


def r_min(g) -> float:
    return (3.0 * voxel_volume(g) / (4.0 * math.pi)) ** (1.0 / 3.0)


def optics_of(g) -> physics.Optics:
    return physics.optics(g.mus_prime_per_mm, g.mua_per_mm, g.n_medium)


def time_edges(g) -> np.ndarray:
    return g.t0_ps + g.dt_ps * np.arange(g.nt + 1, dtype=np.float64)


def tabulate(g) -> np.ndarray:
    """Kq[z, dy, dx, k] for 0 <= dy < ny, 0 <= dx < nx (FP64).

    The full kernel on offsets (-(N-1)..N-1)^2 is Kq[z, |dy|, |dx|, k].
    Only the triangle dy <= dx is evaluated; the other half is its mirror
    (identical inputs rho give identical values).
    """
    o = optics_of(g)
    dv = voxel_volume(g)
    rmin = r_min(g)
    te = time_edges(g)
    n_y, n_x = g.ny, g.nx
    out = np.zeros((g.nz, n_y, n_x, g.nt))
    dys, dxs = np.meshgrid(np.arange(n_y), np.arange(n_x), indexing="ij")
    dys = dys.ravel()
    dxs = dxs.ravel()
    key = dys * dys + dxs * dxs
    uniq, inv = np.unique(key, return_inverse=True)
    rho = g.pitch_mm * np.sqrt(uniq.astype(np.float64))
    for iz, z in enumerate(g.z_mm):
        vals = dv * physics.kernel_bins(rho, float(z), te, o, rmin)
        out[iz] = vals[inv].reshape(n_y, n_x, g.nt)
    return out


def fluorescence_entries(g, mus_em: float, tau: float, iz, dy, dx) -> np.ndarray:
    """Fluorescence-mode kernel time curves for (layer, |dy|, |dx|) triples: [n, nt]."""
    ox = optics_of(g)
    om = physics.optics(mus_em, g.mua_per_mm, g.n_medium)
    dv = voxel_volume(g)
    rmin = r_min(g)
    te = time_edges(g)
    iz, dy, dx = np.atleast_1d(iz), np.atleast_1d(dy), np.atleast_1d(dx)
    out = np.zeros((iz.size, g.nt))
    for n in range(iz.size):
        rho = g.pitch_mm * math.sqrt(float(dy[n] * dy[n] + dx[n] * dx[n]))
        out[n] = dv * physics.fluorescence_bins(rho, float(g.z_mm[iz[n]]), te, ox, om, tau, rmin)
    return out


def tabulate_fluorescence(g, mus_em: float, tau: float) -> np.ndarray:
    """Kq[z, dy, dx, k] in fluorescence mode (small grids: adaptive quadrature per bin)."""
    n_y, n_x = g.ny, g.nx
    out = np.zeros((g.nz, n_y, n_x, g.nt))
    seen = {}
    for iz in range(g.nz):
        for dy in range(n_y):
            for dx in range(n_x):
                key = (iz, dy * dy + dx * dx)
                if key not in seen:
                    seen[key] = fluorescence_entries(g, mus_em, tau, iz, dy, dx)[0]
                out[iz, dy, dx] = seen[key]
    return out


def tabulate_entries(g, iz, dy, dx) -> np.ndarray:
    """Kernel time curves for selected (layer, |dy|, |dx|) triples: [n, nt]."""
    o = optics_of(g)
    dv = voxel_volume(g)
    rmin = r_min(g)
    te = time_edges(g)
    iz = np.atleast_1d(iz)
    dy = np.atleast_1d(dy)
    dx = np.atleast_1d(dx)
    out = np.zeros((iz.size, g.nt))
    for n in range(iz.size):
        rho = g.pitch_mm * math.sqrt(float(dy[n] * dy[n] + dx[n] * dx[n]))
        out[n] = dv * physics.kernel_bins(rho, float(g.z_mm[iz[n]]), te, o, rmin)[0]
    return out
