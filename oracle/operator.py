"""Forward model m = sum_z rho_z (*) mu_z and its adjoint (FP64, CPU).

Test infrastructure (see the package header).

Paper: Eq. 2 (m = J mu) restricted to confocal measurements becomes the
lateral convolution of Eq. 9, extended to 3D as the sum over depth layers of
Eq. 11; the solver applies the operator and its transpose repeatedly
(section "Confocal and Multiplexing in ToF-DOT", "Faster forward models").

Readings:
* the convolution is linear (aperiodic): a physical scan window sees only
  voxels inside the same window, so
      m[k, i, j] = sum_z sum_{i', j'} K_z[i - i', j - j', k] mu_z[i', j']
  over the N x N grid; the paper's "doubly circulant" describes the shift
  invariance, and the FFT evaluation below pads to P >= 2N - 1 so that the
  circular product equals this linear sum exactly;
* the adjoint is the transpose
      g_z[i', j'] = sum_k sum_{i, j} K_z[i - i', j - j', k] r[k, i, j].

Layouts: mu, g [nz][ny][nx]; m, r, d [nt][ny][nx]; kernel quadrant
Kq[nz][ny][nx][nt] as returned by ``oracle.kernel.tabulate``.

Tier 0 (``forward_direct``, ``adjoint_direct``, ``jacobian``) is the plain
definition; tier 1 (``FFTOperator``) is the same operator evaluated with
numpy FFTs and is checked against tier 0.
"""

from __future__ import annotations

import numpy as np


def _win(n, d):
    """Output slice and input slice for a shift by d along one axis."""
    return slice(max(0, d), n - max(0, -d)), slice(max(0, -d), n - max(0, d))


def forward_direct(Kq: np.ndarray, mu: np.ndarray) -> np.ndarray:
    nz, n_y, n_x, nt = Kq.shape
    m = np.zeros((nt, n_y, n_x))
    for z in range(nz):
        for dy in range(-(n_y - 1), n_y):
            oy, iy = _win(n_y, dy)
            for dx in range(-(n_x - 1), n_x):
                ox, ix = _win(n_x, dx)
                w = Kq[z, abs(dy), abs(dx), :]
                m[:, oy, ox] += w[:, None, None] * mu[z, iy, ix][None, :, :]
    return m


def adjoint_direct(Kq: np.ndarray, r: np.ndarray) -> np.ndarray:
    nz, n_y, n_x, nt = Kq.shape
    g = np.zeros((nz, n_y, n_x))
    for z in range(nz):
        for dy in range(-(n_y - 1), n_y):
            oy, iy = _win(n_y, dy)
            for dx in range(-(n_x - 1), n_x):
                ox, ix = _win(n_x, dx)
                w = Kq[z, abs(dy), abs(dx), :]
                # g[z, i', j'] += sum_k w[k] r[k, i' + dy, j' + dx]
                g[z, iy, ix] += np.tensordot(w, r[:, oy, ox], axes=(0, 0))
    return g


def jacobian(Kq: np.ndarray) -> np.ndarray:
    """Explicit J[(k, i, j), (z, i', j')] = K_z[i - i', j - j', k] (tiny grids)."""
    nz, n_y, n_x, nt = Kq.shape
    k = np.arange(nt)[:, None, None, None, None, None]
    i = np.arange(n_y)[None, :, None, None, None, None]
    j = np.arange(n_x)[None, None, :, None, None, None]
    z = np.arange(nz)[None, None, None, :, None, None]
    ip = np.arange(n_y)[None, None, None, None, :, None]
    jp = np.arange(n_x)[None, None, None, None, None, :]
    J = Kq[z, np.abs(i - ip), np.abs(j - jp), k]
    return J.reshape(nt * n_y * n_x, nz * n_y * n_x)


def circular_kernel(Kq: np.ndarray, py: int, px: int) -> np.ndarray:
    """Kernel placed on a py x px torus: Kc[z, dy mod py, dx mod px, k]."""
    nz, n_y, n_x, nt = Kq.shape
    if py < 2 * n_y - 1 or px < 2 * n_x - 1:
        raise ValueError("FFT size must be at least 2N - 1 for a linear convolution")
    Kc = np.zeros((nz, py, px, nt))
    for dy in range(-(n_y - 1), n_y):
        for dx in range(-(n_x - 1), n_x):
            Kc[:, dy % py, dx % px, :] = Kq[:, abs(dy), abs(dx), :]
    return Kc


class FFTOperator:
    """Tier-1 evaluation of the same operator with FP64 FFTs (P = 2N)."""

    def __init__(self, Kq: np.ndarray, workers: int | None = None):
        from scipy import fft as sfft
        self._fft = sfft
        self.workers = workers
        nz, n_y, n_x, nt = Kq.shape
        self.shape = (nz, n_y, n_x, nt)
        self.py, self.px = 2 * n_y, 2 * n_x
        Kc = circular_kernel(Kq, self.py, self.px)
        # spectrum of each (z, k) plane: [nz, nt, py, px//2 + 1] complex
        self.Khat = sfft.rfft2(np.moveaxis(Kc, 3, 1), axes=(2, 3), workers=workers)

    def forward(self, mu: np.ndarray) -> np.ndarray:
        nz, n_y, n_x, nt = self.shape
        muh = self._fft.rfft2(mu, s=(self.py, self.px), axes=(1, 2), workers=self.workers)
        mh = np.einsum("zkab,zab->kab", self.Khat, muh, optimize=True)
        m = self._fft.irfft2(mh, s=(self.py, self.px), axes=(1, 2), workers=self.workers)
        return m[:, :n_y, :n_x]

    def adjoint(self, r: np.ndarray) -> np.ndarray:
        nz, n_y, n_x, nt = self.shape
        rh = self._fft.rfft2(r, s=(self.py, self.px), axes=(1, 2), workers=self.workers)
        gh = np.einsum("zkab,kab->zab", np.conj(self.Khat), rh, optimize=True)
        g = self._fft.irfft2(gh, s=(self.py, self.px), axes=(1, 2), workers=self.workers)
        return g[:, :n_y, :n_x]


class DirectOperator:
    """Tier-0 operator object with the same interface as FFTOperator."""

    def __init__(self, Kq: np.ndarray):
        self.Kq = Kq
        nz, n_y, n_x, nt = Kq.shape
        self.shape = (nz, n_y, n_x, nt)

    def forward(self, mu):
        return forward_direct(self.Kq, mu)

    def adjoint(self, r):
        return adjoint_direct(self.Kq, r)
