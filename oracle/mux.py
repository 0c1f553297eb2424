"""Source multiplexing: y = S m = S J mu (FP64, CPU).

Test infrastructure (see the package header).

Paper: subsection "Multiplexed Confocal ToF-DOT", paragraph "Composite
reconstruction algorithm" (Eq. 12), and section "Advantages of
Multiplexing" (an 8 x 8 array of sources multiplexed with a 64 x 64
Hadamard matrix; Poisson noise at 5 Mcps plus 200 cps of dark counts).
Several sources are on at once and each multiplexed measurement is a linear
combination S of the confocal transients m = J mu, so the reconstruction
fits y = S J mu.  Readings:

* the scan grid (ny rows x nx columns; the paper's is square) is cut into
  tiles of tile_x x tile_y positions (P = tile_x tile_y; the paper's case
  is one 8 x 8 tile); within every tile and time bin the same S (M x P)
  combines the P transients:
      y[t, i, g] = sum_j S[i, j] m[t, y(g, j), x(g, j)]
  with tile g = gy (nx / tile_x) + gx, position j = jy tile_x + jx inside
  it, y(g, j) = gy tile_y + jy, x(g, j) = gx tile_x + jx;
* the objective is Eq. 12 with the squared data term and the regulariser of
  the unmultiplexed solve (the missing weight on the sparsity term is read
  as a typo), so FISTA runs unchanged on the composed operator S J, whose
  adjoint is J^T S^T;
* a +-1 Hadamard matrix cannot be shown by light sources that are either on
  or off; it is realised by the two 0/1 patterns (1 + H)/2 and (1 - H)/2
  (which doubles the number of measurements, as the paper notes), stacked
  as a 2P x P matrix, or by their difference, which is H m itself;
* counting noise with dark counts: a measurement with expected signal
  counts c (S m) gains b expected dark counts per bin, the observation is
  Poisson(c (S m) + b) and the solver receives (counts - b) / c.
"""

from __future__ import annotations

import numpy as np


def sylvester_hadamard(order: int) -> np.ndarray:
    """Hadamard matrix of a power-of-two order by Sylvester's doubling
    H_2k = [[H_k, H_k], [H_k, -H_k]], H_1 = [1]."""
    if order < 1 or order & (order - 1):
        raise ValueError("order must be a power of two")
    h = np.ones((1, 1))
    while h.shape[0] < order:
        h = np.block([[h, h], [h, -h]])
    return h


def two_polarity(h: np.ndarray) -> np.ndarray:
    """The on/off patterns of a +-1 matrix: rows of (1 + H)/2 then (1 - H)/2."""
    h = np.asarray(h, dtype=np.float64)
    return np.vstack([(1.0 + h) / 2.0, (1.0 - h) / 2.0])


def tile_positions(ny: int, tile_x: int, tile_y: int, nx: int | None = None) -> np.ndarray:
    """pos[g, j] = flat scan index y * nx + x of position j of tile g on an
    ny x nx grid (nx defaults to ny)."""
    nx = ny if nx is None else nx
    if nx % tile_x or ny % tile_y:
        raise ValueError("the tile must divide the scan grid")
    ntx, nty = nx // tile_x, ny // tile_y
    pos = np.zeros((ntx * nty, tile_x * tile_y), dtype=np.int64)
    for gy in range(nty):
        for gx in range(ntx):
            g = gy * ntx + gx
            for jy in range(tile_y):
                for jx in range(tile_x):
                    pos[g, jy * tile_x + jx] = (gy * tile_y + jy) * nx + gx * tile_x + jx
    return pos


def forward(S: np.ndarray, m: np.ndarray, tile_x: int, tile_y: int) -> np.ndarray:
    """y[t, i, g] = sum_j S[i, j] m[t, pos(g, j)];  m [nt][ny][nx] -> y [nt][M][ntiles]."""
    S = np.asarray(S, dtype=np.float64)
    nt, ny, nx = m.shape
    pos = tile_positions(ny, tile_x, tile_y, nx)
    flat = np.asarray(m, dtype=np.float64).reshape(nt, ny * nx)
    y = np.zeros((nt, S.shape[0], pos.shape[0]))
    for g in range(pos.shape[0]):
        y[:, :, g] = flat[:, pos[g]] @ S.T
    return y


def adjoint(S: np.ndarray, y: np.ndarray, tile_x: int, tile_y: int, n: int, nx: int | None = None) -> np.ndarray:
    """m[t, pos(g, j)] = sum_i S[i, j] y[t, i, g];  y [nt][M][ntiles] -> m [nt][n][nx]
    (n rows; nx defaults to n)."""
    S = np.asarray(S, dtype=np.float64)
    nx = n if nx is None else nx
    nt = y.shape[0]
    pos = tile_positions(n, tile_x, tile_y, nx)
    flat = np.zeros((nt, n * nx))
    for g in range(pos.shape[0]):
        flat[:, pos[g]] = np.asarray(y[:, :, g], dtype=np.float64) @ S
    return flat.reshape(nt, n, nx)


class MuxOperator:
    """The composed operator S J of Eq. 12 around a confocal operator J
    (anything with forward, adjoint and shape = (nz, ny, nx, nt))."""

    def __init__(self, op, S: np.ndarray, tile_x: int, tile_y: int):
        self.op, self.S, self.tx, self.ty = op, np.asarray(S, dtype=np.float64), tile_x, tile_y
        self.shape = op.shape
        self.n, self.nx = op.shape[1], op.shape[2]

    def forward(self, mu):
        return forward(self.S, self.op.forward(mu), self.tx, self.ty)

    def adjoint(self, y):
        return self.op.adjoint(adjoint(self.S, y, self.tx, self.ty, self.n, self.nx))
