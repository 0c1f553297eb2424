"""Multiplexing patterns: the matrices S of the multiplexed workloads.

Inputs only (which sources are on in each measurement); nothing here
computes any part of the method.  Section "Advantages of Multiplexing"
multiplexes an 8 x 8 source array with a 64 x 64 Hadamard matrix; sources
are either on or off, so the measured patterns are its two 0/1 halves.
"""

from __future__ import annotations

import numpy as np


def hadamard(order: int) -> np.ndarray:
    """+-1 Hadamard matrix of a power-of-two order (Sylvester's doubling)."""
    if order < 1 or order & (order - 1):
        raise ValueError("order must be a power of two")
    h = np.array([[1.0]])
    while h.shape[0] < order:
        h = np.kron(np.array([[1.0, 1.0], [1.0, -1.0]]), h)
    return h


def onoff(order: int) -> np.ndarray:
    """The on/off patterns of the order-`order` Hadamard matrix: rows of
    (1 + H)/2 followed by rows of (1 - H)/2 (2 order x order, entries 0/1)."""
    h = hadamard(order)
    return np.vstack([(1.0 + h) / 2.0, (1.0 - h) / 2.0])


def random_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """A dense seeded Gaussian S (no structure, not symmetric)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal((rows, cols))
