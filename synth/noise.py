"""Poisson counting noise on a noiseless confocal histogram.

The paper applies Poisson noise at a photon count rate to its simulated
measurements (section "Advantages of Multiplexing").  Here the histogram m
(absorption-induced signal, >= 0) is scaled so that its largest bin holds
``peak`` expected counts, sampled, and scaled back:
d = Poisson(s m) / s with s = peak / max(m).
"""

from __future__ import annotations

import numpy as np


def poisson_histogram(m: np.ndarray, peak: float, seed: int) -> np.ndarray:
    m = np.asarray(m, dtype=np.float64)
    mmax = float(m.max()) if m.size else 0.0
    if mmax <= 0.0:
        return np.zeros_like(m)
    s = peak / mmax
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = np.clip(s * m, 0.0, None)
    return rng.poisson(lam).astype(np.float64) / s
