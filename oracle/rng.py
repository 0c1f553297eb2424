"""Counter-based random numbers and Poisson sampling (test infrastructure).

Training data for the learned warm start are generated on the GPU: the
forward model's histogram m is scaled to a peak count, and the counts are
drawn from a Poisson law (the photon-counting noise of the paper's detector
model, section "Multiplexed Measurements").  The GPU and this oracle each
implement the same counter-based generator from its published definition,
so the sampled counts can be compared one by one.

* Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
  as easy as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key;
  each of ten rounds multiplies words 0 and 2 by two fixed odd constants,
  swaps and XORs the high halves with the other words and the key, and the
  key is advanced by two Weyl constants between rounds.
* A uniform in [0, 1) with 53 random bits from two 32-bit words.
* Poisson(lam): sequential search of the CDF for lam < 10; for lam >= 10
  the transformed rejection method with squeeze (Hoermann, "The transformed
  rejection method for generating Poisson random variables", Insurance:
  Mathematics and Economics 12, 1993), one Philox block (two uniforms) per
  trial.

Counter of element i, stream s, trial r: (i mod 2^32, i div 2^32, s, r);
key: (seed mod 2^32, seed div 2^32).
"""

from __future__ import annotations

import numpy as np
from scipy.special import gammaln

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on arrays of 32-bit counter words; returns 4 arrays."""
    c = [np.asarray(v, dtype=np.uint32).copy() for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint32).copy()
    k1 = np.asarray(k1, dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            p0 = M0 * c[0].astype(np.uint64)
            p1 = M1 * c[2].astype(np.uint64)
            hi0, lo0 = (p0 >> np.uint64(32)).astype(np.uint32), (p0 & MASK).astype(np.uint32)
            hi1, lo1 = (p1 >> np.uint64(32)).astype(np.uint32), (p1 & MASK).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def _key(seed: int):
    return np.uint32(seed & 0xFFFFFFFF), np.uint32((seed >> 32) & 0xFFFFFFFF)


def philox_words(seed: int, idx, stream: int = 0, trial=0):
    """Philox output for elements ``idx`` (int64 array), as 4 uint32 arrays."""
    idx = np.asarray(idx, dtype=np.int64)
    k0, k1 = _key(seed)
    lo = (idx & 0xFFFFFFFF).astype(np.uint32)
    hi = (idx >> 32).astype(np.uint32)
    s = np.full(idx.shape, stream & 0xFFFFFFFF, dtype=np.uint32)
    t = np.broadcast_to(np.asarray(trial, dtype=np.uint32), idx.shape)
    return philox4x32_10(lo, hi, s, t, k0, k1)


def uniform53(w_hi, w_lo):
    """(w_hi >> 5) * 2^26 + (w_lo >> 6), scaled by 2^-53: a double in [0, 1)."""
    a = (np.asarray(w_hi, dtype=np.uint32) >> np.uint32(5)).astype(np.float64)
    b = (np.asarray(w_lo, dtype=np.uint32) >> np.uint32(6)).astype(np.float64)
    return (a * 67108864.0 + b) * (1.0 / 9007199254740992.0)


SMALL_MEAN = 10.0
MAX_TRIALS = 1024


def _poisson_small(lam, u):
    """Smallest k with u <= F(k), accumulating p_k = p_{k-1} lam / k."""
    k = np.zeros(lam.shape, dtype=np.int64)
    p = np.exp(-lam)
    F = p.copy()
    active = u > F
    j = 0
    while active.any() and j < 1000:
        j += 1
        k[active] += 1
        p[active] = p[active] * lam[active] / k[active]
        F[active] = F[active] + p[active]
        active &= u > F
    return k


def _ptrs_constants(lam):
    smu = np.sqrt(lam)
    b = 0.931 + 2.53 * smu
    a = -0.059 + 0.02483 * b
    inv_alpha = 1.1239 + 1.1328 / (b - 3.4)
    vr = 0.9277 - 3.6224 / (b - 2.0)
    return a, b, inv_alpha, vr


def poisson_sample(lam, seed: int, stream: int = 0):
    """Poisson counts (int64) with means ``lam`` (float64 >= 0), element i using
    the counters of index i."""
    lam = np.asarray(lam, dtype=np.float64).ravel()
    n = lam.size
    idx = np.arange(n, dtype=np.int64)
    out = np.zeros(n, dtype=np.int64)
    small = lam < SMALL_MEAN
    if small.any():
        w = philox_words(seed, idx[small], stream, 0)
        out[small] = _poisson_small(lam[small], uniform53(w[0], w[1]))
    todo = np.nonzero(~small)[0]
    if todo.size:
        lm = lam[todo]
        a, b, inv_alpha, vr = _ptrs_constants(lm)
        log_lam = np.log(lm)
        res = np.full(todo.size, -1, dtype=np.int64)
        pending = np.ones(todo.size, dtype=bool)
        for trial in range(MAX_TRIALS):
            sel = np.nonzero(pending)[0]
            if sel.size == 0:
                break
            w = philox_words(seed, todo[sel], stream, trial)
            U = uniform53(w[0], w[1]) - 0.5
            V = uniform53(w[2], w[3])
            us = 0.5 - np.abs(U)
            kf = np.floor((2.0 * a[sel] / us + b[sel]) * U + lm[sel] + 0.43)
            quick = (us >= 0.07) & (V <= vr[sel])
            reject = (kf < 0) | ((us < 0.013) & (V > us))
            with np.errstate(divide="ignore", invalid="ignore"):
                lhs = np.log(V * inv_alpha[sel] / (a[sel] / (us * us) + b[sel]))
                rhs = -lm[sel] + kf * log_lam[sel] - gammaln(kf + 1.0)
            accept = quick | (~reject & (lhs <= rhs))
            res[sel[accept]] = kf[accept].astype(np.int64)
            pending[sel[accept]] = False
        # a trial budget this large is never exhausted in practice; the mean
        # rounded to an integer stands in if it were
        res[pending] = np.floor(lm[pending] + 0.5).astype(np.int64)
        out[todo] = res
    return out


def noisy_histogram(m, peak: float, seed: int, stream: int = 0):
    """d = Poisson(s m) / s with s = peak / max(m) (float32 out, float64 inside);
    negative rounding residue in m counts as zero mean."""
    m = np.asarray(m, dtype=np.float32)
    mx = float(m.max())
    s = peak / mx if mx > 0 else 0.0
    lam = np.maximum(m.astype(np.float64), 0.0) * s
    c = poisson_sample(lam, seed, stream)
    d = np.zeros(m.shape, dtype=np.float32) if s == 0 else (c.astype(np.float64) / s).astype(np.float32)
    return d.reshape(m.shape)


def noisy_counts(m, scale: float, background: float, seed: int, stream: int = 0):
    """Counting noise with dark counts (the multiplexing simulations of the
    paper): c = Poisson(scale max(m, 0) + background), returned as
    (c - background) / scale (float32 out, float64 inside)."""
    m = np.asarray(m, dtype=np.float32)
    lam = np.maximum(m.astype(np.float64), 0.0) * scale + background
    c = poisson_sample(lam.ravel(), seed, stream).reshape(m.shape)
    return ((c.astype(np.float64) - background) / scale).astype(np.float32)
