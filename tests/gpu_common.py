"""Shared helpers for the GPU parity tests (inputs and comparisons only)."""

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def unpack_forward_fragments(flat, nmat, ntp, nzp, v, f64):
    """Decode the documented fragment order of the forward spectrum layout.

    Element (s, tt, ch, q, lane, e) holds K_s[t][z] with
    t = 16 tt + row(lane % 16), z = 4 kz ch + kz (lane // 16) + v q + e,
    kz = min(nzp, 64) / 4, row(i) = 4 (i % 4) + i // 4 for FP64 else i.
    Returns [nmat][ntp][nzp].
    """
    kz = min(nzp, 64) // 4
    nq, nch, ntt = kz // v, nzp // (4 * kz), ntp // 16
    a = np.asarray(flat).reshape(nmat, ntt, nch, nq, 64, v)
    tt, ch, q, lane, e = np.meshgrid(np.arange(ntt), np.arange(nch), np.arange(nq),
                                     np.arange(64), np.arange(v), indexing="ij")
    i = lane % 16
    row = 4 * (i % 4) + i // 4 if f64 else i
    t = 16 * tt + row
    z = 4 * kz * ch + kz * (lane // 16) + v * q + e
    out = np.zeros((nmat, ntp, nzp), dtype=np.float64)
    out[:, t.ravel(), z.ravel()] = a.reshape(nmat, -1)
    return out


def matrix_index(a, b):
    lo, hi = min(a, b), max(a, b)
    return hi * (hi + 1) // 2 + lo
