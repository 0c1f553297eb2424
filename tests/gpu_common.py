"""Shared helpers for the GPU parity tests (inputs and comparisons only)."""

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def khat_matrices(k, dims_p, nmat, ntp, nzp, prec_bytes):
    """View the forward-layout spectrum [s][ntp][nzp] of a handle as numpy."""
    import torch
    dt = {8: torch.float64, 4: torch.float32}[prec_bytes]
    n = nmat * ntp * nzp
    return k.khat[: n * prec_bytes].view(dt).reshape(nmat, ntp, nzp).cpu().numpy().astype(np.float64)


def matrix_index(a, b):
    lo, hi = min(a, b), max(a, b)
    return hi * (hi + 1) // 2 + lo
