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


def kernel_curves(g, z_idx, keys):
    """Oracle kernel time curves dV * bin integrals for layer z_idx at squared
    lateral offsets `keys` (in grid steps): [len(keys), nt]."""
    from oracle import kernel as okernel
    from oracle import physics
    o = okernel.optics_of(g)
    rho = g.pitch_mm * np.sqrt(np.asarray(keys, dtype=np.float64))
    return okernel.voxel_volume(g) * physics.kernel_bins(
        rho, float(g.z_mm[z_idx]), okernel.time_edges(g), o, okernel.r_min(g))


def sampled_forward(g, mu, pixels):
    """Oracle m[:, i, j] for each (i, j) in pixels, summing the kernels of the
    support voxels of a sparse volume mu: [len(pixels), nt]."""
    zs, ys, xs = np.nonzero(mu)
    out = np.zeros((len(pixels), g.nt))
    for n, (i, j) in enumerate(pixels):
        for z in np.unique(zs):
            sel = zs == z
            dy = np.abs(ys[sel] - i)
            dx = np.abs(xs[sel] - j)
            keys = dy * dy + dx * dx
            uk, inv = np.unique(keys, return_inverse=True)
            curves = kernel_curves(g, z, uk)
            out[n] += (curves[inv] * mu[z, ys[sel], xs[sel]][:, None]).sum(axis=0)
    return out


def sampled_adjoint(g, r, sources, samples):
    """Oracle g[z, a, b] for (z, a, b) in samples when r is nonzero only at the
    scan points `sources`."""
    out = np.zeros(len(samples))
    for n, (z, a, b) in enumerate(samples):
        keys = [(i - a) ** 2 + (j - b) ** 2 for (i, j) in sources]
        curves = kernel_curves(g, z, keys)
        out[n] = sum(float(curves[q] @ r[:, i, j]) for q, (i, j) in enumerate(sources))
    return out
