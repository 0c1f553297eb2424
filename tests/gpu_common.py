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


class BinRunOperator:
    """The oracle's FFT-tier operator evaluated over runs of time bins.

    Eq. 11 gives every time bin of m as a sum over layers of that bin's
    kernel only, so the forward model is the concatenation of the forwards
    of runs of bins and the adjoint the sum of the runs' adjoints (added in
    run order).  Each run is an ``oracle.operator.FFTOperator`` of its own
    slice of the kernel; runs are built and evaluated in parallel threads
    (numpy's einsum and scipy's FFTs release the interpreter lock), which
    keeps the full-size kernel spectrum in bounded pieces and uses every
    host core.  Same interface as the oracle's operators.
    """

    def __init__(self, Kq, run: int = 32, threads=None):
        import os
        from concurrent.futures import ThreadPoolExecutor

        from oracle import operator as oop
        nz, n_y, n_x, nt = Kq.shape
        self.shape = Kq.shape
        self.bounds = [(t, min(nt, t + run)) for t in range(0, nt, run)]
        self.threads = int(threads or os.cpu_count() or 1)
        self._pool = ThreadPoolExecutor(self.threads)
        self.ops = list(self._pool.map(
            lambda b: oop.FFTOperator(np.ascontiguousarray(Kq[..., b[0]:b[1]]), workers=1), self.bounds))

    def forward(self, mu):
        parts = list(self._pool.map(lambda op: op.forward(mu), self.ops))
        return np.concatenate(parts, axis=0)

    def adjoint(self, r):
        parts = list(self._pool.map(lambda ob: ob[0].adjoint(np.ascontiguousarray(r[ob[1][0]:ob[1][1]])),
                                    zip(self.ops, self.bounds)))
        out = parts[0]
        for p in parts[1:]:
            out = out + p
        return out

    def close(self):
        self._pool.shutdown()
        self.ops = []


def tabulate_layers_parallel(g, threads=None):
    """``oracle.kernel.tabulate(g)`` evaluated one layer per task in parallel
    threads (each layer's kernel depends only on its own depth; the voxel
    thickness is the geometry's, shared by the single-layer geometries)."""
    import dataclasses
    import os
    from concurrent.futures import ThreadPoolExecutor

    from oracle import kernel as okernel
    subs = [dataclasses.replace(g, z_mm=(float(z),)) for z in g.z_mm]
    with ThreadPoolExecutor(int(threads or os.cpu_count() or 1)) as ex:
        parts = list(ex.map(okernel.tabulate, subs))
    return np.concatenate(parts, axis=0)
