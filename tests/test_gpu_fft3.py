"""FFT sizes 48, 96, 192, 384 and 768 (a radix-12 or radix-24 first stage
built from a radix-3 step over power-of-two DFTs; from 384 on the column
block is held in LDS whole): scan sides 17-24, 33-48, 65-96, 129-192 and
257-384 take the smallest length >= 2n - 1 among the powers of two and
these.  Any such
length gives the same cropped linear convolution (Eq. 11), so the FP64
oracle (which picks its own transform length) is the reference: forward
and adjoint in FP64, FP32 and BF16 hi+lo, FISTA in FP64 and FP32, square
and rectangular grids, and the sides just outside each range.
"""

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import operator as oop
from oracle import solver as osolver
from synth.workloads import Geometry, even_layers
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _geom(ny, nx, nz=5, nt=40):
    z, dz = even_layers(1.5, 12.0, nz)
    return Geometry(nx=nx, ny=ny, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=nt, dt_ps=40.0)


@pytest.mark.parametrize("ny,nx,p", [(17, 17, 48), (24, 24, 48), (20, 9, 48), (33, 33, 96), (48, 48, 96),
                                    (40, 23, 96), (65, 65, 192), (96, 96, 192), (70, 96, 192),
                                    (129, 129, 384), (192, 150, 384), (16, 16, 32), (25, 25, 64), (49, 49, 128),
                                    (97, 97, 256), (193, 193, 512), (257, 257, 768), (384, 300, 768),
                                    (385, 385, 1024)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_forward_adjoint_match_oracle(ny, nx, p, prec):
    from paper_2101_11680_amd import ctof as c
    g = _geom(ny, nx)
    F = oop.FFTOperator(okernel.tabulate(g))
    tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 2e-3}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    k = c.tabulate(g, c.PRECISIONS[prec])
    assert k.info.p == p
    rng = np.random.default_rng(ny * 1000 + nx)
    mu = rng.uniform(0.0, 0.05, (g.nz, ny, nx))
    r = rng.standard_normal((g.nt, ny, nx))
    m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    a = to_np(c.adjoint(k, torch.tensor(r, dtype=dt, device="cuda")))
    em, ea = rel_l2(m, F.forward(mu)), rel_l2(a, F.adjoint(r))
    print(f"{ny}x{nx} P={p} {prec}: forward {em:.2e} adjoint {ea:.2e}")
    assert em <= tol and ea <= tol


@pytest.mark.parametrize("ny,nx", [(24, 24), (48, 40), (96, 96), (150, 130)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fista_matches_oracle(ny, nx, prec):
    from paper_2101_11680_amd import ctof as c
    g = _geom(ny, nx, nz=4, nt=32)
    F = oop.FFTOperator(okernel.tabulate(g))
    rng = np.random.default_rng(7)
    mu = np.zeros((g.nz, ny, nx))
    mu[1, ny // 3: ny // 2, nx // 4: nx // 2] = 0.03
    d = F.forward(mu) * (1.0 + 0.01 * rng.standard_normal((g.nt, ny, nx)))
    LA = osolver.power_iteration(F, 30)
    L, lam = osolver.step_constants(LA)
    ref, _ = osolver.fista(F, d, L, lam, 25)
    dt = torch.float64 if prec == "fp64" else torch.float32
    k = c.tabulate(g, c.PRECISIONS[prec])
    got, rep, _ = c.reconstruct(k, torch.tensor(d, dtype=dt, device="cuda"), max_iter=25, lam=lam, lipschitz=L)
    e = rel_l2(to_np(got), ref)
    print(f"{ny}x{nx} P={k.info.p} {prec}: FISTA {e:.2e}")
    assert e <= (1e-10 if prec == "fp64" else 1e-5)
    # a batch mixing the 3 * 2^k size with a power-of-two class
    g2 = _geom(16, 16, nz=4, nt=32)
    k2 = c.tabulate(g2, c.PRECISIONS[prec])
    F2 = oop.FFTOperator(okernel.tabulate(g2))
    d2 = F2.forward(rng.uniform(0.0, 0.02, (g2.nz, 16, 16)))
    ref2, _ = osolver.fista(F2, d2, L, lam, 25)
    mus, _ = c.reconstruct_batched([k, k2], [torch.tensor(d, dtype=dt, device="cuda"),
                                             torch.tensor(d2, dtype=dt, device="cuda")],
                                   max_iter=25, lam=lam, lipschitz=L)
    assert rel_l2(to_np(mus[0]), ref) <= (1e-10 if prec == "fp64" else 1e-5)
    assert rel_l2(to_np(mus[1]), ref2) <= (1e-10 if prec == "fp64" else 1e-5)


def test_fista_fp64_at_768():
    # a short FP64 solve at side 300 (P = 768: radix-24 first stages)
    from paper_2101_11680_amd import ctof as c
    g = _geom(300, 300, nz=2, nt=8)
    F = oop.FFTOperator(okernel.tabulate(g))
    rng = np.random.default_rng(3)
    d = F.forward(rng.uniform(0.0, 0.05, (g.nz, 300, 300)))
    LA = osolver.power_iteration(F, 20)
    L, lam = osolver.step_constants(LA)
    ref, _ = osolver.fista(F, d, L, lam, 8)
    k = c.tabulate(g, c.FP64)
    assert k.info.p == 768
    got, _, _ = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=8, lam=lam, lipschitz=L)
    assert rel_l2(to_np(got), ref) <= 1e-10
