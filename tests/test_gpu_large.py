"""Scan sides above 192 (FFT sizes 512, 1024 and 2048: radix-32 column
stages with the column DFT held in LDS, three stages at 2048) against the
FP64 oracle: forward and adjoint in FP64, FP32 and BF16 hi+lo, short FISTA
runs in FP64, FP64 kernel values before the transform, and batched solves.
Sides 193 (the smallest with P = 512),
200, 256, 400 (P = 1024), 512, 600 (P = 2048), 1024 (the largest
supported) and the rectangles 512 x 96 and 40 x 1024 are covered; 1025 is
refused.
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


def _geom(n, nz=3, nt=20, nx=None):
    z, dz = even_layers(2.0, 8.0, nz)
    return Geometry(nx=nx or n, ny=n, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=nt, dt_ps=50.0)


_ORACLE = {}


def _oracle(n):
    if n not in _ORACLE:
        g = _geom(n)
        _ORACLE[n] = (g, oop.FFTOperator(okernel.tabulate(g)))
    return _ORACLE[n]


@pytest.mark.parametrize("n", [193, 200, 256])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_forward_adjoint_match_oracle(n, prec):
    from paper_2101_11680_amd import ctof as c
    g, F = _oracle(n)
    tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 2e-3}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    k = c.tabulate(g, c.PRECISIONS[prec])
    assert k.info.p == 512
    rng = np.random.default_rng(n)
    mu = rng.uniform(0.0, 0.05, (g.nz, n, n))
    r = rng.standard_normal((g.nt, n, n))
    m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    a = to_np(c.adjoint(k, torch.tensor(r, dtype=dt, device="cuda")))
    em, ea = rel_l2(m, F.forward(mu)), rel_l2(a, F.adjoint(r))
    print(f"n {n} {prec}: forward {em:.2e} adjoint {ea:.2e}")
    assert em <= tol and ea <= tol


def test_fista_fp64_matches_oracle_at_200():
    from paper_2101_11680_amd import ctof as c
    g, F = _oracle(200)
    rng = np.random.default_rng(3)
    mu = np.zeros((g.nz, 200, 200))
    mu[1, 80:95, 100:120] = 0.03
    d = F.forward(mu) * (1.0 + 0.01 * rng.standard_normal((g.nt, 200, 200)))
    LA = osolver.power_iteration(F, 30)
    L, lam = osolver.step_constants(LA)
    ref, hist = osolver.fista(F, d, L, lam, 15)
    k = c.tabulate(g, c.FP64)
    got, rep, h = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=15, lam=lam, lipschitz=L, history=True)
    assert rel_l2(to_np(got), ref) <= 1e-10
    np.testing.assert_allclose(to_np(h)[:, 1], hist[:, 1], rtol=1e-8)


def test_kernel_values_at_256_sampled():
    from paper_2101_11680_amd import ctof as c
    g, _ = _oracle(256)
    q = to_np(c.tabulate_quadrant(g))  # [z][k][dy][dx]
    iz = np.array([0, 1, 2, 2])
    dy = np.array([0, 17, 255, 128])
    dx = np.array([0, 250, 255, 3])
    ref = okernel.tabulate_entries(g, iz, dy, dx)
    got = q[iz, :, dy, dx]
    assert rel_l2(got, ref) <= 1e-12
    assert np.array_equal(q[:, :, 17, 250], q[:, :, 250, 17])  # exact dy <-> dx symmetry


def test_batched_equals_single_at_200():
    from paper_2101_11680_amd import ctof as c
    g, F = _oracle(200)
    k = c.tabulate(g, c.FP32)
    rng = np.random.default_rng(9)
    ds = []
    for s in range(3):
        mu = np.zeros((g.nz, 200, 200))
        mu[s, 40 + 10 * s:60 + 10 * s, 90:110] = 0.04
        ds.append(torch.tensor(F.forward(mu) * (1 + 0.01 * rng.standard_normal((g.nt, 200, 200))),
                               dtype=torch.float32, device="cuda"))
    _, rep0, _ = c.reconstruct(k, ds[0], max_iter=1)
    singles = [c.reconstruct(k, d, max_iter=20, lam=rep0.lam, lipschitz=rep0.lipschitz)[0] for d in ds]
    mus, _ = c.reconstruct_batched([k] * 3, ds, max_iter=20, lam=rep0.lam, lipschitz=rep0.lipschitz)
    for mu1, mub in zip(singles, mus):
        assert rel_l2(to_np(mub), to_np(mu1)) <= 1e-6


@pytest.mark.parametrize("ny,nx,p", [(400, 400, 1024), (512, 512, 1024), (512, 96, 1024), (600, 600, 2048),
                                    (1024, 1024, 2048), (40, 1024, 2048)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fft_sizes_1024_2048_match_oracle(ny, nx, p, prec):
    from paper_2101_11680_amd import ctof as c
    g = _geom(ny, nz=2, nt=8, nx=nx)
    F = oop.FFTOperator(okernel.tabulate(g))
    tol = {"fp64": 1e-12, "fp32": 1e-5}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    k = c.tabulate(g, c.PRECISIONS[prec])
    assert k.info.p == p
    rng = np.random.default_rng(ny + nx)
    mu = rng.uniform(0.0, 0.05, (g.nz, ny, nx))
    r = rng.standard_normal((g.nt, ny, nx))
    m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    a = to_np(c.adjoint(k, torch.tensor(r, dtype=dt, device="cuda")))
    em, ea = rel_l2(m, F.forward(mu)), rel_l2(a, F.adjoint(r))
    print(f"{ny}x{nx} {prec}: forward {em:.2e} adjoint {ea:.2e}")
    assert em <= tol and ea <= tol
    if prec == "fp64" and nx == ny and nx in (400, 600):
        d = F.forward(mu)
        LA = osolver.power_iteration(F, 20)
        L, lam = osolver.step_constants(LA)
        ref, _ = osolver.fista(F, d, L, lam, 8)
        got, _, _ = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=8, lam=lam, lipschitz=L)
        assert rel_l2(to_np(got), ref) <= 1e-10


def test_side_1025_is_refused():
    from paper_2101_11680_amd import ctof as c
    with pytest.raises(c.CtofError) as e:
        c.tabulate(_geom(1025), c.FP32)
    assert e.value.status == -5
    with pytest.raises(c.CtofError):
        c.tabulate(_geom(8, nx=1025), c.FP32)
