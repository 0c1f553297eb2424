"""Rectangular scan grids (ny rows x nx columns) against the FP64 oracle,
which evaluates the ny x nx operator directly (its FFT tier pads each axis
to twice its own side; the library pads both to the FFT size of the longer
side).  Forward and adjoint in FP64, FP32 and BF16 hi+lo for wide, tall,
odd and one-row grids; FISTA in FP64; a batch mixing a rectangular and a
square class; the transposed scan giving the transposed result; and
source multiplexing with tiles that divide each axis (products and a
multiplexed FISTA run against the oracle's rectangular tiling).
"""

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import mux as omux
from oracle import operator as oop
from oracle import solver as osolver
from synth import mux as smux
from synth.workloads import Geometry, even_layers
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _geom(ny, nx, nz=3, nt=24):
    z, dz = even_layers(1.5, 7.0, nz)
    return Geometry(nx=nx, ny=ny, pitch_mm=0.75, z_mm=z, dz_mm=dz, nt=nt, dt_ps=40.0)


@pytest.mark.parametrize("ny,nx", [(24, 40), (40, 24), (17, 30), (1, 9), (9, 1), (100, 7)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_forward_adjoint_match_oracle(ny, nx, prec):
    from paper_2101_11680_amd import ctof as c
    g = _geom(ny, nx)
    F = oop.FFTOperator(okernel.tabulate(g))
    tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 2e-3}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    k = c.tabulate(g, c.PRECISIONS[prec])
    assert (k.info.ny, k.info.nx, k.info.n) == (ny, nx, max(ny, nx))
    rng = np.random.default_rng(ny * 1000 + nx)
    mu = rng.uniform(0.0, 0.05, (g.nz, ny, nx))
    r = rng.standard_normal((g.nt, ny, nx))
    m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    a = to_np(c.adjoint(k, torch.tensor(r, dtype=dt, device="cuda")))
    em, ea = rel_l2(m, F.forward(mu)), rel_l2(a, F.adjoint(r))
    print(f"{ny}x{nx} {prec}: forward {em:.2e} adjoint {ea:.2e}")
    assert m.shape == (g.nt, ny, nx) and a.shape == (g.nz, ny, nx)
    assert em <= tol and ea <= tol


def test_fista_fp64_matches_oracle():
    from paper_2101_11680_amd import ctof as c
    g = _geom(20, 33)
    F = oop.FFTOperator(okernel.tabulate(g))
    mu = np.zeros((g.nz, 20, 33))
    mu[1, 5:9, 10:20] = 0.03
    d = F.forward(mu) * (1.0 + 0.01 * np.random.default_rng(2).standard_normal((g.nt, 20, 33)))
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    ref, hist = osolver.fista(F, d, L, lam, 40)
    k = c.tabulate(g, c.FP64)
    got, rep, h = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=40, lam=lam, lipschitz=L, history=True)
    assert rel_l2(to_np(got), ref) <= 1e-10
    np.testing.assert_allclose(to_np(h)[:, 1], hist[:, 1], rtol=1e-8)
    _, rep2, _ = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=1)
    assert rep2.lipschitz_a == pytest.approx(LA, rel=1e-9)


def test_transposed_scan_gives_transposed_result():
    from paper_2101_11680_amd import ctof as c
    ga, gb = _geom(12, 29), _geom(29, 12)
    ka, kb = c.tabulate(ga, c.FP64), c.tabulate(gb, c.FP64)
    rng = np.random.default_rng(4)
    mu = rng.uniform(0.0, 0.05, (ga.nz, 12, 29))
    ma = to_np(c.forward(ka, torch.tensor(mu, device="cuda")))
    mb = to_np(c.forward(kb, torch.tensor(np.ascontiguousarray(mu.transpose(0, 2, 1)), device="cuda")))
    assert rel_l2(mb, ma.transpose(0, 2, 1)) <= 1e-13
    d = torch.tensor(ma, device="cuda")
    _, rep, _ = c.reconstruct(ka, d, max_iter=1)
    xa, _, _ = c.reconstruct(ka, d, max_iter=30, lam=rep.lam, lipschitz=rep.lipschitz)
    xb, _, _ = c.reconstruct(kb, torch.tensor(np.ascontiguousarray(ma.transpose(0, 2, 1)), device="cuda"),
                             max_iter=30, lam=rep.lam, lipschitz=rep.lipschitz)
    assert rel_l2(to_np(xb), to_np(xa).transpose(0, 2, 1)) <= 1e-12


def test_batched_rectangular_and_square_classes():
    from paper_2101_11680_amd import ctof as c
    gr, gs = _geom(18, 31), _geom(24, 24)
    kr, ks = c.tabulate(gr, c.FP32), c.tabulate(gs, c.FP32)
    rng = np.random.default_rng(6)
    plan = [(gr, kr), (gs, ks), (gr, kr)]
    ds = []
    for g, _ in plan:
        F = oop.FFTOperator(okernel.tabulate(g))
        mu = np.zeros((g.nz, g.ny, g.nx))
        mu[1, 4:9, 6:14] = 0.04
        ds.append(torch.tensor(F.forward(mu) * (1 + 0.01 * rng.standard_normal((g.nt, g.ny, g.nx))),
                               dtype=torch.float32, device="cuda"))
    mus, reps = c.reconstruct_batched([k for _, k in plan], ds, max_iter=300, rel_tol=2e-2, check_every=10)
    for (g, k), d, mu, rep in zip(plan, ds, mus, reps):
        assert mu.shape == (g.nz, g.ny, g.nx)
        mu1, rep1, _ = c.reconstruct(k, d, max_iter=rep.iters)
        assert abs(rep.lipschitz / rep1.lipschitz - 1) <= 1e-12
        assert rel_l2(to_np(mu), to_np(mu1)) <= 1e-6


@pytest.mark.parametrize("ny,nx,tx,ty,M", [(8, 16, 4, 2, 12), (12, 8, 4, 4, 32), (6, 10, 5, 3, 15)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multiplexing_on_rectangular_grids(ny, nx, tx, ty, M, prec):
    from paper_2101_11680_amd import ctof as c
    g = _geom(ny, nx)
    tol = 1e-13 if prec == "fp64" else 1e-6
    dt = torch.float64 if prec == "fp64" else torch.float32
    k = c.tabulate(g, c.PRECISIONS[prec])
    rng = np.random.default_rng(ny * 31 + nx)
    S = rng.standard_normal((M, tx * ty))
    mx = c.Mux(torch.tensor(S, dtype=dt, device="cuda"), tx, ty)
    ntiles = (nx // tx) * (ny // ty)
    assert mx.ntiles(ny, nx) == ntiles
    m = rng.standard_normal((g.nt, ny, nx))
    yy = rng.standard_normal((g.nt, M, ntiles))
    y = to_np(c.mux_forward(k, mx, torch.tensor(m, dtype=dt, device="cuda")))
    assert rel_l2(y, omux.forward(S, m, tx, ty)) <= tol
    back = to_np(c.mux_adjoint(k, mx, torch.tensor(yy, dtype=dt, device="cuda")))
    assert rel_l2(back, omux.adjoint(S, yy, tx, ty, ny, nx)) <= tol
    r = to_np(c.mux_normal(k, mx, torch.tensor(m, dtype=dt, device="cuda"), y=torch.tensor(yy, dtype=dt, device="cuda")))
    assert rel_l2(r, omux.adjoint(S, omux.forward(S, m, tx, ty) - yy, tx, ty, ny, nx)) <= tol


def test_multiplexed_fista_fp64_on_a_rectangle():
    from paper_2101_11680_amd import ctof as c
    g = _geom(8, 16)
    S = smux.onoff(8)  # 4 x 2 tiles, on/off Hadamard patterns
    F = oop.FFTOperator(okernel.tabulate(g))
    Fm = omux.MuxOperator(F, S, 4, 2)
    mu = np.zeros((g.nz, 8, 16))
    mu[1, 2:5, 6:11] = 0.03
    y = Fm.forward(mu) * (1.0 + 0.01 * np.random.default_rng(8).standard_normal(Fm.forward(mu).shape))
    LA = osolver.power_iteration(Fm, 50)
    L, lam = osolver.step_constants(LA)
    ref, hist = osolver.fista(Fm, y, L, lam, 40)
    k = c.tabulate(g, c.FP64)
    mx = c.Mux(torch.tensor(S, device="cuda"), 4, 2)
    got, rep, h = c.reconstruct(k, torch.tensor(y, device="cuda"), max_iter=40, lam=lam, lipschitz=L, mux=mx,
                                history=True)
    assert rel_l2(to_np(got), ref) <= 1e-10
    np.testing.assert_allclose(to_np(h)[:, 1], hist[:, 1], rtol=1e-8, atol=1e-14)
    with pytest.raises(c.CtofError):  # a tile must divide its axis
        c.mux_forward(k, c.Mux(torch.tensor(smux.random_matrix(18, 9, 1), device="cuda"), 3, 3),
                      torch.zeros((g.nt, 8, 16), dtype=torch.float64, device="cuda"))
