"""Degenerate and extreme sizes against the FP64 oracle: a single scan point,
a single layer and a single time bin; all-zero data (the solve must stay at
zero with a zero gradient-mapping denominator, no NaN); the largest layer
count the library takes and a long histogram; a multiplexing tile that is
the whole scan with one measurement row.
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


def _geom(n, nz, nt, dt=50.0, zr=(2.0, 10.0)):
    z, dz = even_layers(zr[0], zr[1], nz)
    if nz == 1:
        dz = 1.0
    return Geometry(nx=n, ny=n, pitch_mm=1.0, z_mm=z, dz_mm=dz, nt=nt, dt_ps=dt)


@pytest.mark.parametrize("n,nz,nt", [(1, 1, 1), (2, 1, 3), (1, 3, 5), (3, 2, 1)])
def test_minimal_sizes_match_oracle(n, nz, nt):
    from paper_2101_11680_amd import ctof as c
    g = _geom(n, nz, nt, dt=200.0)
    F = oop.FFTOperator(okernel.tabulate(g))
    r = np.random.default_rng(n * 100 + nz * 10 + nt)
    mu = r.uniform(0.0, 0.05, (nz, n, n))
    d = r.uniform(0.0, 1.0, (nt, n, n)) * np.abs(F.forward(mu)).max()
    k = c.tabulate(g, c.FP64)
    assert rel_l2(to_np(c.forward(k, torch.tensor(mu, device="cuda"))), F.forward(mu)) <= 1e-12
    assert rel_l2(to_np(c.adjoint(k, torch.tensor(d, device="cuda"))), F.adjoint(d)) <= 1e-12
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    ref, hist = osolver.fista(F, d, L, lam, 20)
    got, rep, h = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=20, lam=lam, lipschitz=L,
                                history=True)
    assert rel_l2(to_np(got), ref) <= 1e-10
    np.testing.assert_allclose(to_np(h)[:, 1], hist[:, 1], rtol=1e-8, atol=1e-14)
    _, rep2, _ = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=1)
    assert rep2.lipschitz_a == pytest.approx(LA, rel=1e-9)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_data_stays_zero(prec):
    from paper_2101_11680_amd import ctof as c
    g = _geom(12, 4, 32)
    p, dt = (c.FP64, torch.float64) if prec == "fp64" else (c.FP32, torch.float32)
    k = c.tabulate(g, p)
    d = torch.zeros((g.nt, g.ny, g.nx), dtype=dt, device="cuda")
    mu0 = torch.full((g.nz, g.ny, g.nx), 0.3, dtype=dt, device="cuda")
    got, rep, h = c.reconstruct(k, d, mu=mu0, max_iter=30, history=True)  # zero start (warm_start off)
    assert torch.count_nonzero(got).item() == 0
    assert rep.gmap0 == 0.0 and rep.datafit == 0.0 and rep.datafit0 == 0.0
    assert np.all(to_np(h) == 0.0)
    # the tolerance rule stops at its first check
    _, rep2, _ = c.reconstruct(k, d, max_iter=100, rel_tol=1e-3, check_every=5)
    assert rep2.iters == 5 and rep2.status == 0


def test_largest_layer_count_matches_oracle():
    from paper_2101_11680_amd import ctof as c
    g = _geom(8, 256, 32, dt=40.0, zr=(1.0, 30.0))
    F = oop.FFTOperator(okernel.tabulate(g))
    r = np.random.default_rng(5)
    mu = r.uniform(0.0, 0.02, (g.nz, 8, 8))
    d = r.standard_normal((g.nt, 8, 8))
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        p, dt = (c.FP64, torch.float64) if prec == "fp64" else (c.FP32, torch.float32)
        k = c.tabulate(g, p)
        assert rel_l2(to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda"))), F.forward(mu)) <= tol
        assert rel_l2(to_np(c.adjoint(k, torch.tensor(d, dtype=dt, device="cuda"))), F.adjoint(d)) <= tol
    with pytest.raises(c.CtofError) as e:
        c.tabulate(_geom(8, 257, 8), c.FP32)
    assert e.value.status == -5


def test_long_histogram_matches_oracle():
    from paper_2101_11680_amd import ctof as c
    g = _geom(8, 2, 4096, dt=5.0, zr=(2.0, 6.0))
    F = oop.FFTOperator(okernel.tabulate(g))
    r = np.random.default_rng(6)
    mu = r.uniform(0.0, 0.05, (g.nz, 8, 8))
    d = r.standard_normal((g.nt, 8, 8))
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        p, dt = (c.FP64, torch.float64) if prec == "fp64" else (c.FP32, torch.float32)
        k = c.tabulate(g, p)
        assert rel_l2(to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda"))), F.forward(mu)) <= tol
        assert rel_l2(to_np(c.adjoint(k, torch.tensor(d, dtype=dt, device="cuda"))), F.adjoint(d)) <= tol


def test_mux_whole_scan_tile_and_single_row():
    from paper_2101_11680_amd import ctof as c
    g = _geom(8, 2, 24)
    k = c.tabulate(g, c.FP64)
    rng = np.random.default_rng(8)
    m = rng.standard_normal((g.nt, 8, 8))
    for S, tx, ty in ((smux.random_matrix(1, 64, 3), 8, 8), (smux.random_matrix(128, 64, 4), 8, 8),
                      (np.ones((1, 1)), 1, 1)):
        mx = c.Mux(torch.tensor(S, device="cuda"), tx, ty)
        y = to_np(c.mux_forward(k, mx, torch.tensor(m, device="cuda")))
        assert rel_l2(y, omux.forward(S, m, tx, ty)) <= 1e-13
        yy = rng.standard_normal(y.shape)
        back = to_np(c.mux_adjoint(k, mx, torch.tensor(yy, device="cuda")))
        assert rel_l2(back, omux.adjoint(S, yy, tx, ty, 8)) <= 1e-13


def test_stage_timing_stride():
    # stage events on every n-th iteration: the counts of timed iterations,
    # an early stop, the same iterates as without events, a negative stride
    # refused
    from paper_2101_11680_amd import ctof as c
    z, dz = even_layers(2.0, 10.0, 8)
    g = Geometry(nx=16, ny=16, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=64, dt_ps=50.0)
    k = c.tabulate(g, c.FP32)
    rng = np.random.default_rng(4)
    d = torch.tensor(rng.uniform(0.0, 1.0, (g.nt, 16, 16)), dtype=torch.float32, device="cuda")
    _, r0, _ = c.reconstruct(k, d, max_iter=1)
    kw = dict(max_iter=20, lam=r0.lam, lipschitz=r0.lipschitz)
    base, rb, _ = c.reconstruct(k, d, **kw)
    assert rb.timed_iters == 0 and rb.ms_loop == 0.0
    for stride, want in ((1, 20), (8, 3), (20, 1), (64, 1)):
        mu, rep, _ = c.reconstruct(k, d, timing=stride, **kw)
        assert rep.timed_iters == want
        assert rep.ms_contract_fwd > 0 and rep.ms_contract_adj > 0 and rep.ms_fft_t > 0 and rep.ms_fft_z > 0
        assert rep.ms_loop >= rep.ms_contract_fwd + rep.ms_contract_adj
        assert torch.equal(mu, base)
    # a stop after 10 iterations leaves the samples at 0 and 8
    _, rep, _ = c.reconstruct(k, d, timing=8, rel_tol=1e9, check_every=10, **kw)
    assert rep.iters == 10 and rep.timed_iters == 2
    with pytest.raises(c.CtofError):
        c.reconstruct(k, d, timing=-1, **kw)
