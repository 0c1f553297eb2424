"""The 2D single-plane workloads (the convolutional model of Eq. 9: one
absorbing plane, a 32x32 or 128x128 confocal scan) against the FP64 oracle:
forward and adjoint to 1e-5 (FP32), FISTA iterates after the same
iterations to 1e-5, and a solve to gradient-mapping ratio 1e-3."""

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import operator as oop
from oracle import solver as osolver
from synth import noise, phantoms, workloads
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name", ["2d32", "2d128"])
def test_2d_operator_and_fista_match_oracle(name):
    from paper_2101_11680_amd import ctof as c
    g = workloads.geometry_for(name)
    w = workloads.workload(name)
    F = oop.FFTOperator(okernel.tabulate(g))
    mu = phantoms.workload_phantom(w, g, 5)
    m = F.forward(mu)
    d = noise.poisson_histogram(m, 1e5, 6)
    k = c.tabulate(g, c.FP32)
    m_gpu = to_np(c.forward(k, torch.tensor(mu, dtype=torch.float32, device="cuda")))
    assert rel_l2(m_gpu, m) <= 1e-5
    g_gpu = to_np(c.adjoint(k, torch.tensor(d, dtype=torch.float32, device="cuda")))
    assert rel_l2(g_gpu, F.adjoint(d)) <= 1e-5
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    ref, hist = osolver.fista(F, d, L, lam, 60)
    dt = torch.tensor(d, dtype=torch.float32, device="cuda")
    got, rep, _ = c.reconstruct(k, dt, max_iter=60, lam=lam, lipschitz=L)
    assert rel_l2(to_np(got), ref) <= 1e-5
    _, rep2, _ = c.reconstruct(k, dt, max_iter=3000, rel_tol=1e-3, check_every=10)
    assert rep2.gmap_ratio <= 1e-3 and rep2.iters < 3000
    assert rep2.lipschitz_a == pytest.approx(LA, rel=1e-4)
