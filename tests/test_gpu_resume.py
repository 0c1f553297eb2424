"""Resumption of the FISTA state, the zero-start fallback as a fresh zero
start, and the gradient-mapping denominator taken inside a zero start's
first step.

The state of FISTA (section "Reconstruction Algorithm") is the iterate
mu_k, its predecessor mu_{k-1} and the counter k of the step-size sequence.
A run of K1 iterations that hands out (mu_K1, mu_{K1-1}, K1) and a second
call resumed from that state must reproduce one uninterrupted run of
K1 + K2 iterations bit for bit: every step of both runs is the same
arithmetic on the same values (same L and lambda, same launches).
"""

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import operator as oop
from oracle import solver as osolver
from synth import noise, phantoms
from synth.workloads import Geometry, even_layers
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def geom(n, nz, nt, z2=12.0, dt=25.0):
    z, dz = even_layers(1.0, z2, nz)
    return Geometry(nx=n, ny=n, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=nt, dt_ps=dt)


GA = geom(24, 6, 48)
GB = geom(13, 5, 40, z2=8.0, dt=30.0)


def _data(g, seed, dtype):
    F = oop.FFTOperator(okernel.tabulate(g))
    mu = phantoms.phantom(g, seed, n_abs=(1, 2), radius=(1.0, 1.5), dmua=(0.02, 0.04),
                          kinds=("sphere", "bar"))
    d = noise.poisson_histogram(F.forward(mu), 1e5, 100 + seed)
    return torch.tensor(d, dtype=dtype, device="cuda"), F, d


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_resume_is_bitwise_uninterrupted(prec):
    from paper_2101_11680_amd import ctof as c
    p = c.PRECISIONS[prec]
    dt = torch.float64 if p == c.FP64 else torch.float32
    k = c.tabulate(GA, p)
    d, _, _ = _data(GA, 3, dt)
    _, rep0, _ = c.reconstruct(k, d, max_iter=1)
    L, lam = rep0.lipschitz, rep0.lam
    full, rf, hf = c.reconstruct(k, d, max_iter=37, lam=lam, lipschitz=L, history=True)
    prev = torch.full_like(full, float("nan"))
    mu1, r1, h1 = c.reconstruct(k, d, max_iter=15, lam=lam, lipschitz=L, history=True, mu_prev=prev)
    assert r1.fista_k == 15
    # the state handed out: mu_15 and mu_14 of the uninterrupted sequence
    mu14, _, _ = c.reconstruct(k, d, max_iter=14, lam=lam, lipschitz=L)
    assert torch.equal(prev, mu14)
    # two resumed chunks: 15 + 10 + 12 = 37
    mu2, r2, h2 = c.reconstruct(k, d, mu=mu1, warm_start=1, max_iter=10, lam=lam, lipschitz=L, history=True,
                                mu_prev=prev, k0=r1.fista_k)
    assert r2.fista_k == 25
    mu3, r3, h3 = c.reconstruct(k, d, mu=mu2, warm_start=1, max_iter=12, lam=lam, lipschitz=L, history=True,
                                mu_prev=prev, k0=r2.fista_k)
    assert r3.fista_k == 37 and r3.iters == 12
    assert torch.equal(mu3, full), float((mu3 - full).abs().max())
    assert r3.datafit == rf.datafit
    # data-fit rows are the same sums of the same partials; the ratios share
    # their numerator, while the denominator ||max(0, A^T d)|| of the resumed
    # (warm) calls comes from the separate adjoint pass instead of the zero
    # start's first step: equal in FP32 and FP64, within the last bits of a
    # few entries with the BF16 split (whose matrix-core sums are not
    # exactly odd in their inputs)
    hs = torch.cat([h1, h2, h3]).cpu().numpy()
    np.testing.assert_array_equal(hs[:, 0], hf.cpu().numpy()[:, 0])
    np.testing.assert_allclose(hs[:, 1], hf.cpu().numpy()[:, 1], rtol=1e-12 if prec != "bf16x3" else 1e-6,
                               atol=0)


def test_resume_batched_is_bitwise_uninterrupted():
    from paper_2101_11680_amd import ctof as c
    ka, kb = c.tabulate(GA, c.FP32), c.tabulate(GB, c.FP32)
    plan = [(ka, GA, 0), (kb, GB, 1), (ka, GA, 2)]
    ds = [_data(g, s, torch.float32)[0] for _, g, s in plan]
    ks = [q[0] for q in plan]
    lips, lams = [], []
    for kk, d in zip(ks, ds):
        _, r, _ = c.reconstruct(kk, d, max_iter=1)
        lips.append(r.lipschitz)
        lams.append(r.lam)
    # one L per handle: the two scans of class A share the first scan's
    lips[2], lams[2] = lips[0], lams[0]
    full, rf = c.reconstruct_batched(ks, ds, max_iter=130, lam=lams, lipschitz=lips)
    prevs = [torch.zeros_like(m) for m in full]
    m1, r1 = c.reconstruct_batched(ks, ds, max_iter=70, lam=lams, lipschitz=lips, mu_prevs=prevs)
    assert all(r.fista_k == 70 for r in r1)
    m2, r2 = c.reconstruct_batched(ks, ds, mus=m1, warm_start=True, max_iter=60, lam=lams, lipschitz=lips,
                                   mu_prevs=prevs, k0=70)
    for q in range(len(plan)):
        assert r2[q].fista_k == 130
        assert torch.equal(m2[q], full[q]), (q, float((m2[q] - full[q]).abs().max()))
        assert r2[q].datafit == rf[q].datafit


def test_fallback_equals_fresh_zero_start():
    # a start 100x too large is discarded after one step; the remaining
    # K - 1 steps are those of a zero-start solve, bit for bit
    from paper_2101_11680_amd import ctof as c
    k = c.tabulate(GA, c.FP32)
    d, _, _ = _data(GA, 5, torch.float32)
    _, rep0, _ = c.reconstruct(k, d, max_iter=1)
    L, lam = rep0.lipschitz, rep0.lam
    zero, rz, hz = c.reconstruct(k, d, max_iter=40, lam=lam, lipschitz=L, history=True)
    def bad():
        return torch.full_like(zero, 50.0)  # (mu is in/out: a fresh start per call)

    mu, rb, hb = c.reconstruct(k, d, mu=bad(), warm_start=2, max_iter=41, lam=lam, lipschitz=L, history=True)
    assert rb.fell_back == 1 and rb.iters == 41 and rb.fista_k == 40
    assert torch.equal(mu, zero)
    assert rb.datafit0 == rz.datafit0 and rb.datafit == rz.datafit
    assert hb.shape == hz.shape
    np.testing.assert_allclose(hb.cpu().numpy(), hz.cpu().numpy(), rtol=1e-12, atol=0)
    # with a tolerance the restarted scan stops where the zero start stops
    zt, rzt, _ = c.reconstruct(k, d, max_iter=3000, lam=lam, lipschitz=L, rel_tol=1e-3, check_every=10)
    bt, rbt, _ = c.reconstruct(k, d, mu=bad(), warm_start=2, max_iter=3000, lam=lam, lipschitz=L,
                               rel_tol=1e-3, check_every=10)
    assert rbt.fell_back == 1 and rbt.iters == rzt.iters + 1
    assert torch.equal(bt, zt)
    # batched: one scan falls back, one keeps its start
    ks = [k, k]
    good = zero.clone()
    mus, reps = c.reconstruct_batched(ks, [d, d], mus=[bad(), good], warm_start=2, max_iter=41, lam=lam,
                                      lipschitz=L)
    assert reps[0].fell_back == 1 and reps[1].fell_back == 0
    assert reps[0].fista_k == 40 and reps[1].fista_k == 41
    assert torch.equal(mus[0], zero)
    assert reps[0].datafit0 == rz.datafit0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_start_denominator_equals_separate_pass(prec):
    # the first step of a zero start sees the gradient -A^T d; the
    # denominator ||max(0, A^T d)|| it accumulates equals the separate
    # adjoint pass that warm starts use (bit for bit: negation is exact in
    # every step of the operator)
    from paper_2101_11680_amd import ctof as c
    p = c.PRECISIONS[prec]
    dt = torch.float64 if p == c.FP64 else torch.float32
    k = c.tabulate(GB, p)
    d, F, dn = _data(GB, 7, dt)
    _, rep0, _ = c.reconstruct(k, d, max_iter=1)
    L, lam = rep0.lipschitz, rep0.lam
    zero = torch.zeros((GB.nz, GB.ny, GB.nx), dtype=dt, device="cuda")
    _, rz, hz = c.reconstruct(k, d, max_iter=20, lam=lam, lipschitz=L, history=True)
    _, rw, hw = c.reconstruct(k, d, mu=zero, warm_start=1, max_iter=20, lam=lam, lipschitz=L, history=True)
    print(f"{prec}: fused {rz.gmap0!r} separate {rw.gmap0!r}")
    assert rz.gmap0 == rw.gmap0
    assert torch.equal(hz, hw)
    ref = osolver.gmap_denominator(F, dn)
    assert abs(rz.gmap0 / ref - 1) <= (1e-12 if p == c.FP64 else 1e-5)
    # with per-layer L1 weights the denominator is ||max(0, A^T d - l1_z)||
    l1 = list(np.linspace(0.0, 0.5, GB.nz) * float(np.abs(F.adjoint(dn)).max()))
    _, rz1, _ = c.reconstruct(k, d, max_iter=3, lam=lam, lipschitz=L, l1=l1)
    _, rw1, _ = c.reconstruct(k, d, mu=zero, warm_start=1, max_iter=3, lam=lam, lipschitz=L, l1=l1)
    assert rz1.gmap0 == rw1.gmap0
    assert abs(rz1.gmap0 / osolver.gmap_denominator(F, dn, l1) - 1) <= (1e-12 if p == c.FP64 else 1e-5)


def test_resume_argument_checks():
    from paper_2101_11680_amd import ctof as c
    k = c.tabulate(GB, c.FP32)
    d, _, _ = _data(GB, 1, torch.float32)
    mu = torch.zeros((GB.nz, GB.ny, GB.nx), dtype=torch.float32, device="cuda")
    prev = torch.zeros_like(mu)
    with pytest.raises(c.CtofError):  # k0 > 0 without mu_{k0-1}
        c.reconstruct(k, d, mu=mu, warm_start=1, max_iter=3, k0=4)
    with pytest.raises(c.CtofError):  # k0 > 0 needs warm_start = 1
        c.reconstruct(k, d, mu=mu, warm_start=2, max_iter=3, k0=4, mu_prev=prev)
    with pytest.raises(c.CtofError):  # negative counter
        c.reconstruct(k, d, mu=mu, warm_start=1, max_iter=3, k0=-1, mu_prev=prev)
    with pytest.raises(c.CtofError):  # mu_prev aliasing mu
        c.reconstruct(k, d, mu=mu, warm_start=1, max_iter=3, k0=4, mu_prev=mu)


def test_resume_matches_oracle_fp64():
    # the resumed run is FISTA from the oracle's point of view as well
    from paper_2101_11680_amd import ctof as c
    k = c.tabulate(GB, c.FP64)
    d, F, dn = _data(GB, 2, torch.float64)
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    ref, _ = osolver.fista(F, dn, L, lam, 30)
    prev = torch.zeros((GB.nz, GB.ny, GB.nx), dtype=torch.float64, device="cuda")
    mu1, r1, _ = c.reconstruct(k, d, max_iter=11, lam=lam, lipschitz=L, mu_prev=prev)
    mu2, r2, _ = c.reconstruct(k, d, mu=mu1, warm_start=1, max_iter=19, lam=lam, lipschitz=L, mu_prev=prev,
                               k0=r1.fista_k)
    assert rel_l2(to_np(mu2), ref) <= 1e-10
