"""Failure paths and reproducibility of the solver boundary.

* A NaN in the data or in a warm start makes an FP64 norm non-finite: the
  solve stops at its next check and returns CTOF_ENONFINITE with the
  report filled up to the iteration it reached.
* Arguments that break a rule are rejected before any GPU work: outputs
  filled with a canary pattern come back byte for byte unchanged.
* Two identical calls give bitwise identical iterates and reports (all
  reductions run in a fixed order).
* A step beyond 2/L_A (an explicit lipschitz below the operator's) makes
  FISTA diverge: the solve returns CTOF_EDIVERGED with the report filled.
"""

import ctypes

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import operator as oop
from synth import noise, phantoms, workloads
from synth.workloads import Geometry, even_layers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CANARY = 0x5A


def geom(n=20, nz=6, nt=48):
    z, dz = even_layers(1.0, 10.0, nz)
    return Geometry(nx=n, ny=n, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=nt, dt_ps=25.0)


def _raw_reconstruct(c, k, d, mu, max_iter, lam, lip, rel_tol=0.0, check_every=10, warm_start=0,
                     history=None, mu_prev=None, k0=0, ws=None):
    """ctof_reconstruct through ctypes, returning (status, report)."""
    i = k.info
    opts = c._SolverOpts(int(max_iter), float(lam), float(lip), 50, float(rel_tol), int(check_every),
                         int(warm_start), history.data_ptr() if history is not None else None, 0, None, None,
                         None, None, mu_prev.data_ptr() if mu_prev is not None else None, int(k0), None)
    rep = c._SolverReport()
    if ws is None:
        _, nb = k.workspace_bytes(max_iter)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    st = c.lib().ctof_reconstruct(k.handle, d.data_ptr(), mu.data_ptr(), ctypes.byref(opts), ctypes.byref(rep),
                                  ws.data_ptr(), ws.numel(), None)
    torch.cuda.synchronize()
    return st, rep


def _problem(c, g, prec=None):
    prec = c.FP32 if prec is None else prec
    dt = torch.float64 if prec == c.FP64 else torch.float32
    F = oop.FFTOperator(okernel.tabulate(g))
    mu = phantoms.phantom(g, 4, n_abs=(1, 2), radius=(1.0, 1.5), dmua=(0.02, 0.04), kinds=("sphere",))
    d = noise.poisson_histogram(F.forward(mu), 1e5, 11)
    k = c.tabulate(g, prec)
    dd = torch.tensor(d, dtype=dt, device="cuda")
    _, rep, _ = c.reconstruct(k, dd, max_iter=1)
    return k, dd, rep.lipschitz, rep.lam


@pytest.mark.parametrize("where", ["data", "start"])
def test_nonfinite_stops_with_filled_report(where):
    from paper_2101_11680_amd import ctof as c
    g = geom()
    k, d, L, lam = _problem(c, g)
    mu = torch.zeros((g.nz, g.ny, g.nx), dtype=torch.float32, device="cuda")
    warm = 0
    if where == "data":
        d = d.clone()
        d[7, 3, 5] = float("nan")
    else:
        mu[2, 4, 4] = float("nan")
        warm = 1
    hist = torch.zeros((60, 2), dtype=torch.float64, device="cuda")
    st, rep = _raw_reconstruct(c, k, d, mu, 60, lam, L, rel_tol=1e-3, check_every=5, warm_start=warm,
                               history=hist)
    assert st == -4, c.lib().ctof_last_error()
    assert rep.status == -4
    assert rep.iters == 5  # stopped at the first check
    assert rep.lipschitz == L and rep.lambda_ == lam
    h = hist.cpu().numpy()
    assert not np.all(np.isfinite(h[: rep.iters]))
    assert np.all(h[rep.iters:] == 0)  # rows past the stop untouched
    # the same scan without the NaN is fine
    st2, rep2 = _raw_reconstruct(c, k, torch.nan_to_num(d), torch.nan_to_num(mu), 60, lam, L, rel_tol=1e-3,
                                 check_every=5, warm_start=warm)
    assert st2 == 0 and rep2.status == 0


def test_nonfinite_batched_reports_the_scan():
    from paper_2101_11680_amd import ctof as c
    g = geom()
    k, d, L, lam = _problem(c, g)
    bad = d.clone()
    bad[0, 0, 0] = float("inf")
    with pytest.raises(c.CtofError) as ei:
        c.reconstruct_batched([k, k], [d, bad], max_iter=20, lam=lam, lipschitz=L)
    assert ei.value.status == -4


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_divergence_is_reported(prec):
    from paper_2101_11680_amd import ctof as c
    g = geom()
    p = c.PRECISIONS[prec]
    k, d, L, lam = _problem(c, g, p)
    dt = torch.float64 if p == c.FP64 else torch.float32
    mu = torch.zeros((g.nz, g.ny, g.nx), dtype=dt, device="cuda")
    # the step 1/L of a lipschitz at a fifth of the operator's is 2.5 times the
    # largest stable one: the error grows about fourfold per step
    st, rep = _raw_reconstruct(c, k, d, mu, 60, lam, 0.2 * L)
    assert st == -6, c.lib().ctof_last_error()
    assert rep.status == -6 and rep.iters == 60
    assert np.isfinite(rep.gmap_ratio) and rep.gmap_ratio > 1e6
    # with a tolerance the scan never meets it and is reported the same way
    st, rep = _raw_reconstruct(c, k, d, mu, 60, lam, 0.2 * L, rel_tol=1e-3, check_every=10)
    assert st == -6 and rep.iters == 60
    # the operator's own L: no divergence over the same iterations
    st, rep = _raw_reconstruct(c, k, d, mu, 60, lam, L)
    assert st == 0 and rep.gmap_ratio < 1.0
    # batched: the diverging scan is flagged, the other one is not
    k2 = c.tabulate(g, p)  # a second handle: a class of its own, with its own L
    with pytest.raises(c.CtofError) as ei:
        c.reconstruct_batched([k, k2], [d, d], max_iter=60, lam=[lam, lam], lipschitz=[0.2 * L, L])
    assert ei.value.status == -6


def _canary_like(t):
    out = torch.empty_like(t)
    out.view(torch.uint8).fill_(CANARY)
    return out


def test_einval_leaves_outputs_untouched():
    from paper_2101_11680_amd import ctof as c
    g = geom()
    k, d, L, lam = _problem(c, g)
    vol = torch.zeros((g.nz, g.ny, g.nx), dtype=torch.float32, device="cuda")
    mu = _canary_like(vol)
    prev = _canary_like(vol)
    hist = _canary_like(torch.zeros((10, 2), dtype=torch.float64, device="cuda"))
    before = [t.clone() for t in (mu, prev, hist)]
    bad_calls = [
        dict(max_iter=0, lam=lam, lip=L),                       # no iterations
        dict(max_iter=10, lam=-1.0, lip=L),                     # explicit L with lambda < 0
        dict(max_iter=10, lam=lam, lip=-2.0),                   # negative L
        dict(max_iter=10, lam=float("nan"), lip=0.0),           # non-finite lambda
        dict(max_iter=10, lam=lam, lip=L, rel_tol=1e-3, check_every=0),
        dict(max_iter=10, lam=lam, lip=L, warm_start=3),
        dict(max_iter=10, lam=lam, lip=L, warm_start=1, k0=3),  # resume without mu_{k0-1}
        dict(max_iter=10, lam=lam, lip=L, warm_start=0, k0=3, mu_prev=prev),
    ]
    for kw in bad_calls:
        st, _ = _raw_reconstruct(c, k, d, mu, history=hist, **kw)
        assert st == -1, (kw, c.lib().ctof_last_error())
    # a workspace one byte short: ENOMEM, nothing written
    _, nb = k.workspace_bytes(10)
    short = torch.empty(nb - 1, dtype=torch.uint8, device="cuda")
    st, _ = _raw_reconstruct(c, k, d, mu, 10, lam, L, history=hist, ws=short)
    assert st == -2
    for t, b in zip((mu, prev, hist), before):
        assert torch.equal(t.view(torch.uint8), b.view(torch.uint8))
    # the operator entry points behave the same way
    m = _canary_like(torch.zeros((g.nt, g.ny, g.nx), dtype=torch.float32, device="cuda"))
    m0 = m.clone()
    opws, _ = k.workspace_bytes(1)
    ws = torch.empty(opws - 1, dtype=torch.uint8, device="cuda")
    assert c.lib().ctof_forward(k.handle, vol.data_ptr(), m.data_ptr(), ws.data_ptr(), ws.numel(), None) == -2
    assert c.lib().ctof_forward(k.handle, None, m.data_ptr(), ws.data_ptr(), ws.numel(), None) == -1
    torch.cuda.synchronize()
    assert torch.equal(m.view(torch.uint8), m0.view(torch.uint8))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_two_runs_are_bitwise_identical(prec):
    from paper_2101_11680_amd import ctof as c
    g = workloads.geometry_for("mid")
    w = workloads.workload("mid")
    k = c.tabulate(g, c.PRECISIONS[prec])
    mu_t = torch.tensor(phantoms.workload_phantom(w, g, 2), dtype=torch.float32, device="cuda")
    m = c.forward(k, mu_t)
    d = torch.tensor(noise.poisson_histogram(m.double().cpu().numpy(), 1e5, 3), dtype=torch.float32,
                     device="cuda")
    runs = [c.reconstruct(k, d, max_iter=60, history=True) for _ in range(2)]
    (mu_a, ra, ha), (mu_b, rb, hb) = runs
    assert torch.equal(mu_a, mu_b)
    assert torch.equal(ha, hb)
    for f in ("datafit0", "datafit", "gmap_ratio", "lipschitz", "gmap0"):
        assert getattr(ra, f) == getattr(rb, f), f
    mus, reps = zip(*[c.reconstruct_batched([k, k], [d, d * 0.5], max_iter=70, rel_tol=1e-2, check_every=10)
                      for _ in range(2)])
    for q in range(2):
        assert torch.equal(mus[0][q], mus[1][q])
        assert reps[0][q].iters == reps[1][q].iters and reps[0][q].datafit == reps[1][q].datafit
