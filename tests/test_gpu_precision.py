"""Precision forms against the FP64 oracle (reduced-precision contraction).

Forward and adjoint at the full 128x128 scan, 64 layers, 512 bins (sampled
oracle outputs); reconstructions after the same iterations with the same L
and lambda at a 32x32 scan, 16 layers, 128 bins, where the oracle's FP64
FISTA runs in seconds.  Bars: forward/adjoint relative L2 1e-5 (FP32),
2e-3 (BF16X3, BF16 hi-only spectrum); reconstruction data fit 1e-4 (FP32),
1e-2 (BF16 forms).  Each result is printed and written to
$CTOF_REPORT_DIR/precision_report.json when that variable names a folder.
"""

import json
import os

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import operator as oop
from oracle import solver as osolver
from synth import noise, phantoms, workloads
from synth.workloads import Geometry, even_layers
from tests.gpu_common import rel_l2, sampled_adjoint, sampled_forward, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FWD_TOL = {"fp32": 1e-5, "bf16x3": 2e-3, "bf16": 2e-3}
FIT_TOL = {"fp32": 1e-4, "bf16x3": 1e-2, "bf16": 1e-2}


def test_precision_report():
    from paper_2101_11680_amd import ctof as c
    report = {}
    g = workloads.geometry_for("precision", seed=0)
    w = workloads.workload("precision")
    mu = phantoms.workload_phantom(w, g, 0)
    zs, ys, xs = np.nonzero(mu)
    rng = np.random.default_rng(3)
    pix = [(int(ys[0]), int(xs[0])), (int(np.median(ys)), int(np.median(xs))), (0, 0), (64, 64),
           (127, 3)] + [(int(a), int(b)) for a, b in rng.integers(0, 128, size=(4, 2))]
    m_ref = sampled_forward(g, mu, pix)
    src = [(int(a), int(b)) for a, b in rng.integers(0, 128, size=(6, 2))]
    r = np.zeros((g.nt, g.ny, g.nx))
    for (i, j) in src:
        r[:, i, j] = rng.standard_normal(g.nt)
    # samples under and around the sources, where A^T r is large: FFT-domain
    # rounding is absolute, so far-field entries far below the peak would
    # measure the rounding floor rather than the path's accuracy
    samp = []
    for (i, j) in src:
        for z in (0, 6, 20, 40, 63):
            for (di, dj) in ((0, 0), (2, -3), (-4, 1)):
                samp.append((z, min(max(i + di, 0), 127), min(max(j + dj, 0), 127)))
    g_ref = sampled_adjoint(g, r, src, samp)
    for prec in ("fp32", "bf16x3", "bf16"):
        k = c.tabulate(g, c.PRECISIONS[prec])
        m = to_np(c.forward(k, torch.tensor(mu, dtype=torch.float32, device="cuda")))
        gg = to_np(c.adjoint(k, torch.tensor(r, dtype=torch.float32, device="cuda")))
        got_m = np.array([m[:, i, j] for (i, j) in pix])
        got_g = np.array([gg[z, a, b] for (z, a, b) in samp])
        report[prec] = {"forward_rel_l2_sampled": rel_l2(got_m, m_ref),
                        "adjoint_rel_l2_sampled": rel_l2(got_g, g_ref)}
        del k
        torch.cuda.empty_cache()

    # reconstruction parity at a shape the oracle solves in seconds
    z, dz = even_layers(1.0, 20.0, 16)
    gs = Geometry(nx=32, ny=32, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=128, dt_ps=25.0)
    F = oop.FFTOperator(okernel.tabulate(gs))
    mu_t = phantoms.phantom(gs, 5, n_abs=(2, 2), radius=(1.0, 1.5), dmua=(0.02, 0.04),
                            kinds=("sphere", "bar"))
    d = noise.poisson_histogram(F.forward(mu_t), 1e5, 9)
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    iters = 100
    mu_ref, _ = osolver.fista(F, d, L, lam, iters)
    fit_ref = osolver.datafit(F, d, mu_ref)
    for prec in ("fp32", "bf16x3", "bf16"):
        k = c.tabulate(gs, c.PRECISIONS[prec])
        mu_g, rep, _ = c.reconstruct(k, torch.tensor(d, dtype=torch.float32, device="cuda"),
                                     max_iter=iters, lam=lam, lipschitz=L)
        report[prec]["recon_datafit_rel"] = abs(rep.datafit / fit_ref - 1)
        report[prec]["recon_iterate_rel_l2"] = rel_l2(to_np(mu_g), mu_ref)
    print(json.dumps(report, indent=1))
    out = os.environ.get("CTOF_REPORT_DIR", "")
    if out and os.path.isdir(out):
        with open(os.path.join(out, "precision_report.json"), "w") as f:
            json.dump(report, f, indent=1)
    for prec, rr in report.items():
        assert rr["forward_rel_l2_sampled"] <= FWD_TOL[prec], (prec, rr)
        assert rr["adjoint_rel_l2_sampled"] <= FWD_TOL[prec], (prec, rr)
        assert rr["recon_datafit_rel"] <= FIT_TOL[prec], (prec, rr)
