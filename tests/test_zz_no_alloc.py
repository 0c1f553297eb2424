"""The allocation-free forward entry point (ctof_forward_noalloc) against
ctof_forward: the same kernels on the library's fixed per-GPU scratch
instead of a caller workspace, so the histograms must agree bit for bit;
two calls in a row (the second on a smaller scan, reusing the scratch that
the first left behind), FP32 and FP64, and the size limit."""

import numpy as np
import pytest

from synth import phantoms, workloads
from synth.workloads import Geometry, even_layers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _small():
    z, dz = even_layers(1.0, 8.0, 5)
    return Geometry(nx=13, ny=11, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=40, dt_ps=30.0)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_forward_equals_forward(prec):
    from paper_2101_11680_amd import ctof as c
    p = c.PRECISIONS[prec]
    dt = torch.float64 if p == c.FP64 else torch.float32
    big = workloads.geometry_for("mid")  # 64 x 64 scan, 32 layers, 256 bins
    for g, seed in ((big, 1), (_small(), 2)):
        k = c.tabulate(g, p)
        op_ws, _ = k.workspace_bytes(1)
        assert op_ws <= 64 << 20
        mu = phantoms.phantom(g, seed, n_abs=(1, 3), radius=(0.8, 1.5), dmua=(0.02, 0.04), kinds=("sphere", "bar"))
        mu_t = torch.tensor(mu, dtype=dt, device="cuda")
        ref = c.forward(k, mu_t)
        got = torch.full_like(ref, float("nan"))
        c.forward_noalloc(k, mu_t, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (prec, g.nx, float((got - ref).abs().max()))
        assert float(ref.abs().max()) > 0


def test_noalloc_forward_rejects_oversized_shapes():
    from paper_2101_11680_amd import ctof as c
    z, dz = even_layers(1.0, 20.0, 16)
    g = Geometry(nx=128, ny=128, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=256, dt_ps=25.0)
    k = c.tabulate(g, c.FP32)
    op_ws, _ = k.workspace_bytes(1)
    assert op_ws > 64 << 20
    mu = torch.zeros((g.nz, g.ny, g.nx), dtype=torch.float32, device="cuda")
    out = torch.full((g.nt, g.ny, g.nx), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(c.CtofError) as ei:
        c.forward_noalloc(k, mu, out)
    assert ei.value.status == -2
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
