"""One kernel handle on several streams.

The handle holds the kernel spectrum and launch choices only; every call
brings its own workspace (the binding keeps one per device and stream), so
the same handle serves calls on any stream, one after another or at once
from several host threads, with bitwise the same results as on the default
stream.
"""

import threading

import pytest

from synth import noise, phantoms, workloads
from synth.workloads import Geometry, even_layers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _problem():
    from paper_2101_11680_amd import ctof
    z, dz = even_layers(1.0, 12.0, 8)
    g = Geometry(nx=40, ny=40, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=96, dt_ps=25.0)
    w = workloads.workload("mid")
    k = ctof.tabulate(g, ctof.FP32)
    mu = torch.tensor(phantoms.workload_phantom(w, g, 3), dtype=torch.float32, device="cuda")
    m = ctof.forward(k, mu)
    d = torch.tensor(noise.poisson_histogram(m.double().cpu().numpy(), 1e5, 17), dtype=torch.float32,
                     device="cuda")
    return ctof, k, mu, d


def test_forward_on_other_streams_is_bitwise_the_same():
    ctof, k, mu, d = _problem()
    ref = ctof.forward(k, mu)
    torch.cuda.synchronize()
    for _ in range(2):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            out = ctof.forward(k, mu, stream=s)
        s.synchronize()
        assert torch.equal(out, ref)


def test_concurrent_solves_on_two_streams():
    ctof, k, mu, d = _problem()
    _, rep0, _ = ctof.reconstruct(k, d, max_iter=1)
    kw = dict(max_iter=40, lam=rep0.lam, lipschitz=rep0.lipschitz)
    ref, rref, _ = ctof.reconstruct(k, d, **kw)
    streams = [torch.cuda.Stream() for _ in range(2)]
    out = [None, None]

    def run(j):
        with torch.cuda.stream(streams[j]):
            out[j] = ctof.reconstruct(k, d, stream=streams[j], **kw)

    torch.cuda.synchronize()
    threads = [threading.Thread(target=run, args=(j,)) for j in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    for j in range(2):
        mu_j, rep_j, _ = out[j]
        assert torch.equal(mu_j, ref)
        assert rep_j.datafit == rref.datafit and rep_j.gmap_ratio == rref.gmap_ratio
