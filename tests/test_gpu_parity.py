"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Tolerances (relative L2 unless stated): FP64 path 1e-12, FP32 path 1e-5,
BF16X3 2e-3, BF16 (hi-only kernel spectrum) 2e-3; reconstructions after the
same iterations with the same L and lambda: data fit 1e-10 (FP64), 1e-4
(FP32).
"""

import math

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import operator as oop
from oracle import solver as osolver
from synth import noise, phantoms, workloads
from synth.workloads import Geometry, even_layers
from tests.gpu_common import matrix_index, rel_l2, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def ct():
    from paper_2101_11680_amd import ctof
    return ctof


def geom(n, nz, nt, pitch=0.5, zr=(1.0, 12.0), dt=25.0, mus=1.0):
    z, dz = even_layers(zr[0], zr[1], nz)
    return Geometry(nx=n, ny=n, pitch_mm=pitch, z_mm=z, dz_mm=dz, nt=nt, dt_ps=dt,
                    mus_prime_per_mm=mus)


TINY = workloads.geometry_for("tiny")
RAGGED = geom(13, 5, 40, pitch=0.7, zr=(1.5, 9.0), dt=30.0, mus=0.9)
SMALL = geom(24, 6, 48, pitch=0.5, zr=(1.0, 12.0), dt=25.0)

_cache = {}


def oracle_kq(g):
    key = ("kq", g)
    if key not in _cache:
        _cache[key] = okernel.tabulate(g)
    return _cache[key]


def oracle_fft(g):
    key = ("fft", g)
    if key not in _cache:
        _cache[key] = oop.FFTOperator(oracle_kq(g))
    return _cache[key]


def gpu_kernel(g, prec):
    key = ("gpu", g, prec)
    if key not in _cache:
        print(f"[tabulate] n={g.nx} nz={g.nz} nt={g.nt} prec={prec}", flush=True)
        _cache[key] = ct().tabulate(g, prec)
    return _cache[key]


# -- kernel tabulation (FP64 on the GPU) ---------------------------------------
@pytest.mark.parametrize("g", [TINY, RAGGED, SMALL], ids=["tiny", "ragged", "small"])
def test_quadrant_fp64_matches_oracle(g):
    q = to_np(ct().tabulate_quadrant(g))          # [z][k][dy][dx]
    ref = np.transpose(oracle_kq(g), (0, 3, 1, 2))  # [z][dy][dx][k] -> [z][k][dy][dx]
    assert rel_l2(q, ref) <= 1e-12
    big = ref > 1e-6 * ref.max()
    assert np.max(np.abs(q[big] / ref[big] - 1)) <= 1e-11
    assert np.array_equal(q, np.swapaxes(q, 2, 3))   # exact dy <-> dx symmetry


def test_quadrant_mid_near_source_floor():
    g = workloads.geometry_for("mid")
    q = to_np(ct().tabulate_quadrant(g))
    rng = np.random.default_rng(0)
    iz = np.concatenate([[0, 0, 0, 1], rng.integers(0, g.nz, 12)])
    dy = np.concatenate([[0, 1, 0, 0], rng.integers(0, g.ny, 12)])
    dx = np.concatenate([[0, 0, 3, 0], rng.integers(0, g.nx, 12)])
    ref = okernel.tabulate_entries(g, iz, dy, dx)
    got = q[iz, :, dy, dx]
    assert rel_l2(got, ref) <= 1e-12


def test_khat_fp64_matches_oracle_spectrum():
    g = TINY
    k = gpu_kernel(g, ct().FP64)
    i = k.info
    P = i.p
    nzp = ((g.nz + 15) // 16) * 16
    ntp = ((g.nt + 31) // 32) * 32
    KH = k.khat[: i.nmat * ntp * nzp * 8].view(torch.float64).reshape(i.nmat, ntp, nzp).cpu().numpy()
    ref = oracle_fft(g).Khat.real / (P * P)       # [nz][nt][P][P/2+1]
    H = P // 2
    worst = 0.0
    scale = np.abs(ref).max()
    for a in range(H + 1):
        for b in range(H + 1):
            s = matrix_index(a, b)
            got = KH[s, : g.nt, : g.nz]              # [t][z]
            exp = ref[:, :, a, b].T                  # kx=a, ky=b -> [t][z]
            worst = max(worst, float(np.abs(got - exp).max()))
    assert worst <= 1e-13 * scale
    assert np.all(KH[:, g.nt:, :] == 0) and np.all(KH[:, :, g.nz:] == 0)


# -- forward / adjoint ----------------------------------------------------------
CASES = [
    (TINY, "fp64", 1e-12),
    (TINY, "fp32", 1e-5),
    (RAGGED, "fp64", 1e-12),
    (RAGGED, "fp32", 1e-5),
    (SMALL, "fp32", 1e-5),
    (SMALL, "bf16x3", 2e-3),
    (SMALL, "bf16", 2e-3),
]


@pytest.mark.parametrize("g,prec,tol", CASES,
                         ids=[f"{n}-{p}" for n, p in
                              [("tiny", "fp64"), ("tiny", "fp32"), ("ragged", "fp64"),
                               ("ragged", "fp32"), ("small", "fp32"), ("small", "bf16x3"),
                               ("small", "bf16")]])
def test_forward_adjoint_parity(g, prec, tol):
    c = ct()
    p = c.PRECISIONS[prec]
    k = gpu_kernel(g, p)
    dt = torch.float64 if p == c.FP64 else torch.float32
    rng = np.random.default_rng(11)
    mu = rng.random((g.nz, g.ny, g.nx))
    r = rng.standard_normal((g.nt, g.ny, g.nx))
    F = oracle_fft(g)
    m_ref = F.forward(mu)
    g_ref = F.adjoint(r)
    m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    gg = to_np(c.adjoint(k, torch.tensor(r, dtype=dt, device="cuda")))
    print(f"{prec}: fwd {rel_l2(m, m_ref):.3e} adj {rel_l2(gg, g_ref):.3e}")
    assert rel_l2(m, m_ref) <= tol
    assert rel_l2(gg, g_ref) <= tol


def test_forward_direct_sum_tiny_fp64():
    c = ct()
    g = TINY
    k = gpu_kernel(g, c.FP64)
    w = workloads.workload("tiny")
    mu = phantoms.workload_phantom(w, g, 3)
    m_ref = oop.forward_direct(oracle_kq(g), mu)
    m = to_np(c.forward(k, torch.tensor(mu, device="cuda")))
    assert rel_l2(m, m_ref) <= 1e-12


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_adjoint_identity_gpu(prec):
    c = ct()
    g = RAGGED
    p = c.PRECISIONS[prec]
    k = gpu_kernel(g, p)
    dt = torch.float64 if p == c.FP64 else torch.float32
    rng = np.random.default_rng(5)
    x = torch.tensor(rng.random((g.nz, g.ny, g.nx)), dtype=dt, device="cuda")
    r = torch.tensor(rng.standard_normal((g.nt, g.ny, g.nx)), dtype=dt, device="cuda")
    ax = c.forward(k, x).double()
    atr = c.adjoint(k, r).double()
    lhs = float((ax * r.double()).sum())
    rhs = float((x.double() * atr).sum())
    tol = 1e-12 if p == c.FP64 else 1e-5
    assert abs(lhs - rhs) <= tol * float(ax.norm()) * float(r.norm())


def test_delta_response_fp64():
    c = ct()
    g = RAGGED
    k = gpu_kernel(g, c.FP64)
    kq = oracle_kq(g)
    for (z, i0, j0) in [(0, 0, 0), (2, 6, 11), (4, 12, 3)]:
        e = torch.zeros((g.nz, g.ny, g.nx), dtype=torch.float64, device="cuda")
        e[z, i0, j0] = 1.0
        m = to_np(c.forward(k, e))
        ii = np.abs(np.arange(g.ny)[:, None] - i0)
        jj = np.abs(np.arange(g.nx)[None, :] - j0)
        exp = np.moveaxis(kq[z][ii, jj, :], 2, 0)
        assert rel_l2(m, exp) <= 1e-12


# -- reconstruction --------------------------------------------------------------
def _tiny_problem(seed=0):
    g = TINY
    w = workloads.workload("tiny")
    mu_true = phantoms.workload_phantom(w, g, seed)
    F = oracle_fft(g)
    d = noise.poisson_histogram(F.forward(mu_true), 1e5, 100 + seed)
    return g, F, d


def test_power_iteration_matches_oracle():
    c = ct()
    g, F, d = _tiny_problem()
    LA = osolver.power_iteration(F, 50)
    k = gpu_kernel(g, c.FP64)
    _, rep, _ = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=1)
    assert abs(rep.lipschitz_a / LA - 1) <= 1e-10
    assert abs(rep.lam / (1e-3 * LA) - 1) <= 1e-10
    assert abs(rep.lipschitz / (1.01 * LA + 1e-3 * LA) - 1) <= 1e-10


@pytest.mark.parametrize("prec,fit_tol,mu_tol", [("fp64", 1e-10, 1e-9), ("fp32", 1e-4, 1e-3)])
def test_reconstruct_matches_oracle_fista(prec, fit_tol, mu_tol):
    c = ct()
    g, F, d = _tiny_problem(1)
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    iters = 50
    mu_ref, hist_ref = osolver.fista(F, d, L, lam, iters)
    p = c.PRECISIONS[prec]
    dt = torch.float64 if p == c.FP64 else torch.float32
    k = gpu_kernel(g, p)
    mu, rep, hist = c.reconstruct(k, torch.tensor(d, dtype=dt, device="cuda"), max_iter=iters,
                                  lam=lam, lipschitz=L, history=True)
    fit_ref = osolver.datafit(F, d, mu_ref)
    print(f"{prec}: datafit gpu {rep.datafit:.10e} oracle {fit_ref:.10e}; mu rel {rel_l2(to_np(mu), mu_ref):.3e}")
    assert rep.iters == iters
    assert abs(rep.datafit / fit_ref - 1) <= fit_tol
    assert rel_l2(to_np(mu), mu_ref) <= mu_tol
    h = hist.cpu().numpy()
    assert np.max(np.abs(h[:, 0] / hist_ref[:, 0] - 1)) <= fit_tol
    assert np.max(np.abs(h[:, 1] - hist_ref[:, 1]) / np.maximum(hist_ref[:, 1], 1e-30)) <= 1e3 * fit_tol
    assert abs(rep.datafit0 / hist_ref[0, 0] - 1) <= fit_tol


def test_reconstruct_rel_tol_stops_early():
    c = ct()
    g, F, d = _tiny_problem(2)
    k = gpu_kernel(g, c.FP64)
    _, rep, hist = c.reconstruct(k, torch.tensor(d, device="cuda"), max_iter=400, rel_tol=5e-2,
                                 check_every=5, history=True)
    assert rep.iters < 400 and rep.iters % 5 == 0
    assert rep.gmap_ratio <= 5e-2
    assert hist.shape[0] == rep.iters


def test_reconstruct_warm_start_from_solution():
    c = ct()
    g, F, d = _tiny_problem(3)
    k = gpu_kernel(g, c.FP64)
    dd = torch.tensor(d, device="cuda")
    mu, rep, _ = c.reconstruct(k, dd, max_iter=300)
    mu2, rep2, _ = c.reconstruct(k, dd, mu=mu.clone(), max_iter=5, warm_start=True,
                                 lam=rep.lam, lipschitz=rep.lipschitz)
    assert rep2.datafit0 <= rep.datafit0
    assert abs(rep2.datafit0 / rep.datafit - 1) <= 1e-9
