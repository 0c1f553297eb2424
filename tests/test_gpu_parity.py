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
from tests.gpu_common import (matrix_index, rel_l2, sampled_adjoint, sampled_forward, to_np,
                              unpack_forward_fragments)

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
P128 = geom(64, 5, 40, pitch=0.5, zr=(1.0, 8.0), dt=25.0)
P256 = geom(128, 3, 32, pitch=0.5, zr=(1.0, 6.0), dt=40.0)
WIDE = geom(40, 33, 36, pitch=0.5, zr=(1.0, 20.0), dt=25.0)

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


def test_fp64_quadrant_entry_equals_sized_one():
    """The unsized entry point (the buffer size fixed by the geometry) gives
    the sized one's values bit for bit, here on a non-square grid."""
    import ctypes
    c = ct()
    g = geom(13, 5, 40, pitch=0.7, zr=(1.5, 9.0), dt=30.0, mus=0.9)
    ref = c.tabulate_quadrant(g)
    gs, _z = c._geometry(g)
    out = torch.full_like(ref, float("nan"))
    st = c.lib().ctof_kernel_tabulate_fp64_quadrant(ctypes.byref(gs), out.data_ptr(), None)
    assert c.STATUS[st] == "CTOF_OK"
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    st = c.lib().ctof_kernel_tabulate_fp64_quadrant(ctypes.byref(gs), None, None)
    assert c.STATUS[st] == "CTOF_EINVAL"


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
    flat = k.khat[: i.nmat * ntp * nzp * 8].view(torch.float64).cpu().numpy()
    KH = unpack_forward_fragments(flat, i.nmat, ntp, nzp, 2, True)
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
    (P128, "fp64", 1e-12),
    (P128, "fp32", 1e-5),
    (P256, "fp64", 1e-12),
    (P256, "fp32", 1e-5),
    (P256, "bf16x3", 2e-3),
    (WIDE, "fp32", 1e-5),
    (WIDE, "fp64", 1e-12),
    (WIDE, "bf16x3", 2e-3),
]


@pytest.mark.parametrize("g,prec,tol", CASES,
                         ids=[f"{n}-{p}" for n, p in
                              [("tiny", "fp64"), ("tiny", "fp32"), ("ragged", "fp64"),
                               ("ragged", "fp32"), ("small", "fp32"), ("small", "bf16x3"),
                               ("small", "bf16"), ("p128", "fp64"), ("p128", "fp32"),
                               ("p256", "fp64"), ("p256", "fp32"), ("p256", "bf16x3"),
                               ("wide", "fp32"), ("wide", "fp64"), ("wide", "bf16x3")]])
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


@pytest.mark.parametrize("prec,fit_tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_skip_final_fit(prec, fit_tol):
    """Without the final forward pass the iterates, history and ratio are the
    same bit for bit, and the reported data fit is the one at the last step's
    extrapolated point y_K, checked against the oracle's history; the batched
    solver reports the same value."""
    c = ct()
    g, F, d = _tiny_problem(4)
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    iters = 30
    _, hist_ref = osolver.fista(F, d, L, lam, iters)
    p = c.PRECISIONS[prec]
    dt = torch.float64 if p == c.FP64 else torch.float32
    k = gpu_kernel(g, p)
    dd = torch.tensor(d, dtype=dt, device="cuda")
    mu1, rep1, h1 = c.reconstruct(k, dd, max_iter=iters, lam=lam, lipschitz=L, history=True)
    mu2, rep2, h2 = c.reconstruct(k, dd, max_iter=iters, lam=lam, lipschitz=L, history=True, final_fit=False)
    assert torch.equal(mu1, mu2) and torch.equal(h1, h2)
    assert rep1.gmap_ratio == rep2.gmap_ratio and rep1.datafit0 == rep2.datafit0
    assert rep2.datafit == h2[-1, 0].item()
    assert abs(rep2.datafit / hist_ref[-1, 0] - 1) <= fit_tol
    # the final fit is at mu_K, below the extrapolated point's near convergence
    assert rep1.datafit != rep2.datafit
    mus, reps = c.reconstruct_batched([k], [dd], max_iter=iters, lam=lam, lipschitz=L, final_fit=False)
    assert abs(reps[0].datafit / rep2.datafit - 1) <= fit_tol
    _, reps1 = c.reconstruct_batched([k], [dd], max_iter=iters, lam=lam, lipschitz=L)
    assert abs(reps1[0].datafit / rep1.datafit - 1) <= fit_tol


def test_skip_final_fit_rejects_other_values():
    import ctypes
    c = ct()
    g, F, d = _tiny_problem(4)
    k = gpu_kernel(g, c.FP64)
    dd = torch.tensor(d, device="cuda")
    mu = torch.zeros((g.nz, g.ny, g.nx), dtype=torch.float64, device="cuda")
    _, nb = k.workspace_bytes(3)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    opts = c._SolverOpts(3, 1e-3, 1.0, 50, 0.0, 10, 0, None, 0, None, None, None, None, None, 0, None, 2)
    rep = c._SolverReport()
    st = c.lib().ctof_reconstruct(k.handle, dd.data_ptr(), mu.data_ptr(), ctypes.byref(opts), ctypes.byref(rep),
                                  ws.data_ptr(), ws.numel(), None)
    assert c.STATUS[st] == "CTOF_EINVAL"
    assert b"skip_final_fit" in c.lib().ctof_last_error()


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


# -- full workload size: sampled outputs the oracle computes one by one ---------
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_full_size_forward_sampled(prec):
    """Full workload shape; the oracle sums the support voxels' kernels for
    whole time curves at selected pixels, including the peak of m.  FP32
    FFT rounding is absolute (about 1e-8 of the largest value), so FP32 is
    held to relative L2 over all sampled curves and to max error relative
    to the sampled peak; FP64 is held to per-pixel relative L2."""
    c = ct()
    p = c.PRECISIONS[prec]
    dt = torch.float64 if p == c.FP64 else torch.float32
    g = workloads.geometry_for("precision", seed=0)
    w = workloads.workload("precision")
    k = gpu_kernel(g, p)
    mu = phantoms.workload_phantom(w, g, 0)
    m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    zs, ys, xs = np.nonzero(mu)
    pk = np.unravel_index(int(np.argmax(np.abs(m))), m.shape)
    cy, cx = int(np.median(ys)), int(np.median(xs))
    pix = [(int(pk[1]), int(pk[2])), (cy, cx), (0, 0), (127, 127), (cy, min(cx + 9, 127)),
           (max(cy - 20, 0), cx), (64, 3)]
    ref = sampled_forward(g, mu, pix)
    got = np.array([m[:, i, j] for (i, j) in pix])
    for n, (i, j) in enumerate(pix):
        print(f"{prec} pixel {(i, j)}: rel {rel_l2(got[n], ref[n]):.3e}")
        if p == c.FP64 and np.abs(ref[n]).max() > 1e-6 * np.abs(m).max():
            assert rel_l2(got[n], ref[n]) <= 1e-11
    tol = 1e-12 if p == c.FP64 else 1e-5
    assert rel_l2(got, ref) <= tol
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def test_full_size_adjoint_sampled_fp32():
    c = ct()
    g = workloads.geometry_for("precision", seed=0)
    k = gpu_kernel(g, c.FP32)
    rng = np.random.default_rng(21)
    r = np.zeros((g.nt, g.ny, g.nx))
    src = [(int(a), int(b)) for a, b in rng.integers(0, 128, size=(8, 2))]
    for (i, j) in src:
        r[:, i, j] = rng.standard_normal(g.nt)
    gg = to_np(c.adjoint(k, torch.tensor(r, dtype=torch.float32, device="cuda")))
    samp = [(int(z), int(a), int(b)) for z, a, b in zip(rng.integers(0, g.nz, 40),
                                                        rng.integers(0, 128, 40),
                                                        rng.integers(0, 128, 40))]
    samp += [(0, src[0][0], src[0][1]), (63, src[1][0], src[1][1])]
    got = np.array([gg[z, a, b] for z, a, b in samp])
    ref = sampled_adjoint(g, r, src, samp)
    err = rel_l2(got, ref)
    print(f"adjoint sampled rel {err:.3e}")
    assert err <= 1e-5


def test_full_size_reconstruct_properties_fp32():
    c = ct()
    g = workloads.geometry_for("precision", seed=0)
    w = workloads.workload("precision")
    k = gpu_kernel(g, c.FP32)
    mu_true = phantoms.workload_phantom(w, g, 0)
    m_true = c.forward(k, torch.tensor(mu_true, dtype=torch.float32, device="cuda"))
    d = noise.poisson_histogram(m_true.double().cpu().numpy(), 1e5, 1000)
    dd = torch.tensor(d, dtype=torch.float32, device="cuda")
    mu, rep, hist = c.reconstruct(k, dd, max_iter=200, history=True)
    h = hist.cpu().numpy()
    print(f"L_A {rep.lipschitz_a:.4e} datafit0 {rep.datafit0:.4e} final {rep.datafit:.4e} gmap {rep.gmap_ratio:.3e}")
    # lambda = 1e-3 L_A is dominated by the shallow layers, so the deep part
    # of the data is regularised away: the fit improves but stays well above
    # the noise level; FISTA itself must have converged
    assert float(mu.min()) >= 0.0
    assert rep.datafit < 0.9 * rep.datafit0
    assert rep.gmap_ratio < 0.05
    assert h[-1, 0] < h[0, 0]
    assert np.all(np.isfinite(h))


# -- contraction launch shapes: blocks per spectrum matrix ------------------------
@pytest.mark.parametrize("g", [SMALL, WIDE, P256], ids=["small", "wide", "p256"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_contraction_parts_parity(g, prec):
    # the forward split into runs of bins and the adjoint split into partial
    # sums (added by the inverse column pass) give the same operator
    c = ct()
    p = c.PRECISIONS[prec]
    dt = torch.float64 if p == c.FP64 else torch.float32
    tol = 1e-12 if p == c.FP64 else 1e-5
    F = oracle_fft(g)
    rng = np.random.default_rng(41)
    mu = rng.random((g.nz, g.ny, g.nx))
    r = rng.standard_normal((g.nt, g.ny, g.nx))
    m_ref, g_ref = F.forward(mu), F.adjoint(r)
    k = c.tabulate(g, p)
    d = torch.tensor(m_ref, dtype=dt, device="cuda")
    _, rep0, _ = c.reconstruct(k, d, max_iter=1)
    base = None
    for fp, ap in [(1, 1), (2, 2), (4, 4), (8, 8), (0, 0)]:
        c.set_contract_parts(k, fp, ap)
        efp, eap = c.get_contract_parts(k)
        assert 1 <= efp <= 8 and 1 <= eap <= 8
        m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
        gg = to_np(c.adjoint(k, torch.tensor(r, dtype=dt, device="cuda")))
        assert rel_l2(m, m_ref) <= tol, (fp, ap)
        assert rel_l2(gg, g_ref) <= tol, (fp, ap)
        # a short solve: same iterates up to the order of the adjoint's sum
        mu_s, rep, _ = c.reconstruct(k, d, max_iter=12, lam=rep0.lam, lipschitz=rep0.lipschitz)
        if base is None:
            base = to_np(mu_s)
        else:
            assert rel_l2(to_np(mu_s), base) <= (1e-13 if p == c.FP64 else 1e-6)
    c.set_contract_parts(k, 0, 0)


def test_contraction_parts_rules():
    c = ct()
    k = c.tabulate(SMALL, c.FP32)
    with pytest.raises(c.CtofError):
        c.set_contract_parts(k, 3, 1)
    c.set_contract_parts(k, 8, 8)
    # 48 bins pad to 64: four 16-bin tiles and four chunks at most
    assert c.get_contract_parts(k) == (4, 4)
    kb = c.tabulate(SMALL, c.BF16X3)
    assert c.get_contract_parts(kb) == (1, 1)  # the BF16 rule: two blocks per matrix from 256 bins
    c.set_contract_parts(kb, 4, 4)
    assert c.get_contract_parts(kb) == (4, 1)  # the BF16 adjoints keep one block per matrix


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
def test_bf16_forward_split_is_bitwise_the_same(prec):
    # a BF16 forward split into runs of bins takes every tile's products in
    # the same order as one block per matrix: the same output bit for bit
    c = ct()
    k = c.tabulate(SMALL, c.PRECISIONS[prec])
    rng = np.random.default_rng(5)
    mu = torch.tensor(rng.random((SMALL.nz, SMALL.ny, SMALL.nx)), dtype=torch.float32, device="cuda")
    base = c.forward(k, mu)
    for fp in (2, 4, 8):
        c.set_contract_parts(k, fp, 0)
        assert torch.equal(c.forward(k, mu), base), fp
    c.set_contract_parts(k, 0, 0)
    assert rel_l2(to_np(base), oracle_fft(SMALL).forward(mu.double().cpu().numpy())) <= 2e-3
