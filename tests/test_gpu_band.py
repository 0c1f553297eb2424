"""The optional band of the kernel spectrum (ctof_kernel_set_band): the
products read, per spectrum matrix, only the 16-bin tiles and the leading
layer groups holding entries >= rel * max |entry|.  The band table is pinned
to the oracle's spectrum (every entry well above the threshold inside the
box, the box's edges each holding an entry near or above it).  Against the
FP64 oracle with a depth range where the band drops most of the spectrum:
forward and adjoint within the precision bars (FP32 1e-5, FP64 1e-12 at
rel 1e-15, BF16 hi+lo 2e-3) at 16, 64 and 80 layers (layer groups of 4 and
16, one and two layer chunks), the per-frequency bound of the header checked
on an input with all its weight at high frequencies in deep layers, FISTA in
FP32, batched solves, rel = 0 restoring the full products bit for bit, and
argument checks.
"""

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import operator as oop
from oracle import solver as osolver
from synth.workloads import Geometry, even_layers
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _geom(n=32, nz=16, nt=256):
    # the depth range and 10 ns window of the benchmark at a smaller grid
    z, dz = even_layers(1.0, 30.0, nz)
    return Geometry(nx=n, ny=n, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=nt, dt_ps=40.0)


@pytest.mark.parametrize("prec,rel,tol", [("fp32", 1e-9, 1e-5), ("fp64", 1e-15, 1e-12), ("bf16x3", 1e-9, 2e-3)])
def test_banded_products_match_oracle(prec, rel, tol):
    from paper_2101_11680_amd import ctof as c
    g = _geom()
    F = oop.FFTOperator(okernel.tabulate(g))
    dt = torch.float64 if prec == "fp64" else torch.float32
    k = c.tabulate(g, c.PRECISIONS[prec])
    rng = np.random.default_rng(1)
    mu = rng.uniform(0.0, 0.05, (g.nz, 32, 32))
    r = rng.standard_normal((g.nt, 32, 32))
    full_m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    kept = c.set_band(k, rel)
    print(f"{prec} rel {rel:g}: spectrum bytes kept {kept:.3f}")
    assert 0.0 < kept < (1.0 if prec == "fp64" else 0.5)
    m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    a = to_np(c.adjoint(k, torch.tensor(r, dtype=dt, device="cuda")))
    assert rel_l2(m, F.forward(mu)) <= tol and rel_l2(a, F.adjoint(r)) <= tol
    # rel = 0 gives the full products back, bit for bit
    assert c.set_band(k, 0.0) == 1.0
    assert np.array_equal(to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda"))), full_m)


def test_band_bound_on_high_frequency_input():
    # all weight in the deepest layer at the highest lateral frequency: the
    # banded forward may drop it, but only within the header's bound
    from paper_2101_11680_amd import ctof as c
    g = _geom()
    k = c.tabulate(g, c.FP64)
    kept = c.set_band(k, 1e-9)
    mu = np.zeros((g.nz, 32, 32))
    yy, xx = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    mu[-1] = np.where((yy + xx) % 2 == 0, 1.0, -1.0)
    banded = to_np(c.forward(k, torch.tensor(mu, device="cuda")))
    c.set_band(k, 0.0)
    full = to_np(c.forward(k, torch.tensor(mu, device="cuda")))
    # per frequency |dm^(f)[t]| <= rel max|Kp| sum_z |mu^_z(f)| (Kp: the
    # packed spectrum, which carries the 1/P^2 of the inverse transform);
    # with unnormalised transforms on the P x P torus Parseval gives
    # ||dm[t]|| <= P ||dm^[t]|| and ||mu^_z|| = P ||mu_z||, so with one
    # layer nonzero ||dm|| <= rel max|Kp| P^2 ||mu|| sqrt(nt)
    F = oop.FFTOperator(okernel.tabulate(g))
    P = F.py
    kmax = np.abs(F.Khat).max() / (P * P)
    bound = 1e-9 * kmax * P * P * np.linalg.norm(mu) * np.sqrt(g.nt)
    print(f"kept {kept:.3f}: |dm| {np.linalg.norm(banded - full):.3e} bound {bound:.3e} |m| {np.linalg.norm(full):.3e}")
    assert np.linalg.norm(banded - full) <= bound


def test_banded_fista_fp32_and_batched():
    from paper_2101_11680_amd import ctof as c
    g = _geom()
    F = oop.FFTOperator(okernel.tabulate(g))
    rng = np.random.default_rng(3)
    ds = []
    for s in range(3):
        mu = np.zeros((g.nz, 32, 32))
        mu[2 + s, 10:16, 12:20] = 0.03
        ds.append(F.forward(mu) * (1.0 + 0.01 * rng.standard_normal((g.nt, 32, 32))))
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    ref, _ = osolver.fista(F, ds[0], L, lam, 60)
    k = c.tabulate(g, c.FP32)
    c.set_band(k, 1e-9)
    dts = [torch.tensor(d, dtype=torch.float32, device="cuda") for d in ds]
    got, rep, _ = c.reconstruct(k, dts[0], max_iter=60, lam=lam, lipschitz=L)
    assert rel_l2(to_np(got), ref) <= 1e-5
    singles = [c.reconstruct(k, d, max_iter=60, lam=lam, lipschitz=L)[0] for d in dts]
    mus, _ = c.reconstruct_batched([k] * 3, dts, max_iter=60, lam=lam, lipschitz=L)
    for a, b in zip(singles, mus):
        assert rel_l2(to_np(b), to_np(a)) <= 1e-6


def test_band_argument_checks():
    from paper_2101_11680_amd import ctof as c
    import ctypes
    k = c.tabulate(_geom(n=8, nz=3, nt=32), c.FP32)
    buf = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    for bad in (-1e-9, 1.0, float("nan")):
        with pytest.raises(c.CtofError):
            c._check(c.lib().ctof_kernel_set_band(k.handle, bad, buf.data_ptr(), buf.numel(), c._stream_ptr()))
    with pytest.raises(c.CtofError):  # too small
        c._check(c.lib().ctof_kernel_set_band(k.handle, 1e-9, buf.data_ptr(), 64, c._stream_ptr()))
    with pytest.raises(c.CtofError):  # misaligned
        c._check(c.lib().ctof_kernel_set_band(k.handle, 1e-9, buf.data_ptr() + 4, buf.numel() - 4, c._stream_ptr()))


def test_band_with_rectangular_grid_and_multiplexing():
    # the band composes with a rectangular scan and with source multiplexing
    from oracle import mux as omux
    from synth import mux as smux
    from paper_2101_11680_amd import ctof as c
    z, dz = even_layers(1.0, 30.0, 16)
    g = Geometry(nx=32, ny=16, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=256, dt_ps=40.0)
    F = oop.FFTOperator(okernel.tabulate(g))
    k = c.tabulate(g, c.FP32)
    kept = c.set_band(k, 1e-9)
    assert 0.0 < kept < 0.5
    rng = np.random.default_rng(9)
    mu = rng.uniform(0.0, 0.05, (g.nz, 16, 32))
    assert rel_l2(to_np(c.forward(k, torch.tensor(mu, dtype=torch.float32, device="cuda"))), F.forward(mu)) <= 1e-5
    S = smux.onoff(16)
    Fm = omux.MuxOperator(F, S, 4, 4)
    mut = np.zeros((g.nz, 16, 32))
    mut[3, 4:9, 10:18] = 0.03
    y = Fm.forward(mut)
    LA = osolver.power_iteration(Fm, 50)
    L, lam = osolver.step_constants(LA)
    ref, _ = osolver.fista(Fm, y, L, lam, 40)
    mx = c.Mux(torch.tensor(S, dtype=torch.float32, device="cuda"), 4, 4)
    got, _, _ = c.reconstruct(k, torch.tensor(y, dtype=torch.float32, device="cuda"), max_iter=40, lam=lam,
                              lipschitz=L, mux=mx)
    assert rel_l2(to_np(got), ref) <= 1e-5


@pytest.mark.parametrize("prec,nz", [("fp32", 64), ("bf16x3", 64), ("fp32", 80), ("fp64", 80)])
def test_banded_products_layer_groups(prec, nz):
    # 64 layers: groups of 16 per lane group, 4 adjoint z tiles; 80 layers:
    # two layer chunks of 64 (the second one skipped for most matrices)
    from paper_2101_11680_amd import ctof as c
    g = _geom(n=16, nz=nz)
    F = oop.FFTOperator(okernel.tabulate(g))
    dt = torch.float64 if prec == "fp64" else torch.float32
    rel, tol = {"fp32": (1e-9, 1e-5), "fp64": (1e-15, 1e-12), "bf16x3": (1e-9, 2e-3)}[prec]
    k = c.tabulate(g, c.PRECISIONS[prec])
    kept = c.set_band(k, rel)
    tab = c.band_table(k)
    nzp = c._layers_packed(nz, k.info.precision)
    print(f"{prec} nz {nz}: bytes kept {kept:.3f}, matrices with fewer layers {(tab[:, 2] < nzp).float().mean():.3f}")
    assert bool((tab[:, 2] < nzp).any())
    rng = np.random.default_rng(5)
    mu = rng.uniform(0.0, 0.05, (nz, 16, 16))
    r = rng.standard_normal((g.nt, 16, 16))
    m = to_np(c.forward(k, torch.tensor(mu, dtype=dt, device="cuda")))
    a = to_np(c.adjoint(k, torch.tensor(r, dtype=dt, device="cuda")))
    assert rel_l2(m, F.forward(mu)) <= tol and rel_l2(a, F.adjoint(r)) <= tol


def test_band_table_is_the_box_of_the_oracle_spectrum():
    # matrix s = (a, b), b (b + 1)/2 <= s, holds the spectrum at (kx, ky) =
    # (a, b) (the same as at (b, a) on the square grid), rows t, columns z.
    # FP64 tabulates entries near rel * max to ~1e-15 max, so entries
    # above 2 rel max must lie inside the box and each edge of the box (first
    # and last tile, last layer group) must hold one above rel max / 2
    from paper_2101_11680_amd import ctof as c
    g = _geom()
    F = oop.FFTOperator(okernel.tabulate(g))
    A = np.abs(F.Khat.real)  # [z][t][ky][kx]
    amax = A.max()
    k = c.tabulate(g, c.FP64)
    for rel in (1e-9, 1e-6):
        c.set_band(k, rel)
        tab = c.band_table(k).numpy()
        kz = 4  # 16 layers: groups of nzp / 4
        P = F.py
        h = P // 2
        assert tab.shape[0] == (h + 1) * (h + 2) // 2
        shrunk_t = shrunk_z = 0
        for s in range(tab.shape[0]):
            b = int((np.sqrt(8 * s + 1) - 1) // 2)
            a = s - b * (b + 1) // 2
            M = A[:, :, b, a].T / amax  # [t][z]
            lo, hi, zend = (int(v) for v in tab[s])
            big = np.argwhere(M >= 2 * rel)
            if hi == lo:  # no entry at or above the threshold
                assert len(big) == 0 and (lo, hi, zend) == (0, 0, 0)
                continue
            if len(big):
                assert big[:, 0].min() >= 16 * lo and big[:, 0].max() < 16 * hi
                assert big[:, 1].max() < zend
            assert (M[16 * lo:16 * lo + 16] >= rel / 2).any()
            assert (M[16 * hi - 16:16 * hi] >= rel / 2).any()
            assert zend % kz == 0 and (M[:, zend - kz:zend] >= rel / 2).any()
            shrunk_t += (hi - lo) < tab[:, 1].max()
            shrunk_z += zend < g.nz
        print(f"rel {rel:g}: matrices with a shorter t range {shrunk_t}, with fewer layers {shrunk_z}")
        assert shrunk_z > 0
    c.set_band(k, 0.0)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
@pytest.mark.parametrize("nz", [20, 64])
def test_pipelined_bf16_adjoint_equals_band_form(prec, nz):
    # without a band the BF16 adjoints at up to 64 layers run the
    # software-pipelined kernel; a band holding every nonzero entry runs the
    # banded kernel over the same products in the same order (the tiles and
    # layer groups it skips hold only zeros): bitwise the same adjoint
    from paper_2101_11680_amd import ctof as c
    g = _geom(n=24, nz=nz, nt=96)
    k = c.tabulate(g, c.PRECISIONS[prec])
    rng = np.random.default_rng(nz)
    r = torch.tensor(rng.standard_normal((g.nt, 24, 24)), dtype=torch.float32, device="cuda")
    full = c.adjoint(k, r)
    c.set_band(k, 1e-300)
    banded = c.adjoint(k, r)
    c.set_band(k, 0.0)
    assert torch.equal(full, banded)
    F = oop.FFTOperator(okernel.tabulate(g))
    assert rel_l2(to_np(full), F.adjoint(r.double().cpu().numpy())) <= 2e-3
