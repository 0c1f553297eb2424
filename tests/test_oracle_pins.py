"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself:
closed forms, library routines, brute force or invariants the paper states.
The paper prints no numeric worked example for this path, so there are no
paper-value fixtures; the closed forms below take their place.
"""

import math

import numpy as np
import pytest
from scipy import integrate, optimize, signal

from oracle import kernel, operator, physics, solver
from synth import noise, phantoms, workloads
from synth.workloads import Geometry, even_layers

OPT = physics.optics(1.0, 0.01, 1.4)
OPTICS_SET = [physics.optics(1.0, 0.01, 1.4), physics.optics(0.8, 0.02, 1.33),
              physics.optics(1.2, 0.005, 1.5)]


def small_geometry(n=6, nz=3, nt=24, dt=50.0, pitch=1.0, z=(2.0, 4.0, 6.0)):
    zz, dz = even_layers(z[0], z[-1], nz)
    return Geometry(nx=n, ny=n, pitch_mm=pitch, z_mm=zz, dz_mm=dz, nt=nt, dt_ps=dt)


# -- P1: infinite-medium Green's function integrates to the CW form --------
@pytest.mark.parametrize("o", OPTICS_SET)
@pytest.mark.parametrize("r", [0.3, 2.0, 12.0])
def test_p1_green_time_integral(o, r):
    v, _ = integrate.quad(lambda t: physics.green_inf(r, t, o), 0, np.inf,
                          epsabs=0, epsrel=1e-13, limit=500)
    assert abs(v / physics.green_inf_cw(r, o) - 1) < 1e-11


# -- P2: extrapolated boundary and the reflectance as a surface flux ---------
@pytest.mark.parametrize("o", OPTICS_SET)
def test_p2_boundary_and_flux(o):
    t = np.array([20.0, 150.0, 900.0])
    for rho in (0.0, 1.5, 7.0):
        # fluence from the pencil beam vanishes on the extrapolated boundary
        assert np.all(physics.phi0(rho, -o.zb, t, o) == 0.0)
        for z in (1.0, 4.0):
            # R = D dPhi/dz at the surface, Phi from a unit source at depth z
            def fluence(zp):
                r1 = math.sqrt(rho * rho + (zp - z) ** 2)
                r2 = math.sqrt(rho * rho + (zp + z + 2 * o.zb) ** 2)
                return physics.green_inf(r1, t, o) - physics.green_inf(r2, t, o)
            h = 1e-4
            fd = o.D * (fluence(h) - fluence(-h)) / (2 * h)
            R = physics.refl(rho, z, t, o)
            assert np.max(np.abs(fd / R - 1)) < 1e-7


# -- P3: time integral of the reflectance is the CW reflectance ------------
@pytest.mark.parametrize("o", OPTICS_SET)
@pytest.mark.parametrize("rho,z", [(0.0, 1.0), (3.0, 4.0), (10.0, 12.0)])
def test_p3_reflectance_cw(o, rho, z):
    v, _ = integrate.quad(lambda t: physics.refl(rho, z, t, o), 0, np.inf,
                          epsabs=0, epsrel=1e-12, limit=1000)
    assert abs(v / physics.refl_cw(rho, z, o) - 1) < 1e-9


# -- P4: closed-form Phi0 (*)_t R equals the numerical time convolution -----
@pytest.mark.parametrize("o", OPTICS_SET)
@pytest.mark.parametrize("rho,z,t", [(0.0, 2.0, 40.0), (3.0, 4.0, 300.0),
                                     (6.0, 10.0, 1500.0), (1.0, 16.0, 3000.0)])
def test_p4_convolution_closed_form(o, rho, z, t):
    f = lambda s: physics.phi0(rho, z, s, o) * physics.refl(rho, z, t - s, o)
    v, _ = integrate.quad(f, 0, t, epsabs=0, epsrel=1e-13, limit=2000,
                          points=[0.05 * t, 0.3 * t, 0.7 * t, 0.95 * t])
    k = physics.kernel_pointwise(rho, z, t, o)
    assert abs(k / v - 1) < 1e-12


# -- P5: Eq. 5 integrated over all time gives the CW Jacobian of Eq. 4 ------
@pytest.mark.parametrize("o", OPTICS_SET)
@pytest.mark.parametrize("rho,z", [(0.0, 2.0), (3.0, 4.0), (10.0, 16.0), (0.5, 1.2)])
def test_p5_time_integral_is_cw_jacobian(o, rho, z):
    te = np.concatenate([np.arange(0.0, 20000.0, 50.0), [1e5, 1e6, 1e8, 1e10]])
    total = physics.kernel_bins(rho, z, te, o).sum()
    cw = physics.phi0_cw(rho, z, o) * physics.refl_cw(rho, z, o)
    assert abs(total / cw - 1) < 1e-13
    assert abs(physics.kernel_total(rho, z, o) / cw - 1) < 1e-13


# -- P6: every bin against adaptive quadrature; bins telescope --------------
@pytest.mark.parametrize("rho,z,dt", [(0.0, 2.0, 50.0), (5.0, 8.0, 50.0),
                                      (0.0, 1.0, 25.0), (12.0, 3.0, 20.0)])
def test_p6_bins_vs_quadrature(rho, z, dt):
    nb = 64
    te = np.arange(nb + 1) * dt
    b = physics.kernel_bins(rho, z, te, OPT)[0]
    for k in range(nb):
        v, _ = integrate.quad(lambda t: physics.kernel_pointwise(rho, z, t, OPT),
                              te[k], te[k + 1], epsabs=0, epsrel=1e-13, limit=500)
        assert abs(b[k] - v) <= 1e-12 * abs(v)
    one = physics.kernel_bins(rho, z, np.array([0.0, te[-1]]), OPT)[0, 0]
    assert abs(b.sum() / one - 1) < 1e-12


def test_p6_near_source_floor():
    # the floor replaces only the source-to-voxel distance and keeps K finite
    g = workloads.geometry_for("mid")
    K = kernel.tabulate_entries(g, [0, 0], [0, 1], [0, 0])
    assert np.all(np.isfinite(K)) and np.all(K >= 0)
    rmin = kernel.r_min(g)
    o = kernel.optics_of(g)
    r11, _ = physics.source_distances(0.0, g.z_mm[0], o)
    assert r11 < rmin  # the z = 1 mm layer at mid triggers the floor


# -- P7: positivity, exact symmetry, real and 8-fold symmetric spectrum -----
def test_p7_kernel_symmetry_and_real_spectrum():
    g = workloads.geometry_for("tiny")
    Kq = kernel.tabulate(g)
    assert np.all(Kq > 0)
    assert np.array_equal(Kq, np.swapaxes(Kq, 1, 2))
    F = operator.FFTOperator(Kq)
    re = np.abs(F.Khat.real).max()
    assert np.abs(F.Khat.imag).max() <= 1e-14 * re
    Kh = F.Khat.real  # [nz, nt, P, P/2+1]
    P = Kh.shape[2]
    H = P // 2
    sub = Kh[:, :, :H + 1, :H + 1]
    assert np.max(np.abs(sub - np.swapaxes(sub, 2, 3))) <= 1e-14 * re
    flip = Kh[:, :, (P - np.arange(P)) % P, :]
    assert np.max(np.abs(Kh - flip)) <= 1e-14 * re


# -- P8: the kernel is the response to a spatial delta ----------------------
def test_p8_delta_response():
    g = workloads.geometry_for("tiny")
    Kq = kernel.tabulate(g)
    nz, n, _, nt = Kq.shape
    for (z, i0, j0) in [(0, 0, 0), (3, 5, 11), (7, 15, 2)]:
        e = np.zeros((nz, n, n))
        e[z, i0, j0] = 1.0
        m = operator.forward_direct(Kq, e)
        ii = np.abs(np.arange(n)[:, None] - i0)
        jj = np.abs(np.arange(n)[None, :] - j0)
        expect = np.moveaxis(Kq[z][ii, jj, :], 2, 0)
        assert np.array_equal(m, expect)


# -- P9: a shifted scene gives a shifted measurement ------------------------
def test_p9_shift_invariance():
    g = small_geometry(n=10)
    Kq = kernel.tabulate(g)
    rng = np.random.default_rng(3)
    mu = np.zeros((g.nz, 10, 10))
    mu[:, 2:5, 1:4] = rng.random((g.nz, 3, 3))
    sy, sx = 3, 4
    mu2 = np.zeros_like(mu)
    mu2[:, 2 + sy:5 + sy, 1 + sx:4 + sx] = mu[:, 2:5, 1:4]
    m = operator.forward_direct(Kq, mu)
    m2 = operator.forward_direct(Kq, mu2)
    a = m2[:, sy:, sx:]
    b = m[:, :10 - sy, :10 - sx]
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(m))


# -- P10 / P11 / P12: adjoint identity, explicit Jacobian, FFT tier ---------
@pytest.fixture(scope="module")
def tiny_setup():
    g = workloads.geometry_for("tiny")
    Kq = kernel.tabulate(g)
    rng = np.random.default_rng(7)
    x = rng.random((g.nz, g.ny, g.nx))
    r = rng.standard_normal((g.nt, g.ny, g.nx))
    return g, Kq, x, r


def test_p10_adjoint_identity(tiny_setup):
    g, Kq, x, r = tiny_setup
    for op in (operator.DirectOperator(Kq), operator.FFTOperator(Kq)):
        ax = op.forward(x)
        lhs = float(np.vdot(ax, r))
        rhs = float(np.vdot(x, op.adjoint(r)))
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(ax) * np.linalg.norm(r)


def test_p11_explicit_jacobian(tiny_setup):
    g, Kq, x, r = tiny_setup
    J = operator.jacobian(Kq)
    m0 = operator.forward_direct(Kq, x)
    m1 = (J @ x.ravel()).reshape(m0.shape)
    assert np.linalg.norm(m1 - m0) <= 1e-14 * np.linalg.norm(m0)
    g0 = operator.adjoint_direct(Kq, r)
    g1 = (J.T @ r.ravel()).reshape(g0.shape)
    assert np.linalg.norm(g1 - g0) <= 1e-14 * np.linalg.norm(g0)


def test_p12_fft_tier_matches_direct(tiny_setup):
    g, Kq, x, r = tiny_setup
    F = operator.FFTOperator(Kq)
    m0 = operator.forward_direct(Kq, x)
    assert np.linalg.norm(F.forward(x) - m0) <= 1e-13 * np.linalg.norm(m0)
    g0 = operator.adjoint_direct(Kq, r)
    assert np.linalg.norm(F.adjoint(r) - g0) <= 1e-13 * np.linalg.norm(g0)


def test_p12_fft_tier_rectangular_grid():
    zz, dz = even_layers(2.0, 5.0, 2)
    g = Geometry(nx=7, ny=5, pitch_mm=0.8, z_mm=zz, dz_mm=dz, nt=12, dt_ps=40.0)
    Kq = kernel.tabulate(g)
    x = np.random.default_rng(0).random((2, 5, 7))
    F = operator.FFTOperator(Kq)
    m0 = operator.forward_direct(Kq, x)
    assert np.linalg.norm(F.forward(x) - m0) <= 1e-13 * np.linalg.norm(m0)
    r = np.random.default_rng(1).standard_normal((12, 5, 7))
    g0 = operator.adjoint_direct(Kq, r)
    assert np.linalg.norm(F.adjoint(r) - g0) <= 1e-13 * np.linalg.norm(g0)
    # the 5 x 7 operator is the 7 x 7 one restricted to voxels and scan
    # points of the first five rows (absorbers elsewhere zero, the other
    # rows' measurements dropped), with the same kernel values
    gs = Geometry(nx=7, ny=7, pitch_mm=0.8, z_mm=zz, dz_mm=dz, nt=12, dt_ps=40.0)
    Ks = kernel.tabulate(gs)
    assert np.array_equal(Ks[:, :5, :, :], Kq)
    xs = np.zeros((2, 7, 7))
    xs[:, :5, :] = x
    ms = operator.forward_direct(Ks, xs)
    assert np.linalg.norm(ms[:, :5, :] - m0) <= 1e-14 * np.linalg.norm(m0)
    rs = np.zeros((12, 7, 7))
    rs[:, :5, :] = r
    assert np.linalg.norm(operator.adjoint_direct(Ks, rs)[:, :5, :] - g0) <= 1e-14 * np.linalg.norm(g0)


# -- P13: FISTA reaches the constrained least-squares minimiser -------------
class _JOp:
    def __init__(self, J, shape):
        self.J = J
        self.shape = shape

    def forward(self, mu):
        nz, n_y, n_x, nt = self.shape
        return (self.J @ mu.ravel()).reshape(nt, n_y, n_x)

    def adjoint(self, r):
        nz, n_y, n_x, nt = self.shape
        return (self.J.T @ r.ravel()).reshape(nz, n_y, n_x)


def test_p13_fista_matches_bounded_lsq():
    g = small_geometry()
    Kq = kernel.tabulate(g)
    J = operator.jacobian(Kq)
    op = _JOp(J, Kq.shape)
    mu_true = phantoms.phantom(g, 4, n_abs=(2, 2), radius=(1.2, 1.2), dmua=(0.03, 0.03))
    d = noise.poisson_histogram(op.forward(mu_true), 1e5, 11)
    L_A = float(np.linalg.eigvalsh(J.T @ J)[-1])
    L, lam = solver.step_constants(L_A)
    mu, hist = solver.fista(op, d, L, lam, 20000)
    A = np.vstack([J, math.sqrt(lam) * np.eye(J.shape[1])])
    b = np.concatenate([d.ravel(), np.zeros(J.shape[1])])
    ref = optimize.lsq_linear(A, b, bounds=(0, np.inf), method="bvls", tol=1e-15).x
    assert np.linalg.norm(mu.ravel() - ref) <= 1e-6 * np.linalg.norm(ref)
    assert hist[-1, 1] < 1e-8


def test_fista_rate_and_momentum_pins(monkeypatch):
    # Beck and Teboulle's guarantee for FISTA with a constant step 1/L,
    # L >= Lipschitz constant of the smooth part (here L_A + lam):
    #   F(mu_k) - F* <= 2 L ||mu_0 - mu*||^2 / (k + 1)^2   for every k,
    # with F* and mu* from the library's bounded least squares; and the
    # momentum sequence's t_k >= (k + 1) / 2 (recovered from the weights
    # beta_k = (t_k - 1) / t_{k+1}).  Without momentum (beta = 0, plain
    # projected gradient) the same bound fails on this problem, so the pin
    # sees whether the weights accelerate at all.
    g = small_geometry()
    Kq = kernel.tabulate(g)
    J = operator.jacobian(Kq)
    op = _JOp(J, Kq.shape)
    mu_true = phantoms.phantom(g, 4, n_abs=(2, 2), radius=(1.2, 1.2), dmua=(0.03, 0.03))
    d = noise.poisson_histogram(op.forward(mu_true), 1e5, 11)
    L_A = float(np.linalg.eigvalsh(J.T @ J)[-1])
    L, lam = solver.step_constants(L_A)
    A = np.vstack([J, math.sqrt(lam) * np.eye(J.shape[1])])
    b = np.concatenate([d.ravel(), np.zeros(J.shape[1])])
    xs = optimize.lsq_linear(A, b, bounds=(0, np.inf), method="bvls", tol=1e-15).x
    F_star = 0.5 * float(np.sum((A @ xs - b) ** 2))
    assert abs(solver.objective(op, d, xs.reshape(g.nz, g.ny, g.nx), lam) / F_star - 1) < 1e-12
    R2 = float(xs @ xs)  # mu_0 = 0
    ks = (1, 2, 3, 5, 10, 20, 50, 100, 200, 500)

    def ratios():
        out = []
        for k in ks:
            mu, _ = solver.fista(op, d, L, lam, k)
            out.append((solver.objective(op, d, mu, lam) - F_star) / (2 * L * R2 / (k + 1) ** 2))
        return np.array(out)

    r = ratios()
    assert np.all(r <= 1.0), r
    assert np.all(r >= -1e-12)
    beta = solver.fista_betas(400)
    assert beta[0] == 0.0 and all(0.0 <= x < 1.0 for x in beta)
    t = [1.0, None]
    # t_2 is the one value not recoverable from beta_1 = 0: the golden ratio
    t[1] = (1.0 + math.sqrt(5.0)) / 2.0
    for k in range(1, 399):
        t.append((t[k] - 1.0) / beta[k])
    for k, tk in enumerate(t[:399], start=1):
        assert tk >= (k + 1) / 2 - 1e-9 and tk <= k + 1e-9
    monkeypatch.setattr(solver, "fista_betas", lambda iters, k0=0: [0.0] * iters)
    r0 = ratios()
    assert np.max(r0) > 1.5, r0


def test_power_iteration_vs_eigvalsh():
    g = small_geometry()
    Kq = kernel.tabulate(g)
    J = operator.jacobian(Kq)
    op = _JOp(J, Kq.shape)
    ev = float(np.linalg.eigvalsh(J.T @ J)[-1])
    est50 = solver.power_iteration(op, 50)
    assert est50 <= ev * (1 + 1e-12) and est50 >= 0.9 * ev
    assert abs(solver.power_iteration(op, 1000) / ev - 1) < 1e-10


def test_fista_betas_closed_form():
    b = solver.fista_betas(5)
    t = [1.0]
    for _ in range(5):
        t.append((1 + math.sqrt(1 + 4 * t[-1] ** 2)) / 2)
    assert b[0] == 0.0
    assert np.allclose(b, [(t[k] - 1) / t[k + 1] for k in range(5)], rtol=0, atol=1e-15)


# -- P14: a single layer is the 2D convolution of Eq. 9 (library routine) ---
def test_p14_single_plane_is_2d_convolution():
    g = small_geometry(n=9, nz=3, nt=6)
    Kq = kernel.tabulate(g)
    rng = np.random.default_rng(5)
    mu = rng.random((g.nz, 9, 9))
    n = 9
    total = np.zeros((g.nt, n, n))
    for z in range(g.nz):
        one = np.zeros_like(mu)
        one[z] = mu[z]
        m_z = operator.forward_direct(Kq, one)
        for k in range(g.nt):
            full = np.zeros((2 * n - 1, 2 * n - 1))
            dy = np.abs(np.arange(-(n - 1), n))
            full[:, :] = Kq[z][dy[:, None], dy[None, :], k]
            conv = signal.convolve2d(mu[z], full, mode="full")[n - 1:2 * n - 1, n - 1:2 * n - 1]
            assert np.max(np.abs(conv - m_z[k])) <= 1e-14 * np.max(np.abs(conv))
        total += m_z
    # Eq. 11: the 3D model is the sum of the per-layer 2D models
    m = operator.forward_direct(Kq, mu)
    assert np.max(np.abs(total - m)) <= 1e-14 * np.max(np.abs(m))


# -- P15: seeded Poisson noise has the stated mean and variance ------------
def test_p15_noise_statistics():
    m = np.full(200000, 2.5e-3)
    m[0] = 5e-3  # the peak bin fixes the scale s = peak / max(m)
    peak = 50.0
    d = noise.poisson_histogram(m, peak, 123)
    s = peak / m.max()
    body = d[1:]
    mean_err = (body.mean() - 2.5e-3) / math.sqrt(2.5e-3 / s / body.size)
    assert abs(mean_err) < 5
    var = body.var()
    # Var of a scaled Poisson is m / s; its sampling sd is about var*sqrt(2/n)
    assert abs(var / (2.5e-3 / s) - 1) < 5 * math.sqrt(2.0 / body.size) + 1e-3
    assert np.array_equal(d, noise.poisson_histogram(m, peak, 123))


def test_phantoms_seeded_and_nonempty():
    for name in ("tiny", "mid", "learned"):
        w = workloads.workload(name)
        g = workloads.geometry_for(name)
        for seed in range(4):
            mu = phantoms.workload_phantom(w, g, seed)
            assert mu.shape == (g.nz, g.ny, g.nx)
            assert mu.min() >= 0 and mu.max() > 0
            assert np.array_equal(mu, phantoms.workload_phantom(w, g, seed))
