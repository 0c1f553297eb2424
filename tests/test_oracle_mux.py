"""Pins of the multiplexing oracle (paper Eq. 12 and section "Advantages of
Multiplexing") against facts that do not come from it: an independent
Hadamard construction, a hand-worked tile example, the adjoint identity,
the exact reduction of a Hadamard-multiplexed solve to the unmultiplexed
one, the non-negative least-squares solution of a small composite problem,
and the first two moments of the dark-count noise.
"""

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

from oracle import kernel as okernel
from oracle import mux as omux
from oracle import operator as oop
from oracle import rng as orng
from oracle import solver as osolver
from synth import phantoms
from synth.workloads import Geometry, even_layers


@pytest.mark.parametrize("order", [1, 2, 4, 8, 16, 64])
def test_sylvester_matches_scipy_and_is_orthogonal(order):
    h = omux.sylvester_hadamard(order)
    np.testing.assert_array_equal(h, scipy.linalg.hadamard(order).astype(np.float64))
    np.testing.assert_array_equal(h @ h.T, order * np.eye(order))


def test_two_polarity_patterns():
    h = omux.sylvester_hadamard(16)
    s = omux.two_polarity(h)
    assert s.shape == (32, 16)
    assert set(np.unique(s)) == {0.0, 1.0}
    np.testing.assert_array_equal(s[:16] - s[16:], h)
    np.testing.assert_array_equal(s[:16] + s[16:], np.ones((16, 16)))


def test_forward_hand_example():
    # 2 x 2 scan, tiles of 2 x 1 (two tiles, one per row), S of 3 x 2:
    # tile 0 holds positions (0,0),(0,1) = 1, 10; tile 1 holds 100, 1000.
    S = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    m = np.array([[[1.0, 10.0], [100.0, 1000.0]]])
    y = omux.forward(S, m, tile_x=2, tile_y=1)
    assert y.shape == (1, 3, 2)
    np.testing.assert_array_equal(y[0, :, 0], [21.0, 43.0, 65.0])
    np.testing.assert_array_equal(y[0, :, 1], [2100.0, 4300.0, 6500.0])
    # tiles of 1 x 2 (two tiles, one per column): (0,0),(1,0) = 1, 100
    y = omux.forward(S, m, tile_x=1, tile_y=2)
    np.testing.assert_array_equal(y[0, :, 0], [201.0, 403.0, 605.0])
    np.testing.assert_array_equal(y[0, :, 1], [2010.0, 4030.0, 6050.0])


def test_identity_gather_matches_reshape():
    # with S = I the forward is a pure gather; compare with a reshape route
    rng = np.random.default_rng(3)
    nt, n, tx, ty = 5, 12, 4, 3
    m = rng.standard_normal((nt, n, n))
    y = omux.forward(np.eye(tx * ty), m, tx, ty)
    ref = m.reshape(nt, n // ty, ty, n // tx, tx).transpose(0, 1, 3, 2, 4).reshape(nt, -1, ty * tx)
    np.testing.assert_array_equal(y, ref.transpose(0, 2, 1))
    pos = omux.tile_positions(n, tx, ty)
    np.testing.assert_array_equal(np.sort(pos.ravel()), np.arange(n * n))


@pytest.mark.parametrize("ny,nx,tx,ty", [(6, 12, 4, 3), (12, 4, 2, 4), (3, 10, 5, 1)])
def test_rectangular_gather_matches_reshape(ny, nx, tx, ty):
    # a ny x nx grid: the tiles partition it, and with S = I the forward is
    # the same reshape gather as on a square grid, tiles row by row
    rng = np.random.default_rng(ny * 100 + nx)
    nt = 4
    m = rng.standard_normal((nt, ny, nx))
    y = omux.forward(np.eye(tx * ty), m, tx, ty)
    ref = m.reshape(nt, ny // ty, ty, nx // tx, tx).transpose(0, 1, 3, 2, 4).reshape(nt, -1, ty * tx)
    np.testing.assert_array_equal(y, ref.transpose(0, 2, 1))
    pos = omux.tile_positions(ny, tx, ty, nx)
    np.testing.assert_array_equal(np.sort(pos.ravel()), np.arange(ny * nx))
    S = rng.standard_normal((7, tx * ty))
    yy = rng.standard_normal((nt, 7, (nx // tx) * (ny // ty)))
    lhs = np.vdot(omux.forward(S, m, tx, ty), yy)
    rhs = np.vdot(m, omux.adjoint(S, yy, tx, ty, ny, nx))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_adjoint_identity():
    rng = np.random.default_rng(4)
    nt, n, tx, ty, M = 3, 8, 4, 2, 13
    S = rng.standard_normal((M, tx * ty))
    m = rng.standard_normal((nt, n, n))
    y = rng.standard_normal((nt, M, (n // tx) * (n // ty)))
    lhs = np.vdot(omux.forward(S, m, tx, ty), y)
    rhs = np.vdot(m, omux.adjoint(S, y, tx, ty, n))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def _small(seed, n=8, nz=3, nt=32):
    z, dz = even_layers(2.0, 10.0, nz)
    g = Geometry(nx=n, ny=n, pitch_mm=1.0, z_mm=z, dz_mm=dz, nt=nt, dt_ps=50.0)
    Kq = okernel.tabulate(g)
    F = oop.FFTOperator(Kq)
    mu = phantoms.phantom(g, seed, n_abs=(1, 2), radius=(1.0, 2.0), dmua=(0.02, 0.05), kinds=("sphere",))
    return g, Kq, F, mu


def test_hadamard_solve_reduces_to_demultiplexed_solve():
    # S^T S = P I makes 1/2||S A mu - y||^2 = P/2 ||A mu - S^T y / P||^2 + const,
    # so FISTA with (P L, lam) on S A follows FISTA with (L, lam / P) on A.
    g, Kq, F, mu = _small(5)
    H = omux.sylvester_hadamard(16)
    Fm = omux.MuxOperator(F, H, 4, 4)
    y = Fm.forward(mu) + 1e-3 * np.random.default_rng(6).standard_normal((g.nt, 16, 4)) * np.abs(
        Fm.forward(mu)).max()
    LA = osolver.power_iteration(F, 50)
    LAm = osolver.power_iteration(Fm, 50)
    assert LAm == pytest.approx(16 * LA, rel=1e-12)
    L, lam = osolver.step_constants(LA)
    mu_m, h_m = osolver.fista(Fm, y, 16 * L, lam, 60)
    m_tilde = omux.adjoint(H, y, 4, 4, g.nx) / 16
    mu_p, h_p = osolver.fista(F, m_tilde, L, lam / 16, 60)
    scale = np.abs(mu_p).max()
    np.testing.assert_allclose(mu_m, mu_p, rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(h_m[:, 1], h_p[:, 1], rtol=1e-9)


def test_composite_solve_reaches_nnls_solution():
    # a non-orthogonal S (the stacked on/off patterns): FISTA's limit is the
    # non-negative least-squares solution of [S J; sqrt(lam) I] mu = [y; 0]
    g, Kq, F, mu = _small(7, n=4, nz=2, nt=16)
    S = omux.two_polarity(omux.sylvester_hadamard(4))
    Fm = omux.MuxOperator(F, S, 2, 2)
    y = Fm.forward(mu)
    y = y + 0.02 * np.abs(y).max() * np.random.default_rng(8).standard_normal(y.shape)
    J = oop.jacobian(Kq)
    # rows of S J in the (t, i, g) order of y
    SJ = np.stack([Fm.forward(e.reshape(mu.shape)) for e in np.eye(mu.size)], axis=-1).reshape(-1, mu.size)
    # the same composite from the explicit Jacobian, without the operator
    pos = omux.tile_positions(g.nx, 2, 2)
    Jt = J.reshape(g.nt, g.nx * g.nx, -1)
    SJ2 = np.einsum("ij,tgjk->tigk", S, Jt[:, pos, :]).reshape(-1, mu.size)
    np.testing.assert_allclose(SJ, SJ2, rtol=1e-12, atol=1e-12 * np.abs(SJ2).max())
    LA = osolver.power_iteration(Fm, 200)
    assert LA == pytest.approx(np.linalg.norm(SJ2, 2) ** 2, rel=1e-6)
    L, lam = osolver.step_constants(LA)
    mu_f, _ = osolver.fista(Fm, y, L, lam, 12000)
    Aug = np.vstack([SJ2, np.sqrt(lam) * np.eye(mu.size)])
    ref, _ = scipy.optimize.nnls(Aug, np.concatenate([y.ravel(), np.zeros(mu.size)]), maxiter=10000)
    np.testing.assert_allclose(mu_f.ravel(), ref, rtol=0, atol=1e-8 * np.abs(ref).max())


def test_dark_count_noise_moments():
    # zero signal: counts are Poisson(b), so (c - b)/s has mean 0 and
    # variance b / s^2; with signal, the mean is m
    n = 200000
    m = np.zeros(n, dtype=np.float32)
    m[n // 2:] = 3.0
    s, b = 2.0, 7.5
    d = orng.noisy_counts(m, s, b, seed=11).astype(np.float64)
    lo, hi = d[: n // 2], d[n // 2:]
    se0 = np.sqrt(b / s ** 2 / lo.size)
    assert abs(lo.mean()) < 5 * se0
    assert lo.var() == pytest.approx(b / s ** 2, rel=0.03)
    se1 = np.sqrt((s * 3.0 + b) / s ** 2 / hi.size)
    assert abs(hi.mean() - 3.0) < 5 * se1
    assert hi.var() == pytest.approx((s * 3.0 + b) / s ** 2, rel=0.03)
    # counts are integers: (d s + b) is integral
    c = d * s + b
    np.testing.assert_allclose(c, np.round(c), atol=1e-3)


def test_dark_count_noise_without_background_is_plain_poisson():
    rng = np.random.default_rng(12)
    m = rng.uniform(0, 5, 5000).astype(np.float32)
    d = orng.noisy_counts(m, 3.0, 0.0, seed=13, stream=2)
    c = orng.poisson_sample(np.maximum(m.astype(np.float64), 0) * 3.0, 13, 2)
    np.testing.assert_array_equal(d, (c / 3.0).astype(np.float32))
