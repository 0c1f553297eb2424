"""Pins of the oracle's per-layer L1 objective (paper Eqs. 8 and 10).

FISTA with the L1 prox is checked against an independent solver of the same
problem (scipy L-BFGS-B: with mu >= 0 the L1 term is linear, so the
objective is a smooth bound-constrained QP), against the optimality (KKT)
conditions, and against plain FISTA when the weights are zero; the layer
energy against the squared column norm from the explicit Jacobian; the
layer-wise threshold against a hand-built example.
"""

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import kernel as okernel
from oracle import operator as oop
from oracle import solver as osolver
from synth import noise, phantoms, workloads


@pytest.fixture(scope="module")
def tiny():
    g = workloads.geometry_for("tiny")
    K = okernel.tabulate(g)
    F = oop.FFTOperator(K)
    w = workloads.workload("tiny")
    mu = phantoms.workload_phantom(w, g, 3)
    d = noise.poisson_histogram(F.forward(mu), 1e5, 4)
    LA = osolver.power_iteration(F, 50)
    L, lam = osolver.step_constants(LA)
    return g, K, F, d, L, lam


def _l1(F, d, frac=0.05):
    # depth weights proportional to each layer's sensitivity, scaled to a
    # fraction of the data's back-projection
    e = osolver.layer_energy(F)
    top = float(np.max(F.adjoint(d)))
    return frac * top * e / e.max()


@pytest.fixture(scope="module")
def solved(tiny):
    g, K, F, d, L, lam = tiny
    l1 = _l1(F, d)
    mu, hist = osolver.fista(F, d, L, lam, 20000, l1=l1)
    return l1, mu, hist


def test_l1_fista_matches_bound_constrained_qp(tiny, solved):
    g, K, F, d, L, lam = tiny
    l1, mu, hist = solved
    shape = mu.shape
    w1 = l1[:, None, None]

    # variables and objective scaled to order one (mu = s x, F / c) so that
    # L-BFGS-B's absolute tolerances mean something
    s = float(np.max(F.adjoint(d))) / L
    c = 0.5 * float(np.vdot(d, d))

    def fun(x):
        m = s * x.reshape(shape)
        r = F.forward(m) - d
        val = 0.5 * np.vdot(r, r) + 0.5 * lam * np.vdot(m, m) + np.sum(w1 * m)
        grad = F.adjoint(r) + lam * m + w1
        return float(val) / c, (s / c) * grad.ravel()

    res = minimize(fun, np.zeros(mu.size), jac=True, method="L-BFGS-B", bounds=[(0.0, None)] * mu.size,
                   options=dict(maxiter=50000, maxfun=100000, ftol=1e-16, gtol=1e-14, maxcor=50))
    ref = s * res.x.reshape(shape)
    f_fista = osolver.objective(F, d, mu, lam, l1)
    f_ref = osolver.objective(F, d, ref, lam, l1)
    assert f_fista <= f_ref * (1 + 1e-9)
    assert np.linalg.norm(mu - ref) <= 1e-4 * np.linalg.norm(ref)



def test_uniform_l1_sparsifies(tiny):
    g, K, F, d, L, lam = tiny
    top = float(np.max(F.adjoint(d)))
    plain, _ = osolver.fista(F, d, L, lam, 3000)
    counts = [np.count_nonzero(osolver.fista(F, d, L, lam, 3000, l1=f * top * np.ones(g.nz))[0])
              for f in (1e-3, 1e-2, 5e-2)]
    assert counts[0] < np.count_nonzero(plain) and counts[1] < counts[0] and counts[2] < counts[1]


def test_l1_fista_kkt(tiny, solved):
    g, K, F, d, L, lam = tiny
    l1, mu, hist = solved
    grad = F.adjoint(F.forward(mu) - d) + lam * mu + l1[:, None, None]
    scale = np.max(np.abs(F.adjoint(d)))
    pos = mu > 1e-12 * np.max(mu)
    assert np.max(np.abs(grad[pos])) <= 1e-6 * scale
    assert np.min(grad[~pos]) >= -1e-6 * scale
    assert hist[-1, 1] <= 1e-6


def test_zero_l1_weights_are_plain_fista(tiny):
    g, K, F, d, L, lam = tiny
    a, ha = osolver.fista(F, d, L, lam, 40)
    b, hb = osolver.fista(F, d, L, lam, 40, l1=np.zeros(g.nz))
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ha, hb)


def test_l1_gmap_denominator(tiny):
    g, K, F, d, L, lam = tiny
    l1 = _l1(F, d)
    # one FISTA step from zero: rho_1 = 1 by definition of the denominator
    _, hist = osolver.fista(F, d, L, lam, 1, l1=l1)
    assert hist[0, 1] == pytest.approx(1.0, rel=1e-12)


def test_layer_energy_is_jacobian_column_norm(tiny):
    g, K, F, d, L, lam = tiny
    e = osolver.layer_energy(F)
    J = oop.jacobian(K)  # [nt * ny * nx, nz * ny * nx]
    n = g.nx
    for z in range(g.nz):
        col = J[:, (z * n + n // 2) * n + n // 2]
        assert e[z] == pytest.approx(float(col @ col), rel=1e-12)
    # sensitivity falls with depth
    assert np.all(np.diff(e) < 0)


def test_layer_threshold_example():
    mu = np.zeros((2, 2, 3))
    mu[0] = [[1.0, 0.2, 0.05], [0.5, 0.09, 0.11]]
    mu[1] = [[0.0, 0.02, 0.019], [0.001, 0.0, 0.0]]
    out = osolver.layer_threshold(mu, 0.1)
    np.testing.assert_array_equal(out[0], [[1.0, 0.2, 0.0], [0.5, 0.0, 0.11]])
    np.testing.assert_array_equal(out[1], [[0.0, 0.02, 0.019], [0.0, 0.0, 0.0]])
