"""Step size and FISTA for the regularised least-squares problem (FP64, CPU).

Test infrastructure (see the package header).

Paper: section "Reconstruction Algorithm" poses the reconstruction as a
convex regularised least-squares problem (Eqs. 7-8) solved with FISTA
(Beck and Teboulle); Eq. 10 adds per-depth weights.  Readings:

* objective  F(mu) = 1/2 ||A mu - d||^2 + (lam/2) ||mu||^2,  mu >= 0
  (squared data term so that FISTA's smooth part is differentiable;
  Tikhonov plus non-negativity as in the workloads);
* Lipschitz constant L = 1.01 L_A + lam with L_A = ||A||^2 from 50 power
  iterations of A^T A started at the normalised all-ones vector, the
  estimate being the Rayleigh quotient of the last normalised iterate;
  lam = 1e-3 L_A unless given; step tau = 1 / L;
* FISTA with constant step and no restart:
      y_1 = mu_0,  t_1 = 1
      mu_k = max(0, y_k - tau (A^T (A y_k - d) + lam y_k))
      t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
      y_{k+1} = mu_k + ((t_k - 1) / t_{k+1}) (mu_k - mu_{k-1})
* convergence measure: the gradient-mapping ratio
      rho_k = ||y_k - mu_k|| / (tau ||G(0)||),  ||G(0)|| = ||max(0, A^T d)||,
  the same denominator for any starting point;
* optionally the paper's sparsity term with per-layer weights (Eqs. 8 and
  10): F gains sum_z l1_z ||mu_z||_1.  With mu >= 0 its prox subtracts
  tau l1_z before the clamp,
      mu_k = max(0, y_k - tau (grad f(y_k) + l1_z)),
  and the gradient mapping at zero becomes ||max(0, A^T d - l1_z)||;
* the layer-wise threshold applied to a result: values of layer z below
  frac * max |mu_z| are set to zero (a reading of the paper's
  post-processing of its 3D reconstructions; the rule is not stated).
"""

from __future__ import annotations

import math

import numpy as np


def power_iteration(op, iters: int = 50):
    nz, n_y, n_x, nt = op.shape
    v = np.ones((nz, n_y, n_x))
    v /= np.linalg.norm(v)
    rq = 0.0
    for _ in range(iters):
        w = op.adjoint(op.forward(v))
        rq = float(np.vdot(v, w))
        v = w / np.linalg.norm(w)
    return rq


def step_constants(L_A: float, lam: float | None = None):
    if lam is None or lam < 0:
        lam = 1e-3 * L_A
    L = 1.01 * L_A + lam
    return L, lam


def fista_betas(iters: int, k0: int = 0):
    """beta_k = (t_k - 1) / t_{k+1} for k = 1..iters (t_1 = 1)."""
    t = 1.0
    out = []
    for _ in range(k0 + iters):
        tn = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        out.append((t - 1.0) / tn)
        t = tn
    return out[k0:]


def _layers(l1, nz):
    if l1 is None:
        return 0.0
    w = np.asarray(l1, dtype=np.float64)
    assert w.shape == (nz,)
    return w[:, None, None]


def gmap_denominator(op, d, l1=None) -> float:
    nz = op.shape[0]
    return float(np.linalg.norm(np.maximum(0.0, op.adjoint(d) - _layers(l1, nz))))


def fista(op, d, L: float, lam: float, iters: int, mu0=None, l1=None):
    """Run FISTA; returns (mu, history) with history[k] = (datafit(y_k), rho_k).
    l1: per-layer L1 weights (nz numbers) or None."""
    nz, n_y, n_x, nt = op.shape
    tau = 1.0 / L
    w1 = _layers(l1, nz)
    mu = np.zeros((nz, n_y, n_x)) if mu0 is None else np.array(mu0, dtype=np.float64)
    mu_prev = mu.copy()
    y = mu.copy()
    g0 = gmap_denominator(op, d, l1)
    hist = []
    for beta in fista_betas(iters):
        r = op.forward(y) - d
        datafit = 0.5 * float(np.vdot(r, r))
        grad = op.adjoint(r) + lam * y
        mu = np.maximum(0.0, y - tau * (grad + w1))
        gm = float(np.linalg.norm(y - mu)) / (tau * g0) if g0 > 0 else 0.0
        hist.append((datafit, gm))
        y = mu + beta * (mu - mu_prev)
        mu_prev = mu
    return mu, np.array(hist)


def objective(op, d, mu, lam: float, l1=None) -> float:
    r = op.forward(mu) - d
    f = 0.5 * float(np.vdot(r, r)) + 0.5 * lam * float(np.vdot(mu, mu))
    if l1 is not None:
        f += float(np.sum(_layers(l1, mu.shape[0]) * np.abs(mu)))
    return f


def layer_threshold(mu, frac: float):
    """Zero the values of each layer below frac times its maximum magnitude."""
    mu = np.array(mu, dtype=np.float64)
    m = np.abs(mu).reshape(mu.shape[0], -1).max(axis=1)
    mu[np.abs(mu) < frac * m[:, None, None]] = 0.0
    return mu


def layer_energy(op):
    """||A e_z||^2 for a unit absorber at the window centre of each layer."""
    nz, n_y, n_x, _ = op.shape
    out = np.zeros(nz)
    for z in range(nz):
        e = np.zeros((nz, n_y, n_x))
        e[z, n_y // 2, n_x // 2] = 1.0
        m = op.forward(e)
        out[z] = float(np.vdot(m, m))
    return out


def datafit(op, d, mu) -> float:
    r = op.forward(mu) - d
    return 0.5 * float(np.vdot(r, r))
