"""Diffusion physics behind the confocal sensitivity kernel (FP64, CPU).

Test infrastructure (see the package header): used only by tests, the smoke
check and the CPU baseline of the benchmark.

Paper: section "Computation of the Sensitivity Matrix".  The CW Jacobian is
the product of the fluence Phi0 from the source and the reflectance R back to
the detector (Eqs. 3-4); the time-resolved Jacobian is their convolution in
time (Eq. 5).  The paper cites, but does not write out, the diffusion
Green's functions.  Readings taken here (semi-infinite homogeneous medium,
refractive index n inside and 1 outside):

* light speed     c = 0.299792458 / n  mm/ps
* diffusion coef. D = 1 / (3 (mu_a + mu_s'))  mm
* pencil beam     isotropic unit point source at depth z0 = 1/(mu_a + mu_s')
* boundary        extrapolated boundary at z = -z_b, z_b = 2 A D with
                  A = (1 + R_eff)/(1 - R_eff),
                  R_eff = -1.440/n^2 + 0.710/n + 0.668 + 0.0636 n
* infinite medium G(r, t) = c (4 pi D c t)^(-3/2) exp(-r^2/(4 D c t) - mu_a c t)
* Phi0            G(r11, t) - G(r12, t): source at z0, negative image at
                  -(z0 + 2 z_b)
* R               outward flux D dPhi/dz at the surface from a unit point
                  source at the voxel (reciprocity), with its own image
* Phi0 (*)_t R    the exact continuous convolution (closed form below),
                  not a discrete convolution of binned curves
* near source     the source-to-voxel distance is floored at r_min, the
                  radius of a sphere of one voxel's volume

Closed form of the convolution.  In Laplace space the infinite-medium
Green's function is exp(-kappa r)/(4 pi D r) with
kappa = sqrt((s/c + mu_a)/D), and the reflectance is
(1/4pi) sum_j w_j (kappa + 1/r2_j) exp(-kappa r2_j)/r2_j^2.  Their product
is a sum of exp(-kappa a) and kappa exp(-kappa a) terms with a = r1_i + r2_j,
whose inverse transforms are elementary, giving

  k(t) = sum_ij sigma_i w_j / (16 pi^2 D r1_i r2_j^2) / (2 sqrt(pi D c))
         * t^(-3/2) exp(-a^2/(4 D c t) - mu_a c t) * (a^2/(2 D c t) - 1 + a/r2_j)

with sigma = (+1, -1) for source and image, w = (z, z + 2 z_b),
r1 = distances from source / image to the voxel, r2 = from the voxel / its
image to the detector.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import special

C0_MM_PER_PS = 0.299792458


@dataclasses.dataclass(frozen=True)
class Optics:
    c: float       # mm/ps
    D: float       # mm
    z0: float      # mm
    reff: float
    A: float
    zb: float      # mm
    mua: float     # 1/mm
    mueff: float   # 1/mm


def optics(mus_prime: float, mua: float, n: float) -> Optics:
    c = C0_MM_PER_PS / n
    D = 1.0 / (3.0 * (mua + mus_prime))
    z0 = 1.0 / (mua + mus_prime)
    reff = -1.440 / (n * n) + 0.710 / n + 0.668 + 0.0636 * n
    A = (1.0 + reff) / (1.0 - reff)
    zb = 2.0 * A * D
    mueff = math.sqrt(mua / D)
    return Optics(c=c, D=D, z0=z0, reff=reff, A=A, zb=zb, mua=mua, mueff=mueff)


# --- time-domain Green's functions (Eqs. 3-5 ingredients) -----------------

def green_inf(r, t, o: Optics):
    """Fluence rate at distance r, time t from a unit-energy isotropic pulse."""
    r = np.asarray(r, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    tt = np.where(t > 0, t, 1.0)
    val = o.c * (4 * np.pi * o.D * o.c * tt) ** -1.5 * np.exp(
        -r * r / (4 * o.D * o.c * tt) - o.mua * o.c * tt)
    return np.where(t > 0, val, 0.0)


def source_distances(rho, z, o: Optics):
    r11 = np.sqrt(rho * rho + (z - o.z0) ** 2)
    r12 = np.sqrt(rho * rho + (z + o.z0 + 2 * o.zb) ** 2)
    return r11, r12


def detector_distances(rho, z, o: Optics):
    r21 = np.sqrt(rho * rho + z * z)
    r22 = np.sqrt(rho * rho + (z + 2 * o.zb) ** 2)
    return r21, r22


def phi0(rho, z, t, o: Optics):
    """Fluence at voxel (lateral offset rho, depth z) from the pencil beam."""
    r11, r12 = source_distances(rho, z, o)
    return green_inf(r11, t, o) - green_inf(r12, t, o)


def refl(rho, z, t, o: Optics):
    """Surface flux at lateral offset rho from a unit pulse at depth z."""
    t = np.asarray(t, dtype=np.float64)
    tt = np.where(t > 0, t, 1.0)
    fourDct = 4 * o.D * o.c * tt
    zi = z + 2 * o.zb
    val = (0.5 * (4 * np.pi * o.D * o.c) ** -1.5 * tt ** -2.5
           * np.exp(-o.mua * o.c * tt - rho * rho / fourDct)
           * (z * np.exp(-z * z / fourDct) + zi * np.exp(-zi * zi / fourDct)))
    return np.where(t > 0, val, 0.0)


# --- continuous-wave forms (Eq. 4) -----------------------------------------

def green_inf_cw(r, o: Optics):
    return np.exp(-o.mueff * r) / (4 * np.pi * o.D * r)


def phi0_cw(rho, z, o: Optics):
    r11, r12 = source_distances(rho, z, o)
    return green_inf_cw(r11, o) - green_inf_cw(r12, o)


def refl_cw(rho, z, o: Optics):
    r21, r22 = detector_distances(rho, z, o)
    out = 0.0
    for w, r in ((z, r21), (z + 2 * o.zb, r22)):
        out = out + w * (o.mueff + 1.0 / r) * np.exp(-o.mueff * r) / (r * r)
    return out / (4 * np.pi)


# --- the exact time convolution Phi0 (*)_t R (Eq. 5) ------------------------

def _terms(rho, z, o: Optics, r_min: float):
    """The four image terms: (sigma_i w_j / (16 pi^2 D r1_i r2_j^2), a_ij, r2_j)."""
    r11, r12 = source_distances(rho, z, o)
    r11 = np.maximum(r11, r_min)
    r21, r22 = detector_distances(rho, z, o)
    out = []
    for sigma, r1 in ((1.0, r11), (-1.0, r12)):
        for w, r2 in ((z, r21), (z + 2 * o.zb, r22)):
            amp = sigma * w / (16 * np.pi ** 2 * o.D * r1 * r2 * r2)
            out.append((amp, r1 + r2, r2))
    return out


def kernel_pointwise(rho, z, t, o: Optics, r_min: float = 0.0):
    """k(rho, z, t) = (Phi0 (*)_t R)(t) in closed form (module header)."""
    t = np.asarray(t, dtype=np.float64)
    tt = np.where(t > 0, t, 1.0)
    Dc = o.D * o.c
    norm = 1.0 / (2.0 * math.sqrt(math.pi * Dc))
    total = 0.0
    for amp, a, r2 in _terms(rho, z, o, r_min):
        total = total + amp * norm * tt ** -1.5 * np.exp(
            -a * a / (4 * Dc * tt) - o.mua * o.c * tt) * (
            a * a / (2 * Dc * tt) - 1.0 + a / r2)
    return np.where(t > 0, total, 0.0)


def _antiderivative(alpha, beta, g, T):
    """F(T) = int_0^T s^(-3/2) exp(-alpha/s - beta s) (2 alpha/s + g - 1) ds.

    Uses d/ds [2 e(s)/sqrt(s)] = (2 alpha/s - 1) s^(-3/2) e(s) - 2 beta s^(-1/2) e(s),
    so F = 2 e(T)/sqrt(T) + g I_{3/2}(T) + 2 beta I_{1/2}(T) with the
    incomplete integrals I_nu(T) = int_0^T s^(-nu) e(s) ds written through
    the scaled complementary error function (no overflow, no cancellation
    in the dominant terms).
    """
    T = np.asarray(T, dtype=np.float64)
    pos = T > 0
    Ts = np.where(pos, T, 1.0)
    x = np.sqrt(alpha / Ts)
    y = np.sqrt(beta * Ts)
    E = np.exp(-x * x - y * y)
    ep = E * special.erfcx(x + y)
    em = np.where(x >= y, E * special.erfcx(np.where(x >= y, x - y, 0.0)),
                  np.exp(-2 * x * y) * special.erfc(x - y))
    i32 = math.sqrt(math.pi) / (2 * np.sqrt(alpha)) * (em + ep)
    i12 = math.sqrt(math.pi) / (2 * np.sqrt(beta)) * (em - ep)
    F = 2 * E / np.sqrt(Ts) + g * i32 + 2 * beta * i12
    return np.where(pos, F, 0.0)


_GL_X, _GL_W = np.polynomial.legendre.leggauss(16)


def _integrand(alpha, beta, g, s):
    return s ** -1.5 * np.exp(-alpha / s - beta * s) * (2 * alpha / s + g - 1.0)


def kernel_bins(rho, z, t_edges, o: Optics, r_min: float = 0.0):
    """Integral of k(rho, z, t) over each time bin [t_edges[k], t_edges[k+1]).

    ``rho`` may be an array (one row per value); returns [len(rho), nbins].
    Per image term, the exact antiderivative difference F(hi) - F(lo) is used
    while F(lo) <= 100 |F(hi) - F(lo)|; later bins, where that difference
    would cancel, use 16-point Gauss-Legendre on the closed-form integrand.
    """
    rho = np.atleast_1d(np.asarray(rho, dtype=np.float64))[:, None]
    te = np.asarray(t_edges, dtype=np.float64)[None, :]
    Dc = o.D * o.c
    beta = o.mua * o.c
    norm = 1.0 / (2.0 * math.sqrt(math.pi * Dc))
    lo = te[:, :-1]
    hi = te[:, 1:]
    half = 0.5 * (hi - lo)
    mid = 0.5 * (hi + lo)
    total = np.zeros((rho.shape[0], te.shape[1] - 1))
    for amp, a, r2 in _terms(rho, z, o, r_min):
        alpha = a * a / (4 * Dc)
        g = a / r2
        F = _antiderivative(alpha, beta, g, te)
        Flo, Fhi = F[:, :-1], F[:, 1:]
        dF = Fhi - Flo
        gl = np.zeros_like(dF)
        for xg, wg in zip(_GL_X, _GL_W):
            gl = gl + wg * _integrand(alpha, beta, g, mid + half * xg)
        gl = gl * half
        exact_ok = Flo <= 100.0 * np.abs(dF)
        total = total + amp * norm * np.where(exact_ok, dF, gl)
    return total


def kernel_total(rho, z, o: Optics, r_min: float = 0.0):
    """Integral of k over all t > 0: sum_ij amp * norm * F(infinity)."""
    Dc = o.D * o.c
    norm = 1.0 / (2.0 * math.sqrt(math.pi * Dc))
    total = 0.0
    for amp, a, r2 in _terms(np.asarray(rho, dtype=np.float64), z, o, r_min):
        # F(inf) = 2 sqrt(pi D c) exp(-mu_eff a) (mu_eff + 1/r2)
        total = total + amp * norm * 2 * math.sqrt(math.pi * Dc) * np.exp(
            -o.mueff * a) * (o.mueff + 1.0 / r2)
    return total


# --- fluorescence mode ------------------------------------------------------
#
# Paper: section "Materials and Methods" (simulation setup): fluorescence
# needs the optical properties of the excitation and of the emission
# wavelength, and the time-resolved signal convolved with an exponential of
# the fluorophore's lifetime.  Readings: the excitation fluence Phi0 uses
# the excitation optics (source depth, boundary, D), the emission flux R the
# emission optics; the two share the refractive index and the background
# absorption mu_a; the lifetime enters as E_tau(t) = exp(-t/tau)/tau, so the
# sensitivity of the emission histogram to the fluorophore yield of a voxel
# is W = Phi0_ex (*)_t E_tau (*)_t R_em.  With a shared mu_a the two
# diffusion wavenumbers are proportional, kappa_ex = kappa_em sqrt(D_em/D_ex),
# so the Laplace-domain product keeps one exponential exp(-kappa_em a) with
# a = r1 sqrt(D_em/D_ex) + r2 and amplitude w / (16 pi^2 D_ex r1 r2^2): the
# same inverse transform as in the absorption case with D = D_em.

def fluorescence_terms(rho, z, ox: Optics, om: Optics, r_min: float = 0.0):
    """Image terms (amplitude, a, r2) of Phi0_ex (*)_t R_em."""
    r11 = np.maximum(np.sqrt(rho * rho + (z - ox.z0) ** 2), r_min)
    r12 = np.sqrt(rho * rho + (z + ox.z0 + 2 * ox.zb) ** 2)
    r21 = np.sqrt(rho * rho + z * z)
    r22 = np.sqrt(rho * rho + (z + 2 * om.zb) ** 2)
    scale = math.sqrt(om.D / ox.D)
    out = []
    for sigma, r1 in ((1.0, r11), (-1.0, r12)):
        for w, r2 in ((z, r21), (z + 2 * om.zb, r22)):
            amp = sigma * w / (16 * np.pi ** 2 * ox.D * r1 * r2 * r2)
            out.append((amp, r1 * scale + r2, r2))
    return out


def fluorescence_pointwise(rho, z, t, ox: Optics, om: Optics, r_min: float = 0.0):
    """(Phi0_ex (*)_t R_em)(t) in closed form (no lifetime)."""
    t = np.asarray(t, dtype=np.float64)
    tt = np.where(t > 0, t, 1.0)
    Dc = om.D * om.c
    norm = 1.0 / (2.0 * math.sqrt(math.pi * Dc))
    total = 0.0
    for amp, a, r2 in fluorescence_terms(rho, z, ox, om, r_min):
        total = total + amp * norm * tt ** -1.5 * np.exp(
            -a * a / (4 * Dc * tt) - om.mua * om.c * tt) * (a * a / (2 * Dc * tt) - 1.0 + a / r2)
    return np.where(t > 0, total, 0.0)


def fluorescence_bins(rho, z, t_edges, ox: Optics, om: Optics, tau: float, r_min: float = 0.0):
    """Bin integrals of W = Phi0_ex (*) E_tau (*) R_em over [t_edges[k], t_edges[k+1]).

    tau == 0: adaptive quadrature of the pointwise closed form over each bin.
    tau > 0: int_bin (k (*) E_tau)(t) dt = int_0^hi k(s) w(s) ds with the
    exact weight w(s) = exp(-(max(lo, s) - s)/tau) - exp(-(hi - s)/tau),
    integrated adaptively with breakpoints at the bin edges.
    """
    from scipy import integrate
    te = np.asarray(t_edges, dtype=np.float64)
    out = np.zeros(len(te) - 1)
    f = lambda s: float(fluorescence_pointwise(rho, z, s, ox, om, r_min))
    # time of the peak of the first image term helps the adaptive rule
    a0 = fluorescence_terms(rho, z, ox, om, r_min)[0][1]
    t_peak = a0 * a0 / (6 * om.D * om.c)
    for k in range(len(te) - 1):
        lo, hi = te[k], te[k + 1]
        if tau == 0.0:
            pts = [p for p in (t_peak,) if lo < p < hi]
            out[k] = integrate.quad(f, lo, hi, points=pts or None, epsabs=0.0, epsrel=1e-12, limit=400)[0]
            continue

        def wk(s, lo=lo, hi=hi):
            return f(s) * (math.exp(-(max(lo, s) - s) / tau) - math.exp(-(hi - s) / tau))
        pts = sorted(p for p in (t_peak, lo) if 0.0 < p < hi)
        out[k] = integrate.quad(wk, 0.0, hi, points=pts or None, epsabs=0.0, epsrel=1e-12, limit=800)[0]
    return out
