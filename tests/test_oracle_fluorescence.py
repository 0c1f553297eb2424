"""Pins of the fluorescence-mode oracle kernel (section "Materials and
Methods": excitation and emission optics, lifetime convolution) against
facts that do not come from it: a brute-force time convolution of the
excitation fluence and the emission flux, the absorption kernel when both
wavelengths share their optics, the Laplace transform of the diffusion
Green's functions (whose value at zero is the CW product of Eq. 4), and a
double-integral evaluation of the lifetime convolution.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import physics as ph

OX = ph.optics(1.0, 0.02, 1.4)   # excitation
OM = ph.optics(0.8, 0.02, 1.4)   # emission: less scattering, same absorption


@pytest.mark.parametrize("rho,z,t", [(0.0, 3.0, 150.0), (2.0, 4.0, 300.0), (5.0, 6.0, 900.0), (1.0, 2.0, 60.0)])
def test_pointwise_equals_brute_force_convolution(rho, z, t):
    # (Phi0_ex (*) R_em)(t) = int_0^t Phi0(s; excitation) R(t - s; emission) ds
    f = lambda s: float(ph.phi0(rho, z, s, OX)) * float(ph.refl(rho, z, t - s, OM))
    ref = integrate.quad(f, 0.0, t, epsabs=0.0, epsrel=1e-11, limit=400)[0]
    got = float(ph.fluorescence_pointwise(rho, z, t, OX, OM))
    assert got == pytest.approx(ref, rel=1e-8)


def test_same_optics_no_lifetime_is_the_absorption_kernel():
    te = np.arange(0, 33) * 40.0
    for rho, z in [(0.0, 2.0), (1.5, 5.0), (4.0, 3.0)]:
        got = ph.fluorescence_bins(rho, z, te, OX, OX, 0.0)
        ref = ph.kernel_bins(rho, z, te, OX)[0]
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def _laplace_product(rho, z, p):
    # Laplace transforms of the two Green's-function sums, written out:
    # fluence exp(-k r)/(4 pi D r) with its negative image, flux
    # (1/4pi) w (k + 1/r) exp(-k r)/r^2 with its image
    kx = math.sqrt((p / OX.c + OX.mua) / OX.D)
    km = math.sqrt((p / OM.c + OM.mua) / OM.D)
    r11 = math.hypot(rho, z - OX.z0)
    r12 = math.hypot(rho, z + OX.z0 + 2 * OX.zb)
    phi = (math.exp(-kx * r11) / r11 - math.exp(-kx * r12) / r12) / (4 * math.pi * OX.D)
    r21 = math.hypot(rho, z)
    r22 = math.hypot(rho, z + 2 * OM.zb)
    refl = sum(w * (km + 1 / r) * math.exp(-km * r) / (r * r) for w, r in ((z, r21), (z + 2 * OM.zb, r22)))
    return phi * refl / (4 * math.pi)


@pytest.mark.parametrize("p", [0.0, 0.002, 0.02])
def test_laplace_transform_of_the_closed_form(p):
    rho, z = 1.5, 4.0
    f = lambda t: float(ph.fluorescence_pointwise(rho, z, t, OX, OM)) * math.exp(-p * t)
    ref = _laplace_product(rho, z, p)
    got = integrate.quad(f, 0.0, np.inf, epsabs=0.0, epsrel=1e-11, limit=400)[0]
    assert got == pytest.approx(ref, rel=1e-8)


def test_lifetime_preserves_the_total_and_the_cw_product():
    # E_tau integrates to one: the bins over a long window add up to the
    # Laplace transform at zero, the product of the CW fluence and flux
    rho, z, tau = 2.0, 5.0, 600.0
    te = np.concatenate([np.arange(0, 20) * 50.0, 1000.0 + np.arange(1, 80) * 500.0])
    got = ph.fluorescence_bins(rho, z, te, OX, OM, tau).sum()
    ref = float(ph.phi0_cw(rho, z, OX)) * float(ph.refl_cw(rho, z, OM))
    assert got == pytest.approx(ref, rel=1e-7)
    assert ref == pytest.approx(_laplace_product(rho, z, 0.0), rel=1e-12)


def test_lifetime_convolution_by_double_integral():
    rho, z, tau = 1.0, 3.0, 500.0
    te = np.array([0.0, 100.0, 250.0, 600.0])
    got = ph.fluorescence_bins(rho, z, te, OX, OM, tau)
    k = lambda s: float(ph.fluorescence_pointwise(rho, z, s, OX, OM))
    for j in range(3):
        lo, hi = te[j], te[j + 1]
        inner = lambda t: integrate.quad(lambda s: k(s) * math.exp(-(t - s) / tau) / tau, 0.0, t,
                                         epsabs=0.0, epsrel=1e-11, limit=200)[0]
        ref = integrate.quad(inner, lo, hi, epsabs=0.0, epsrel=1e-10, limit=200)[0]
        assert got[j] == pytest.approx(ref, rel=1e-8)


def test_long_lifetime_delays_and_short_lifetime_recovers():
    rho, z = 1.0, 3.0
    te = np.arange(0, 41) * 50.0
    k0 = ph.fluorescence_bins(rho, z, te, OX, OM, 0.0)
    short = ph.fluorescence_bins(rho, z, te, OX, OM, 0.05)
    np.testing.assert_allclose(short, k0, rtol=0, atol=2e-3 * k0.max())
    long_ = ph.fluorescence_bins(rho, z, te, OX, OM, 1000.0)
    assert np.argmax(long_) > np.argmax(k0)
