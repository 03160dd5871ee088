"""Pins for the oracle's SPH kernels (CPU).

* Normalisation: the kernel integrates to one over its support (Sec. 2.3,
  kernel-normalisation equation), checked by adaptive quadrature -- independent
  of the exact rational arithmetic the oracle uses for the Wendland constant.
* dW/dr agrees with a central finite difference of W.
* dW/dr <= 0 (so the Brookshaw pair weight F_ij is non-negative) and W, dW/dr
  vanish at the edge of the support (so the strictness of the neighbour
  predicate cannot change any operator entry).
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import kernels

SURFACE = {1: 2.0, 2: 2.0 * math.pi, 3: 4.0 * math.pi}
CASES = [(d, k) for d in (1, 2, 3) for k in (kernels.CUBIC_SPLINE, kernels.WENDLAND_C4)]


@pytest.mark.parametrize("dim,kern", CASES)
def test_normalisation_by_quadrature(dim, kern):
    h = 0.37
    kappa = kernels.KAPPA[kern]
    f = lambda r: float(kernels.W(r, h, dim, kern)) * SURFACE[dim] * r ** (dim - 1)
    val, err = integrate.quad(f, 0.0, kappa * h, points=[h] if kappa > 1 else None,
                              epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-11


@pytest.mark.parametrize("dim,kern", CASES)
def test_derivative_matches_finite_difference(dim, kern):
    h = 0.8
    rng = np.random.default_rng(5)
    r = rng.uniform(0.01, kernels.KAPPA[kern] * h - 0.01, 200)
    eps = 1e-6
    fd = (kernels.W(r + eps, h, dim, kern) - kernels.W(r - eps, h, dim, kern)) / (2 * eps)
    an = kernels.dWdr(r, h, dim, kern)
    assert np.allclose(fd, an, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("dim,kern", CASES)
def test_monotone_and_vanishing_at_support(dim, kern):
    h = 1.0
    kappa = kernels.KAPPA[kern]
    r = np.linspace(0.0, kappa * h * 1.2, 2001)
    assert np.all(kernels.dWdr(r, h, dim, kern) <= 0.0)
    assert kernels.W(kappa * h, h, dim, kern) == 0.0
    assert kernels.dWdr(kappa * h, h, dim, kern) == 0.0


def test_wendland_constants_closed_form():
    # k_d from the normalisation integral worked by hand:
    # int_0^1 psi = 1/3, int_0^1 psi q = 5/72, int_0^1 psi q^2 = 1/45.
    assert kernels.wendland_norm(1) == pytest.approx(1.5, rel=1e-15)
    assert kernels.wendland_norm(2) == pytest.approx(36.0 / (5.0 * math.pi), rel=1e-15)
    assert kernels.wendland_norm(3) == pytest.approx(45.0 / (4.0 * math.pi), rel=1e-15)
