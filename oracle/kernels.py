"""SPH kernels W(r, h) and dW/dr in 1, 2 and 3 dimensions (oracle, FP64).

* Wendland "C4" of the paper (Sec. 2.3, the Wendland C4 equation): the printed
  polynomial psi(q) = (1-q)^5 (8 q^2 + 5 q + 1) for q = r/h <= 1, zero beyond,
  scaled by a dimension-dependent constant chosen so that the kernel integrates
  to one (the kernel-normalisation equation of Sec. 2.3).  The paper does not
  print the constant; it is computed here from that condition with exact
  rational integration.
* Cubic B-spline (M4), support 2h, used by the synthetic workloads: the
  textbook piecewise cubic with sigma_d = 2/3, 10/(7 pi), 1/pi.

The derivative is with respect to r, so the gradient with respect to x_i of
W(|x_i - x_j|, h) is dW/dr * x_ij / r.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

CUBIC_SPLINE = 0
WENDLAND_C4 = 1

# support radius in units of h
KAPPA = {CUBIC_SPLINE: 2.0, WENDLAND_C4: 1.0}

CUBIC_SIGMA = {1: 2.0 / 3.0, 2: 10.0 / (7.0 * math.pi), 3: 1.0 / math.pi}


def _poly_mul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _wendland_radial_integral(dim: int) -> Fraction:
    """Exact value of int_0^1 psi(q) q^(dim-1) dq for the printed polynomial."""
    one_minus_q = [Fraction(1), Fraction(-1)]
    p = [Fraction(1)]
    for _ in range(5):
        p = _poly_mul(p, one_minus_q)
    p = _poly_mul(p, [Fraction(1), Fraction(5), Fraction(8)])
    return sum(c / (k + dim) for k, c in enumerate(p))


def wendland_norm(dim: int) -> float:
    """Constant k with int W dV = 1 (unit sphere surface: 2, 2 pi, 4 pi)."""
    surface = {1: 2.0, 2: 2.0 * math.pi, 3: 4.0 * math.pi}[dim]
    return 1.0 / (surface * float(_wendland_radial_integral(dim)))


def W(r, h, dim: int, kernel: int):
    r = np.asarray(r, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    q = r / h
    if kernel == CUBIC_SPLINE:
        w = np.where(q < 1.0, 1.0 - 1.5 * q * q + 0.75 * q ** 3,
                     np.where(q < 2.0, 0.25 * (2.0 - q) ** 3, 0.0))
        return CUBIC_SIGMA[dim] * w / h ** dim
    if kernel == WENDLAND_C4:
        w = np.where(q < 1.0, (1.0 - q) ** 5 * (8.0 * q * q + 5.0 * q + 1.0), 0.0)
        return wendland_norm(dim) * w / h ** dim
    raise ValueError(kernel)


def dWdr(r, h, dim: int, kernel: int):
    """Radial derivative of W; it is <= 0 for both kernels."""
    r = np.asarray(r, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    q = r / h
    if kernel == CUBIC_SPLINE:
        dw = np.where(q < 1.0, -3.0 * q + 2.25 * q * q,
                      np.where(q < 2.0, -0.75 * (2.0 - q) ** 2, 0.0))
        return CUBIC_SIGMA[dim] * dw / h ** (dim + 1)
    if kernel == WENDLAND_C4:
        # d/dq [(1-q)^5 (8q^2+5q+1)] = -14 q (4q+1) (1-q)^4
        dw = np.where(q < 1.0, -14.0 * q * (4.0 * q + 1.0) * (1.0 - q) ** 4, 0.0)
        return wendland_norm(dim) * dw / h ** (dim + 1)
    raise ValueError(kernel)
