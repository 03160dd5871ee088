"""Per-particle material energy solve, the operator M^-1 of Sec. 3.2 (oracle, FP64).

For each particle, given the source P_i, solve

    u(e) = rho/dt (e - e^{n-1}) + c sigma_a a T(e)^4 - P = 0,   T = e / c_v,

by Newton's method e <- e - u(e)/J(e) with J = rho/dt + 4 c sigma_a a T^3 / c_v,
until the Newton step satisfies |e_new - e| <= tol |e_new|.  sigma_a is the value frozen at the start of
the step.  The paper gives no safeguard; u is strictly increasing and convex
on e >= 0 with u(0) <= 0 <= u(e^{n-1} + dt P / rho), so the physical root is
unique in that bracket and a Newton step that leaves the current bracket is
replaced by bisection.  All particles advance together, as the paper
describes for the temperature update.
"""
from __future__ import annotations

import numpy as np


def solve(e_prev, P, rho, cv, sigma_a, dt: float, c: float, a: float, e_start,
          tol: float = 1e-14, max_iter: int = 200):
    """Returns (e, iterations_per_particle, nonphysical_mask)."""
    e_prev = np.asarray(e_prev, dtype=np.float64)
    lo = np.zeros_like(e_prev)
    hi = e_prev + dt * P / rho
    nonphysical = hi < 0.0
    e = np.minimum(np.maximum(np.asarray(e_start, dtype=np.float64), lo), hi)
    e = np.where(nonphysical, 0.0, e)
    active = ~nonphysical
    its = np.zeros(e.shape, dtype=np.int64)
    for _ in range(max_iter):
        if not active.any():
            break
        T = e / cv
        u = rho / dt * (e - e_prev) + c * sigma_a * a * T ** 4 - P
        J = rho / dt + 4.0 * c * sigma_a * a * T ** 3 / cv
        root = u == 0.0
        hi = np.where(active & (u > 0.0), e, hi)
        lo = np.where(active & (u < 0.0), e, lo)
        e_newton = e - u / J
        small = np.abs(e_newton - e) <= tol * np.abs(e_newton)
        outside = ~((e_newton > lo) & (e_newton < hi))
        e_new = np.where(small | ~outside, e_newton, 0.5 * (lo + hi))
        e_new = np.where(root, e, e_new)
        conv = root | small
        its += active
        e = np.where(active, e_new, e)
        active = active & ~conv
    return e, its, nonphysical
