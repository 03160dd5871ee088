"""Solves of the symmetric positive-definite radiation system (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package; the library never does.

The paper solves the diffusion equation with a Krylov method preconditioned by
algebraic multigrid (Sec. 3.2); the system has one solution, so the oracle
may use any exact-enough method: a dense factorisation for small systems, or
conjugate gradients with a diagonal (Jacobi) preconditioner.  "Exact enough"
is taken per unknown: the radiation energy of one system can span many
decades (a cold medium ahead of a hot front), and a stop on the relative
residual ||b - A x||_2 / ||b||_2 alone leaves the small unknowns with large
relative errors.  So every solve also runs until the componentwise measure
max_i |b - A x|_i / (a_ii |x_i|) is below the tolerance, and ends with steps
of iterative refinement whose residual is accumulated in extended precision
(the x87 80-bit format numpy calls longdouble).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def dense(A: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    return np.linalg.solve(A.toarray(), b)


def residual_ext(A: sp.csr_matrix, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """b - A x with products and sums in extended precision, rounded to FP64."""
    Al = A.astype(np.longdouble)
    return (b.astype(np.longdouble) - Al @ x.astype(np.longdouble)).astype(np.float64)


def componentwise(A: sp.csr_matrix, x: np.ndarray, r: np.ndarray, scale=None) -> float:
    """max_i |r_i| / (a_ii s_i) with s = |x| (or the given scale): a row whose
    scale is zero counts 0 if its residual is zero and infinity otherwise."""
    s = np.abs(x) if scale is None else scale
    den = A.diagonal() * s
    ar = np.abs(r)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(den > 0.0, ar / np.where(den > 0.0, den, 1.0), np.where(ar > 0.0, np.inf, 0.0))
    return float(q.max(initial=0.0))


def pcg_jacobi(A: sp.csr_matrix, b: np.ndarray, x0=None, tol: float = 1e-14,
               max_iter: int = 10000, cw_tol: float = 0.0, cw_scale=None):
    """Textbook preconditioned CG, stopped when ||r||/||b|| <= tol and, if
    cw_tol > 0, the componentwise measure of r (scaled by |x|, or by cw_scale)
    is <= cw_tol; or when neither measure has halved for 50 iterations (the
    rounding floor).  Returns (x, iterations, final relative residual)."""
    dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    r = b - A @ x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    rel = np.linalg.norm(r) / bn
    cw = componentwise(A, x, r, cw_scale) if cw_tol > 0.0 else 0.0
    best, best_cw = rel, cw
    stall = 0
    while (rel > tol or cw > cw_tol) and it < max_iter:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = np.linalg.norm(r) / bn
        cw = componentwise(A, x, r, cw_scale) if cw_tol > 0.0 else 0.0
        if rel < 0.5 * best or cw < 0.5 * best_cw:
            best, best_cw = min(best, rel), min(best_cw, cw)
            stall = 0
        else:
            stall += 1
            if stall > 50:          # rounding floor reached
                break
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    true_rel = np.linalg.norm(b - A @ x) / bn
    return x, it, true_rel


def solve(A: sp.csr_matrix, b: np.ndarray, x0=None, tol: float = 1e-14,
          refine_steps: int = 3):
    """The solution of A x = b, accurate per unknown: a dense solve (up to 2000
    unknowns) or PCG to tol in both measures, then up to refine_steps steps of
    iterative refinement with the residual in extended precision, until the
    componentwise measure of that residual is <= tol."""
    small = A.shape[0] <= 2000
    if small:
        x = dense(A, b)
    else:
        x = pcg_jacobi(A, b, x0, tol, cw_tol=tol)[0]
    for _ in range(refine_steps):
        r = residual_ext(A, x, b)
        if componentwise(A, x, r) <= tol:
            break
        if small:
            d = dense(A, r)
        else:
            d = pcg_jacobi(A, r, None, tol, cw_tol=tol, cw_scale=np.abs(x))[0]
        x = x + d
    return x
