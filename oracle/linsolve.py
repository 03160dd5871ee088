"""Solves of the symmetric positive-definite radiation system (oracle, FP64).

The paper solves the diffusion equation with a Krylov method preconditioned by
algebraic multigrid (Sec. 3.2); the system has one solution, so the oracle
may use any exact-enough method: a dense factorisation for small systems, or
conjugate gradients with a diagonal (Jacobi) preconditioner, stopping on the
relative residual ||b - A x||_2 / ||b||_2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def dense(A: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    return np.linalg.solve(A.toarray(), b)


def pcg_jacobi(A: sp.csr_matrix, b: np.ndarray, x0=None, tol: float = 1e-14,
               max_iter: int = 10000):
    """Textbook preconditioned CG.  Returns (x, iterations, final relative residual)."""
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
    best = rel
    stall = 0
    while rel > tol and it < max_iter:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = np.linalg.norm(r) / bn
        if rel < 0.5 * best:
            best = rel
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


def solve(A: sp.csr_matrix, b: np.ndarray, x0=None, tol: float = 1e-14):
    if A.shape[0] <= 2000:
        return dense(A, b)
    return pcg_jacobi(A, b, x0, tol)[0]
