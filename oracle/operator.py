"""Frozen per-step data, the Brookshaw diffusion operator and the right-hand
side of the linear radiation solve (oracle, FP64).

Linear system (Sec. 3.2, the equation defining the diffusion solve D^-1):

    (1/dt + c sigma_a,i f_i) E_i
        - sum_j V_j (D_i + D_j) (E_i - E_j) x_ij . dW_ij / (x_ij . x_ij) = P_i

with D_i = c lambda_i / sigma_t,i (Sec. 2.4) and the symmetrised kernel
gradient dW_ij = 1/2 [dW(x_ij, h_i) + dW(x_ij, h_j)] (Sec. 2.3).  Since
dW(x_ij, h) = W'(r, h) x_ij / r, the pair weight is

    F_ij = -1/2 [W'(r, h_i) + W'(r, h_j)] / r >= 0,    a_ij = V_j (D_i + D_j) F_ij,

and row i reads (1/dt + c sigma_a f)_i E_i + sum_j a_ij (E_i - E_j) = P_i.

Multiplying row i by V_i gives the symmetric M-matrix that is solved:

    A_ii = V_i (1/dt + c sigma_a,i f_i) + V_i sum_j a_ij       (all neighbours j)
    A_ij = -V_i V_j (D_i + D_j) F_ij                           (interior j)

Constant-value ghosts (Sec. 3.1) are not unknowns: their coupling moves to the
right-hand side, g_i = V_i sum_{j ghost} a_ij E_j.

Right-hand side (Sec. 2.2 inexact Newton equation; Sec. 3.2 operators S and N):

    b_i = V_i [E_i^{n-1}/dt + c sigma_a,i a T_i^4 - (1 - f_i) c sigma_a,i E_i^l + Q_E,i] + g_i

Frozen data (Sec. 3.2: computed at the start of the step): T = e/c_v;
sigma_a = sigma0_a T^p; sigma_t = sigma_a + sigma_s; Fleck factor
f = 1/(1 + c sigma_a dt 4 a T^3 / (rho c_v)) (Sec. 2.2); V = m/rho (Sec. 2.3);
lambda = 1/3, or a flux limiter of R = |grad E| / (sigma_t E) (Sec. 2.1) with
grad E_i = sum_j V_j (E_j - E_i) dW_ij (first SPH derivative, Sec. 2.3) at E^{n-1}.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import kernels
from .neighbors import disp, pairs, pair_r2

LIMITER_NONE = 0
LIMITER_LARSEN = 1
LIMITER_LEVERMORE = 2


@dataclass
class Frozen:
    T: np.ndarray
    sigma_a: np.ndarray
    sigma_t: np.ndarray
    f: np.ndarray
    V: np.ndarray
    lam: np.ndarray
    D: np.ndarray


def pair_geometry(prob, ptr, idx):
    """(i, j, r, F_ij) for every neighbour pair."""
    I, J = pairs(ptr, idx)
    r = np.sqrt(pair_r2(prob.pos, I, J, prob.period))
    dwi = kernels.dWdr(r, prob.h[I], prob.dim, prob.kernel)
    dwj = kernels.dWdr(r, prob.h[J], prob.dim, prob.kernel)
    F = -0.5 * (dwi + dwj) / r
    return I, J, r, F


def grad_E(prob, ptr, idx, E):
    """First SPH derivative of E at every particle (Sec. 2.3)."""
    I, J, r, F = pair_geometry(prob, ptr, idx)
    V = prob.m / prob.rho
    # dW_ij = 1/2 [W'(r,h_i) + W'(r,h_j)] x_ij / r = -F_ij x_ij
    g = np.zeros((prob.dim, prob.n_total))
    w = V[J] * (E[J] - E[I]) * (-F)
    for ax in range(prob.dim):
        xij = disp(prob.pos, ax, I, J, prob.period)
        g[ax] = np.bincount(I, weights=w * xij, minlength=prob.n_total)
    return g


def flux_limiter(R, kind: int, k: float):
    """lambda(R) of Sec. 2.1: Larsen (3^k + R^k)^(-1/k), Levermore
    (2 + R)/(6 + 3R + R^2).  Above R = 1 the Levermore quotient is evaluated
    with u = 1/R, as u(1 + 2u)/(1 + 3u + 6u^2), which is the same function and
    stays finite as R grows without bound (lambda -> 0, lambda R -> 1)."""
    R = np.asarray(R, dtype=float)
    if kind == LIMITER_LARSEN:
        return (3.0 ** k + R ** k) ** (-1.0 / k)
    if kind == LIMITER_LEVERMORE:
        out = np.empty_like(R)
        lo = R <= 1.0
        out[lo] = (2.0 + R[lo]) / (6.0 + 3.0 * R[lo] + R[lo] * R[lo])
        with np.errstate(divide="ignore"):
            u = 1.0 / R[~lo]
        out[~lo] = u * (1.0 + 2.0 * u) / (1.0 + 3.0 * u + 6.0 * u * u)
        return out
    return np.full_like(R, 1.0 / 3.0)


def limiter_ratio(grad_norm, sigma_t, E):
    """R = |grad E| / (sigma_t E) (Sec. 2.1), with its two degenerate cases
    fixed: no gradient gives R = 0 (the diffusion limit, also where E = 0),
    and a gradient where E <= 0 gives R = infinity (the free-streaming limit)."""
    g = np.asarray(grad_norm, dtype=float)
    den = np.asarray(sigma_t * E, dtype=float)
    with np.errstate(divide="ignore", invalid="ignore"):
        R = np.where(den > 0.0, g / np.where(den > 0.0, den, 1.0), np.inf)
    return np.where(g == 0.0, 0.0, R)


def frozen(prob, ptr, idx) -> Frozen:
    T = prob.e / prob.cv
    sigma_a = prob.sigma0_a * T ** prob.opacity_exponent
    sigma_t = sigma_a + prob.sigma_s
    f = 1.0 / (1.0 + prob.c * sigma_a * prob.dt * 4.0 * prob.a * T ** 3 / (prob.rho * prob.cv))
    V = prob.m / prob.rho
    lam = np.full(prob.n_total, 1.0 / 3.0)
    if prob.limiter != LIMITER_NONE:
        g = grad_E(prob, ptr, idx, prob.E)
        R = limiter_ratio(np.sqrt(np.sum(g * g, axis=0)), sigma_t, prob.E)
        nin = prob.n_interior
        lam[:nin] = flux_limiter(R[:nin], prob.limiter, prob.limiter_k)
    D = prob.c * lam / sigma_t
    return Frozen(T=T, sigma_a=sigma_a, sigma_t=sigma_t, f=f, V=V, lam=lam, D=D)


@dataclass
class System:
    A: sp.csr_matrix          # V-scaled symmetric operator over interior particles
    g: np.ndarray             # ghost coupling moved to the right-hand side
    pair_a: tuple             # (I, J, a_ij) for every pair, for balance checks


def assemble(prob, ptr, idx, fz: Frozen) -> System:
    nin = prob.n_interior
    I, J, r, F = pair_geometry(prob, ptr, idx)
    V, D = fz.V, fz.D
    a = V[J] * (D[I] + D[J]) * F
    rows = I < nin
    suma = np.bincount(I[rows], weights=a[rows], minlength=nin)
    diag = V[:nin] * (1.0 / prob.dt + prob.c * fz.sigma_a[:nin] * fz.f[:nin]) + V[:nin] * suma
    inner = rows & (J < nin)
    off = -(V[I[inner]] * V[J[inner]]) * (D[I[inner]] + D[J[inner]]) * F[inner]
    ghost = rows & (J >= nin)
    g = V[:nin] * np.bincount(I[ghost], weights=a[ghost] * prob.E[J[ghost]], minlength=nin)
    A = sp.csr_matrix((np.concatenate([off, diag]),
                       (np.concatenate([I[inner], np.arange(nin)]),
                        np.concatenate([J[inner], np.arange(nin)]))), shape=(nin, nin))
    A.sort_indices()
    return System(A=A, g=g, pair_a=(I, J, a))


def rhs(prob, fz: Frozen, sysm: System, e_l: np.ndarray, E_l: np.ndarray) -> np.ndarray:
    nin = prob.n_interior
    sl = slice(0, nin)
    T = e_l / prob.cv[sl]
    B = prob.a * T ** 4
    ca = prob.c * fz.sigma_a[sl]
    P = prob.E[sl] / prob.dt + ca * B - (1.0 - fz.f[sl]) * ca * E_l + prob.Q_E[sl]
    return fz.V[sl] * P + sysm.g


def apply_unscaled(prob, ptr, idx, fz: Frozen, E_full: np.ndarray) -> np.ndarray:
    """Left-hand side of the diffusion-solve equation evaluated directly as the
    paper's pair sum (no matrix), at every interior particle; ``E_full`` holds
    interior unknowns followed by ghost values."""
    nin = prob.n_interior
    I, J, r, F = pair_geometry(prob, ptr, idx)
    a = fz.V[J] * (fz.D[I] + fz.D[J]) * F
    s = np.bincount(I, weights=a * (E_full[I] - E_full[J]), minlength=prob.n_total)[:nin]
    return (1.0 / prob.dt + prob.c * fz.sigma_a[:nin] * fz.f[:nin]) * E_full[:nin] + s


def brookshaw(prob, ptr, idx, k: np.ndarray, g: np.ndarray) -> np.ndarray:
    """SPH second derivative <d(k dg)>_i of Sec. 2.3 for arbitrary fields k, g
    (all particles):  sum_j V_j (k_i + k_j)(g_i - g_j) x_ij.dW_ij/|x_ij|^2."""
    I, J, r, F = pair_geometry(prob, ptr, idx)
    V = prob.m / prob.rho
    # x_ij . dW_ij / |x_ij|^2 = 1/2 [W'(r,h_i)+W'(r,h_j)] / r = -F_ij
    w = V[J] * (k[I] + k[J]) * (g[I] - g[J]) * (-F)
    return np.bincount(I, weights=w, minlength=prob.n_total)


def frozen_at(prob, ids, nbrs_of) -> dict:
    """The frozen data of ``frozen`` for the particles ``ids`` only (same
    formulas); ``nbrs_of(i)`` gives the ascending neighbour list of i, needed
    for the flux limiter's gradient.  Returns {i: (sigma_a, f, V, D)}."""
    out = {}
    for i in ids:
        i = int(i)
        T = prob.e[i] / prob.cv[i]
        sigma_a = prob.sigma0_a[i] * T ** prob.opacity_exponent
        sigma_t = sigma_a + prob.sigma_s[i]
        f = 1.0 / (1.0 + prob.c * sigma_a * prob.dt * 4.0 * prob.a * T ** 3 /
                   (prob.rho[i] * prob.cv[i]))
        V = prob.m[i] / prob.rho[i]
        lam = 1.0 / 3.0
        if prob.limiter != LIMITER_NONE and i < prob.n_interior:
            J = nbrs_of(i).astype(np.int64)
            I = np.full(J.shape, i)
            r = np.sqrt(pair_r2(prob.pos, I, J, prob.period))
            F = -0.5 * (kernels.dWdr(r, prob.h[I], prob.dim, prob.kernel) +
                        kernels.dWdr(r, prob.h[J], prob.dim, prob.kernel)) / r
            Vj = prob.m[J] / prob.rho[J]
            w = Vj * (prob.E[J] - prob.E[i]) * (-F)
            g = np.array([np.sum(w * disp(prob.pos, ax, I, J, prob.period))
                          for ax in range(prob.dim)])
            R = limiter_ratio(np.sqrt(np.sum(g * g)), sigma_t, prob.E[i])
            lam = float(flux_limiter(np.array([float(R)]), prob.limiter, prob.limiter_k)[0])
        out[i] = (sigma_a, f, V, prob.c * lam / sigma_t)
    return out


def rows_at(prob, rows, nbrs_of) -> dict:
    """Rows of the V-scaled system of ``assemble`` for the interior particles
    ``rows`` only (same formulas).  Returns {i: (diag, cols, vals, g_i)} with
    the interior columns ascending."""
    nin = prob.n_interior
    need = set(int(i) for i in rows)
    for i in rows:
        need.update(int(j) for j in nbrs_of(i))
    fz = frozen_at(prob, sorted(need), nbrs_of)
    out = {}
    for i in rows:
        i = int(i)
        J = nbrs_of(i).astype(np.int64)
        I = np.full(J.shape, i)
        r = np.sqrt(pair_r2(prob.pos, I, J, prob.period))
        F = -0.5 * (kernels.dWdr(r, prob.h[I], prob.dim, prob.kernel) +
                    kernels.dWdr(r, prob.h[J], prob.dim, prob.kernel)) / r
        sa_i, f_i, V_i, D_i = fz[i]
        Vj = np.array([fz[int(j)][2] for j in J])
        Dj = np.array([fz[int(j)][3] for j in J])
        a = Vj * (D_i + Dj) * F
        diag = V_i * (1.0 / prob.dt + prob.c * sa_i * f_i) + V_i * np.sum(a)
        inner = J < nin
        vals = -(V_i * Vj[inner]) * (D_i + Dj[inner]) * F[inner]
        g = V_i * np.sum(a[~inner] * prob.E[J[~inner]])
        out[i] = (diag, J[inner].astype(np.int32), vals, g)
    return out
