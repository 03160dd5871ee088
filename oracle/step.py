"""Algorithm 1 of the paper (nonlinear elimination), convergence test and energy
sums (oracle, FP64).

One backward-Euler time step:

1. freeze the material data at the start of the step (Sec. 3.2) and assemble
   the diffusion system once;
2. e^{n,0} = e^{n-1}, E^{n,0} = E^{n-1}; solve m(e, E^{n,0}) = 0 for e;
3. repeat: solve r_dagger = 0 (the linear diffusion system) for E^{l+1} with
   B^{n,l} = a T(e^l)^4 and E^{n,l} on the right; solve m(e, E^{l+1}) = 0 for
   e^{l+1} (source Q_e + c sigma_a E^{l+1}, operators R and A of Sec. 3.2);
   until |e^{l+1} - e^l| / |e^{l+1}| < eps_e and |E^{l+1} - E^l| / |E^{l+1}| < eps_E
   (Sec. 2.2, convergence equations; the max over particles is taken).

Energy (Sec. 2.5): sum_i (m_i e_i + V_i E_i) over the interior particles.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import linsolve, material, neighbors, operator
from .kernels import KAPPA


@dataclass
class StepResult:
    e: np.ndarray
    E: np.ndarray
    outer: int
    delta_e: list = field(default_factory=list)
    delta_E: list = field(default_factory=list)
    material_its: list = field(default_factory=list)
    energy_before: float = 0.0
    energy_after: float = 0.0
    boundary_flux: float = 0.0      # dt * sum_i sum_{j ghost} V_i a_ij (E_j - E_i)
    source_energy: float = 0.0      # dt * sum_i V_i (Q_e,i + Q_E,i)


def energy(prob, e, E) -> float:
    nin = prob.n_interior
    return float(np.sum(prob.m[:nin] * e) + np.sum((prob.m / prob.rho)[:nin] * E))


def material_update(prob, fz, E_new, e_start, tol):
    nin = prob.n_interior
    sl = slice(0, nin)
    P = prob.Q_e[sl] + prob.c * fz.sigma_a[sl] * E_new
    return material.solve(prob.e[sl], P, prob.rho[sl], prob.cv[sl], fz.sigma_a[sl],
                          prob.dt, prob.c, prob.a, e_start, tol=tol)


def be_residual(prob, fz, ptr, idx, e: np.ndarray, E: np.ndarray):
    """The backward-Euler system G = [m, r] of Sec. 2.2 (the starting point of
    the nonlinear elimination) at the interior state (e, E), the opacities
    and diffusion coefficients frozen at the start of the step as in the rest
    of the step (ghost radiation energies fixed at prob.E):

        m_i = rho_i/dt (e_i - e_i^{n-1}) + c sigma_a,i (B_i - E_i) - Q_e,i
        r_i = (E_i - E_i^{n-1})/dt + sum_j V_j (D_i + D_j) F_ij (E_i - E_j)
              + c sigma_a,i (E_i - B_i) - Q_E,i,

    B = a (e/c_v)^4, the diffusion term the Brookshaw pair sum of Sec. 2.3
    over every neighbour (not the assembled matrix).  Returns (m, r)."""
    nin = prob.n_interior
    sl = slice(0, nin)
    B = prob.a * (e / prob.cv[sl]) ** 4
    ca = prob.c * fz.sigma_a[sl]
    m = prob.rho[sl] / prob.dt * (e - prob.e[sl]) + ca * (B - E) - prob.Q_e[sl]
    Efull = prob.E.copy()
    Efull[sl] = E
    I, J, _, F = operator.pair_geometry(prob, ptr, idx)
    a = fz.V[J] * (fz.D[I] + fz.D[J]) * F
    lap = np.bincount(I, weights=a * (Efull[I] - Efull[J]), minlength=prob.n_total)[sl]
    r = (E - prob.E[sl]) / prob.dt + lap + ca * (E - B) - prob.Q_E[sl]
    return m, r


def rel_change(new, old) -> float:
    return float(np.max(np.abs(new - old) / np.abs(new))) if new.size else 0.0


def time_step(prob, ptr=None, idx=None, eps_e: float = 1e-12, eps_E: float = 1e-12,
              inner_tol_e: float = 1e-14, solve_tol: float = 1e-14, max_outer: int = 50,
              fixed_outer=None, solver=None) -> StepResult:
    """One time step of Algorithm 1 from the state stored in ``prob``.

    ``fixed_outer`` runs exactly that many outer iterations (deterministic work
    for parity runs); otherwise iterate until the outer tolerances are met."""
    if ptr is None:
        ptr, idx = neighbors.build(prob.pos, prob.h, KAPPA[prob.kernel], prob.period)
    nin = prob.n_interior
    fz = operator.frozen(prob, ptr, idx)
    sysm = operator.assemble(prob, ptr, idx, fz)
    solver = solver or (lambda A, b, x0: linsolve.solve(A, b, x0, solve_tol))
    e_prev = prob.e[:nin].copy()
    E_prev = prob.E[:nin].copy()
    res = StepResult(e=e_prev, E=E_prev, outer=0)
    res.energy_before = energy(prob, e_prev, E_prev)
    E = E_prev.copy()
    e, its, _ = material_update(prob, fz, E, e_prev, inner_tol_e)
    res.material_its.append(int(its.max(initial=0)))
    n_outer = fixed_outer if fixed_outer is not None else max_outer
    for _ in range(n_outer):
        b = operator.rhs(prob, fz, sysm, e, E)
        E_new = solver(sysm.A, b, E)
        e_new, its, _ = material_update(prob, fz, E_new, e, inner_tol_e)
        de, dE = rel_change(e_new, e), rel_change(E_new, E)
        res.delta_e.append(de)
        res.delta_E.append(dE)
        res.material_its.append(int(its.max(initial=0)))
        e, E = e_new, E_new
        res.outer += 1
        if fixed_outer is None and de < eps_e and dE < eps_E:
            break
    res.e, res.E = e, E
    res.energy_after = energy(prob, e, E)
    I, J, a = sysm.pair_a
    gm = (I < nin) & (J >= nin)
    V = fz.V
    res.boundary_flux = prob.dt * float(np.sum(V[I[gm]] * a[gm] * (prob.E[J[gm]] - E[I[gm]])))
    res.source_energy = prob.dt * float(np.sum(V[:nin] * (prob.Q_e[:nin] + prob.Q_E[:nin])))
    return res


def advance(prob, res: StepResult) -> None:
    """Store the converged state as the start of the next step."""
    nin = prob.n_interior
    prob.e[:nin] = res.e
    prob.E[:nin] = res.E
    prob.t += prob.dt
