"""Time-step driver over the C ABI (host side, argument marshalling only).

Algorithm 1 of the paper as a host loop: ``rt_assemble`` once per time step
(material data frozen, preconditioner set up once), then ``rt_newton_step``
per outer iteration until the relative changes of e and E fall below the
outer tolerances (Sec. 2.2) or a fixed number of outer iterations has run.
Arrays are torch device tensors; every computation runs in librt.so.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

from . import rt

FIELDS = ("m", "rho", "cv", "sigma0_a", "sigma_s", "e", "E", "Q_e", "Q_E")


@dataclass
class DeviceProblem:
    dim: int
    n_total: int
    n_interior: int
    pos: object
    h: object
    arrays: dict
    dt: float
    c: float
    a: float
    opacity_exponent: float
    limiter: int
    limiter_k: float
    kernel: int
    period: object = None   # per-axis periods (0 = open axis) or None


def upload(prob, device) -> DeviceProblem:
    """Copy a problem description (numpy arrays, see ``synth.Problem``) to the device."""
    import torch
    t = lambda x: torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()
    return DeviceProblem(dim=prob.dim, n_total=prob.n_total, n_interior=prob.n_interior,
                         pos=t(prob.pos), h=t(prob.h), arrays={k: t(getattr(prob, k)) for k in FIELDS},
                         dt=prob.dt, c=prob.c, a=prob.a, opacity_exponent=prob.opacity_exponent,
                         limiter=prob.limiter, limiter_k=prob.limiter_k, kernel=prob.kernel,
                         period=(None if getattr(prob, "period", None) is None
                                 else [float(v) for v in prob.period]))


@dataclass
class StepReport:
    outer: int = 0
    status: int = 0
    delta_e: list = field(default_factory=list)
    delta_E: list = field(default_factory=list)
    krylov: list = field(default_factory=list)
    refinements: list = field(default_factory=list)
    energy_prev: float = 0.0
    energy: float = 0.0
    solve_seconds: float = 0.0
    newton_seconds: float = 0.0
    spmv64_calls: int = 0
    spmv64_seconds: float = 0.0
    spmv32_calls: int = 0
    spmv32_seconds: float = 0.0
    resid_calls: int = 0
    resid_seconds: float = 0.0
    cw_residual: list = field(default_factory=list)
    init_rel_residual: list = field(default_factory=list)
    replacements: list = field(default_factory=list)
    final_residual: Optional[tuple] = None   # (rad_rel, mat_rel) of the step's last state


def time_step(ctx: rt.Context, dp: DeviceProblem, nb: rt.Neighbors, A: int = 0,
              amg: Optional[rt.rt_amg_opts] = None, solve: Optional[rt.rt_solve_opts] = None,
              eps_e: float = 1e-8, eps_E: float = 1e-8, material_tol: float = 1e-14,
              max_outer: int = 50, fixed_outer: Optional[int] = None,
              shapes: Optional[list] = None, sorted_state: bool = True,
              recompute_residual: bool = False, final_residual: bool = False):
    """One backward-Euler step.  Returns (e, E, A, report) with e, E the new
    interior energies (device tensors, user order).  shapes: per-level
    (FP64, FP32[, FP64 residual]) SpMV shape indices (-1: default), e.g. the
    "chosen" list of Context.tune on an earlier matrix of the same problem,
    applied after assembly.
    sorted_state: keep e, E in the library's sorted order during the outer
    iterations (one conversion each way per step instead of per iteration).
    recompute_residual: start every solve from b - A x formed by a product
    instead of the residual carried over from the last outer iteration.
    final_residual: also evaluate the backward-Euler residual G at the step's
    last state (one more FP64 product); the starting states' relative
    radiation residuals are the solves' init_rel_residual."""
    A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                     dp.limiter_k, amg=amg, A=A)
    if shapes:
        levels = ctx.matrix_info(A).levels
        for lvl, chosen in enumerate(shapes[:levels]):
            for prod, s in zip((rt.RT_PREC_FP64, rt.RT_PREC_MIXED, rt.RT_PRODUCT_RESIDUAL), chosen):
                rt.rt_matrix_set_spmv_shape(A, lvl, prod, s)
    nin = dp.n_interior
    import torch
    e_user = dp.arrays["e"][:nin].clone()
    E_user = dp.arrays["E"][:nin].clone()
    if sorted_state:
        e, E = torch.empty_like(e_user), torch.empty_like(E_user)
        rt.rt_to_sorted(ctx.handle, nb.handle, e_user.data_ptr(), e.data_ptr())
        rt.rt_to_sorted(ctx.handle, nb.handle, E_user.data_ptr(), E.data_ptr())
    else:
        e, E = e_user, E_user
    solve = solve or rt.solve_opts()
    nopts = rt.newton_opts(solve, material_tol, state_order=1 if sorted_state else 0,
                           recompute_residual=1 if recompute_residual else 0)
    rep = StepReport()
    n_outer = fixed_outer if fixed_outer is not None else max_outer
    for ell in range(n_outer):
        status, st = ctx.newton_step(A, e, E, ell, nopts)
        rep.status = max(rep.status, status)
        rep.outer += 1
        rep.delta_e.append(st.delta_e)
        rep.delta_E.append(st.delta_E)
        rep.krylov.append(st.solve.iterations)
        rep.refinements.append(st.solve.refinements)
        rep.energy_prev = st.energy_prev
        rep.energy = st.energy
        rep.solve_seconds += st.solve.seconds
        rep.newton_seconds += st.seconds
        rep.spmv64_calls += st.solve.spmv_calls
        rep.spmv64_seconds += st.solve.spmv_seconds
        rep.spmv32_calls += st.solve.spmv32_calls
        rep.spmv32_seconds += st.solve.spmv32_seconds
        rep.resid_calls += st.solve.resid_calls
        rep.resid_seconds += st.solve.resid_seconds
        rep.cw_residual.append(st.solve.cw_residual)
        rep.init_rel_residual.append(st.solve.init_rel_residual)
        rep.replacements.append(st.solve.replacements)
        if fixed_outer is None and st.delta_e < eps_e and st.delta_E < eps_E:
            break
    if final_residual:
        g = ctx.newton_residual(A, e, E, 1 if sorted_state else 0)
        rep.final_residual = (g.rad_rel, g.mat_rel)
    if sorted_state:
        rt.rt_to_user(ctx.handle, nb.handle, e.data_ptr(), e_user.data_ptr())
        rt.rt_to_user(ctx.handle, nb.handle, E.data_ptr(), E_user.data_ptr())
        e, E = e_user, E_user
    return e, E, A, rep


def advance(dp: DeviceProblem, e, E) -> None:
    """Store the step's result as the state at the start of the next step."""
    nin = dp.n_interior
    dp.arrays["e"][:nin] = e
    dp.arrays["E"][:nin] = E


def run_adaptive(ctx: rt.Context, dp: DeviceProblem, t_end: float, dt0: float,
                 eta_target: float = 0.05, dt_min: float = 0.0, dt_max: float = float("inf"),
                 max_growth: float = 10.0, amg: Optional[rt.rt_amg_opts] = None,
                 solve: Optional[rt.rt_solve_opts] = None, eps_e: float = 1e-8,
                 eps_E: float = 1e-8, material_tol: float = 1e-14, tiny: float = 1e-15,
                 callback=None):
    """Time steps from t = 0 to t_end with the step control of Sec. 3.3.

    The particles are stationary, so the neighbour lists and the matrix
    structure are built once; every step re-assembles the values on that
    structure and runs Algorithm 1 to the outer tolerances.  After a step the
    library returns the fractional changes (eta_e, eta_E) and the next step is
    dt (eta_target/eta)^(1/2) for the more restrictive of the two, at most
    max_growth times the last step, within [dt_min, dt_max]; the last step is
    shortened to land on t_end.  Returns (steps, [(t, dt, StepReport)]).
    callback(t, e, E) is called after every step."""
    nin = dp.n_interior
    nb = ctx.build_neighbors(dp.pos, dp.h, nin, dp.kernel, period=dp.period)
    A = 0
    t, dt = 0.0, dt0
    history = []
    while t < t_end * (1.0 - 1e-14):
        dt = min(dt, t_end - t)
        dp.dt = dt
        e_old = dp.arrays["e"][:nin].clone()
        E_old = dp.arrays["E"][:nin].clone()
        e, E, A, rep = time_step(ctx, dp, nb, A=A, amg=amg, solve=solve, eps_e=eps_e, eps_E=eps_E,
                                 material_tol=material_tol)
        eta_e, eta_E = rt.rt_fractional_change(ctx.handle, A, e.data_ptr(), e_old.data_ptr(),
                                               E.data_ptr(), E_old.data_ptr(), eta_target, tiny)
        advance(dp, e, E)
        t += dt
        history.append((t, dt, rep))
        if callback:
            callback(t, e, E)
        props = [dt * (eta_target / eta) ** 0.5 if eta > 0.0 else float("inf")
                 for eta in (eta_e, eta_E)]
        dt = max(dt_min, min(min(props), max_growth * dt, dt_max))
    return len(history), history


def run_fixed(ctx: rt.Context, dp: DeviceProblem, dt: float, steps: int, sources=None,
              amg: Optional[rt.rt_amg_opts] = None, solve: Optional[rt.rt_solve_opts] = None,
              eps_e: float = 1e-8, eps_E: float = 1e-8, material_tol: float = 1e-14,
              fixed_outer: Optional[int] = None, callback=None):
    """``steps`` backward-Euler steps of length dt from t = 0 (Algorithm 1 per
    step).  sources(t) -> (Q_e, Q_E), device tensors over all particles, gives
    the sources of the step ending at t (time-dependent problems such as the
    manufactured solution of Sec. 4.3); None keeps dp's sources.  Neighbour
    lists and the matrix structure are built once.  Returns (t, [StepReport]).
    callback(t, e, E) is called after every step.  A step that ends with a
    soft status (a solve not converged, a clamped material root) raises
    RtError with that status; the state then holds the previous step."""
    nin = dp.n_interior
    nb = ctx.build_neighbors(dp.pos, dp.h, nin, dp.kernel, period=dp.period)
    A = 0
    dp.dt = dt
    t = 0.0
    reports = []
    for s in range(steps):
        t = (s + 1) * dt
        if sources is not None:
            Qe, QE = sources(t)
            dp.arrays["Q_e"].copy_(Qe)
            dp.arrays["Q_E"].copy_(QE)
        e, E, A, rep = time_step(ctx, dp, nb, A=A, amg=amg, solve=solve, eps_e=eps_e,
                                 eps_E=eps_E, material_tol=material_tol, fixed_outer=fixed_outer)
        if rep.status != rt.RT_OK:
            raise rt.RtError("run_fixed", rep.status, f"step {s + 1} did not complete")
        advance(dp, e, E)
        reports.append(rep)
        if callback:
            callback(t, e, E)
    return t, reports
