"""Pins for the oracle's linear solve, material Newton and Algorithm 1 (CPU).

* Linear solve: Jacobi-PCG agrees with a dense LAPACK solve.
* Material solve (Sec. 3.2): the per-particle root agrees with a 40-digit
  mpmath root of the same quartic.
* Infinite medium (Sec. 4.1 set-up, dimensionless units): a uniform field makes
  the Brookshaw sum vanish, so one backward-Euler step of the coupled system
  is the scalar system rho (e - e0)/dt = c sigma_a (E - a T^4),
  (E - E0)/dt = c sigma_a (a T^4 - E).  Algorithm 1 iterated to convergence
  must reproduce its 40-digit root, conserve m e + V E (Sec. 2.5) and relax to
  the equilibrium a T^4 + rho c_v T = rho e0 + E0 with E = B.
* First order in time (Sec. 4.1): against SciPy's Radau IIA solution of the
  two ODEs, halving dt halves the error.
* Energy balance with Dirichlet ghosts: the change of sum(m e + V E) equals the
  source term plus the flux exchanged with the ghosts, to the outer tolerance.
"""
import mpmath
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.integrate import solve_ivp

import synth
from oracle import linsolve, material, neighbors, operator, step

mpmath.mp.dps = 40


def _bisect(f, lo, hi, n=200):
    """40-digit bisection for an increasing function with f(lo) <= 0 <= f(hi)."""
    lo, hi = mpmath.mpf(lo), mpmath.mpf(hi)
    for _ in range(n):
        mid = (lo + hi) / 2
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    return (lo + hi) / 2


def test_pcg_matches_dense():
    p = synth.config1(n=40)
    ptr, idx = neighbors.build(p.pos, p.h, 2.0)
    fz = operator.frozen(p, ptr, idx)
    s = operator.assemble(p, ptr, idx, fz)
    b = np.random.default_rng(0).standard_normal(p.n_interior)
    xd = np.linalg.solve(s.A.toarray(), b)
    xc, it, rel = linsolve.pcg_jacobi(s.A, b, tol=1e-15)
    assert np.max(np.abs(xc - xd)) / np.max(np.abs(xd)) < 1e-13


def _marshak_system(n):
    p = synth.config4(n=n)
    ptr, idx = neighbors.build(p.pos, p.h, 2.0)
    fz = operator.frozen(p, ptr, idx)
    s = operator.assemble(p, ptr, idx, fz)
    return p, fz, s, operator.rhs(p, fz, s, p.e[:p.n_interior], p.E[:p.n_interior])


def _mp_solve(A, b):
    mpmath.mp.dps = 40
    M = mpmath.matrix(A.toarray().tolist())
    return np.array([float(v) for v in mpmath.lu_solve(M, mpmath.matrix(b.tolist()))])


def test_solve_accurate_per_unknown_vs_mpmath():
    """The oracle's solve matches a 40-digit LU solve of the same FP64 system
    in every unknown to 2e-15 relative: on the radiation-front system (E over
    three decades at this size) and on a diagonally dominant M-matrix whose
    solution spans twelve decades, where an error of 1e-16 of the largest
    unknown would be an error of 1e-4 in the smallest."""
    p, fz, s, b = _marshak_system(6)
    xe = _mp_solve(s.A, b)
    assert xe.max() / xe.min() > 1e3
    x = linsolve.solve(s.A, b)
    assert np.max(np.abs(x - xe) / xe) < 2e-15
    assert linsolve.componentwise(s.A, x, linsolve.residual_ext(s.A, x, b)) < 1e-15
    import scipy.sparse as sps
    rng = np.random.default_rng(5)
    n = 120
    off = -rng.uniform(0.0, 0.3, n - 1)
    A = sps.diags([off, np.zeros(n), off], [-1, 0, 1]).tolil()
    A.setdiag(1.0 + rng.uniform(0.0, 0.2, n) - np.asarray(A.sum(axis=1)).ravel())
    A = A.tocsr()
    b = A @ (10.0 ** np.linspace(0.0, -12.0, n))
    xe = _mp_solve(A, b)
    assert xe.max() / xe.min() > 1e11
    x = linsolve.solve(A, b)
    assert np.max(np.abs(x - xe) / xe) < 2e-15
    # the PCG path with the componentwise stop (the normwise one alone leaves
    # errors near 1e-11 in the smallest unknowns here)
    xc = linsolve.pcg_jacobi(A, b, tol=1e-14, cw_tol=1e-14)[0]
    assert np.max(np.abs(xc - xe) / xe) < 1e-13


def test_pcg_componentwise_stop_on_a_front():
    """PCG (the path of larger systems) continued until the componentwise
    measure is met agrees per unknown with the dense solve refined in extended
    precision; stopped on the normwise test alone it is allowed to stop
    earlier, never later."""
    p, fz, s, b = _marshak_system(14)
    assert p.n_interior > 2000
    x = linsolve.solve(s.A, b)
    xd = linsolve.dense(s.A, b)
    xd = xd + linsolve.dense(s.A, linsolve.residual_ext(s.A, xd, b))
    assert np.max(np.abs(x - xd) / np.abs(xd)) < 1e-13
    _, its_norm, _ = linsolve.pcg_jacobi(s.A, b, tol=1e-14)
    _, its_cw, _ = linsolve.pcg_jacobi(s.A, b, tol=1e-14, cw_tol=1e-14)
    assert its_cw >= its_norm


def test_componentwise_measure_edge_cases():
    A = __import__("scipy.sparse", fromlist=["csr_matrix"]).csr_matrix(np.diag([2.0, 4.0, 1.0]))
    x = np.array([1.0, 0.0, 0.0])
    assert linsolve.componentwise(A, x, np.array([0.2, 0.0, 0.0])) == pytest.approx(0.1)
    assert linsolve.componentwise(A, x, np.array([0.2, 1e-300, 0.0])) == np.inf


def _quartic_root(e_prev, P, rho, cv, sig, dt, c=1.0, a=1.0):
    f = lambda e: rho / dt * (e - e_prev) + c * sig * a * (e / cv) ** 4 - P
    hi = e_prev + dt * P / rho
    return _bisect(f, 0, hi)


def test_material_newton_vs_mpmath():
    rng = np.random.default_rng(11)
    n = 40
    e_prev = 10 ** rng.uniform(-4, 1, n)
    rho = rng.uniform(0.5, 4, n)
    cv = rng.uniform(0.5, 2, n)
    sig = 10 ** rng.uniform(-2, 6, n)
    dt = 10 ** rng.uniform(-5, -1, n)
    P = 10 ** rng.uniform(-3, 2, n) * sig
    e, its, bad = material.solve(e_prev, P, rho, cv, sig, dt, 1.0, 1.0, e_prev, tol=1e-15)
    assert not bad.any()
    for i in range(n):
        ref = _quartic_root(mpmath.mpf(e_prev[i]), mpmath.mpf(P[i]), mpmath.mpf(rho[i]),
                            mpmath.mpf(cv[i]), mpmath.mpf(sig[i]), mpmath.mpf(dt[i]))
        assert abs(e[i] - float(ref)) <= 4e-15 * float(ref)


def _infinite_problem(e0, E0, dt, n=6, sigma0=1.0, p=0.0):
    prob = synth.config2_infinite(T0=e0, E0=E0, n=n, sigma0=sigma0, dt=dt)
    prob.opacity_exponent = p
    return prob


def _scalar_be_step(e0, E0, dt, sig):
    """Exact BE step of the coupled scalar system (rho = c = a = c_v = 1)."""
    e0, E0, dt, sig = map(mpmath.mpf, (e0, E0, dt, sig))
    f = lambda e: (e - e0) / dt - sig * (E0 + e0 - e - e ** 4)
    e = _bisect(f, 0, e0 + dt * sig * (E0 + e0))
    return e, E0 + e0 - e


@pytest.mark.parametrize("e0,E0,dt", [(1.0, 1e-16, 0.1), (1.0, 1e-16, 1e-3),
                                       (1e-4, 1.0, 0.1), (1e-4, 1.0, 1e-3)])
def test_infinite_medium_step_closed_form(e0, E0, dt):
    prob = _infinite_problem(e0, E0, dt)
    r = step.time_step(prob, eps_e=1e-14, eps_E=1e-14, max_outer=200)
    e_ref, E_ref = _scalar_be_step(e0, E0, dt, 1.0)
    assert np.allclose(r.e, float(e_ref), rtol=1e-12, atol=0)
    assert np.allclose(r.E, float(E_ref), rtol=1e-12, atol=0)
    assert abs(r.energy_after - r.energy_before) <= 1e-13 * r.energy_before


def test_infinite_medium_variable_opacity_closed_form():
    # sigma_a = 10 T^-3 frozen at the start of the step
    e0, E0, dt = 1.0, 0.01, 1e-3
    prob = _infinite_problem(e0, E0, dt, sigma0=10.0, p=-3.0)
    r = step.time_step(prob, eps_e=1e-14, eps_E=1e-14, max_outer=200)
    e_ref, E_ref = _scalar_be_step(e0, E0, dt, 10.0 * e0 ** -3)
    assert np.allclose(r.e, float(e_ref), rtol=1e-12, atol=0)
    assert np.allclose(r.E, float(E_ref), rtol=1e-12, atol=0)


@pytest.mark.parametrize("e0,E0", [(1.0, 1e-16), (1e-4, 1.0)])
def test_equilibrium(e0, E0):
    prob = _infinite_problem(e0, E0, 10.0, n=4)
    for _ in range(40):
        r = step.time_step(prob, eps_e=1e-14, eps_E=1e-14, max_outer=200)
        step.advance(prob, r)
    T = _bisect(lambda T: T ** 4 + T - (e0 + E0), 0, 2)
    assert np.allclose(r.e, float(T), rtol=1e-12)
    assert np.allclose(r.E, float(T) ** 4, rtol=1e-12)


def test_first_order_in_time_vs_radau():
    e0, E0, t_end = 1.0, 1e-16, 1.0
    ref = solve_ivp(lambda t, y: [y[1] - y[0] ** 4, y[0] ** 4 - y[1]], (0, t_end), [e0, E0],
                    method="Radau", rtol=1e-13, atol=1e-16)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        prob = _infinite_problem(e0, E0, dt, n=3)
        for _ in range(int(round(t_end / dt))):
            r = step.time_step(prob, eps_e=1e-14, eps_E=1e-14, max_outer=200)
            step.advance(prob, r)
        errs.append(abs(r.e[0] - ref.y[0, -1]))
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


def test_energy_balance_with_ghosts():
    prob = synth.config1(n=24)
    r = step.time_step(prob, eps_e=1e-13, eps_E=1e-13)
    lhs = r.energy_after - r.energy_before
    rhs = r.source_energy + r.boundary_flux
    assert abs(lhs - rhs) <= 1e-12 * r.energy_before


def test_manufactured_step_close_to_exact():
    prob = synth.config1(n=32)
    r = step.time_step(prob)
    e_x, E_x, _, _ = prob.mms(prob.dt)
    nin = prob.n_interior
    assert np.max(np.abs(r.e - e_x[:nin]) / e_x[:nin]) < 1e-4
    assert np.max(np.abs(r.E - E_x[:nin]) / E_x[:nin]) < 2e-3


def _infinite_medium_run(e0, E0, dt0, t_end=10.0):
    """The paper's infinite-medium run: adaptive steps from dt0 to t_end (the
    last step shortened to land on t_end)."""
    import synth
    from oracle import timestep
    prob = synth.config2_infinite(e0, E0, n=2, sigma0=1.0, dt=dt0)
    prob.opacity_exponent = 0.0
    nin = prob.n_interior
    V = prob.m[:nin] / prob.rho[:nin]
    t, dt = 0.0, dt0
    ts, es, Es = [0.0], [e0], [E0]
    while t < t_end * (1.0 - 1e-14):
        dt = min(dt, t_end - t)
        prob.dt = dt
        e_old, E_old = prob.e[:nin].copy(), prob.E[:nin].copy()
        r = step.time_step(prob, eps_e=1e-12, eps_E=1e-12, inner_tol_e=1e-14, solve_tol=1e-14)
        step.advance(prob, r)
        t += dt
        ts.append(t)
        es.append(float(r.e[0]))
        Es.append(float(r.E[0]))
        dt = timestep.next_dt(dt, r.e, e_old, r.E, E_old, V, eta_target=0.05, dt_max=0.1,
                              max_growth=10.0)
    return np.array(ts), np.array(es), np.array(Es)


@pytest.mark.parametrize("case", ["hot_material", "hot_radiation"])
def test_infinite_medium_vs_paper(case):
    """Paper-printed values of the two infinite-medium runs (Sec. 4.1 and its
    initial-condition table, tests/golden/infinite_medium_sec4_1.json): the
    step count with the Sec. 3.3 controller, and the time-integrated L1 errors
    against a Radau IIA reference (Simpson's rule over the step times).  The
    step counts agree to within one (the paper does not say how it counts the
    last step); they pin the reading of the controller's floor term (the mean
    radiation energy in both fractional changes: with each energy's own mean
    the hot-radiation run takes 275 steps instead of 155).  The errors are of
    the printed size (the paper's error integral is not fully specified) and
    keep the printed material/radiation ratio; total energy is conserved."""
    import json
    import os
    from scipy.integrate import simpson, solve_ivp
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "infinite_medium_sec4_1.json")))[case]
    ts, es, Es = _infinite_medium_run(g["e0"], g["E0"], g["dt_init"])
    assert abs((len(ts) - 1) - g["steps"]) <= 1
    f = lambda t, y: [y[1] - y[0] ** 4, -y[1] + y[0] ** 4]
    ref = solve_ivp(f, (0.0, ts[-1]), [g["e0"], g["E0"]], method="Radau", t_eval=ts,
                    rtol=1e-12, atol=1e-22).y
    Te_ref, Tr_ref = ref[0], np.abs(ref[1]) ** 0.25
    l1_e = simpson(np.abs(Te_ref - es), x=ts) / simpson(Te_ref, x=ts)
    l1_r = simpson(np.abs(Tr_ref - np.abs(Es) ** 0.25), x=ts) / simpson(Tr_ref, x=ts)
    assert 0.5 < l1_e / g["l1_material"] < 2.5 and 0.5 < l1_r / g["l1_radiation"] < 2.5
    assert abs(l1_e / l1_r - g["l1_material"] / g["l1_radiation"]) < 0.1
    assert abs((es[-1] + Es[-1]) - (g["e0"] + g["E0"])) <= 1e-13

def _be_parts(prob):
    ptr, idx = neighbors.build(prob.pos, prob.h, 2.0, prob.period)
    fz = operator.frozen(prob, ptr, idx)
    return ptr, idx, fz


@pytest.mark.parametrize("e0,E0,dt", [(1.0, 1e-16, 0.1), (1e-4, 1.0, 1e-3)])
def test_be_residual_zero_at_the_scalar_root(e0, E0, dt):
    """G of Sec. 2.2 vanishes at the exact backward-Euler step of the infinite
    medium (40-digit root of the scalar system; no diffusion in a uniform
    state) and has the signs of its terms off it."""
    prob = _infinite_problem(e0, E0, dt)
    ptr, idx, fz = _be_parts(prob)
    e_ref, E_ref = _scalar_be_step(e0, E0, dt, 1.0)
    nin = prob.n_interior
    e = np.full(nin, float(e_ref))
    E = np.full(nin, float(E_ref))
    m, r = step.be_residual(prob, fz, ptr, idx, e, E)
    scale_m = max(e0, float(e_ref)) / dt
    scale_r = max(E0, float(E_ref)) / dt + float(e_ref) ** 4
    assert np.max(np.abs(m)) <= 1e-13 * scale_m and np.max(np.abs(r)) <= 1e-13 * scale_r
    # off the root, the signs of the derivatives: dm/de >= rho/dt, dr/dE >=
    # 1/dt, dm/dE = -c sigma_a
    m2, _ = step.be_residual(prob, fz, ptr, idx, e * (1 + 1e-6), E)
    m3, r3 = step.be_residual(prob, fz, ptr, idx, e, E * (1 + 1e-6))
    assert np.all(m2 > m) and np.all(r3 > r) and np.all(m3 < m)


@pytest.mark.parametrize("name", ["mms2d", "densitystep3d", "marshak3d"])
def test_be_residual_matches_the_assembled_system(name):
    """V_i r_i(e, E) = (A E - b(e, E))_i: the pair-sum residual against the
    assembled matrix and Algorithm 1's right-hand side evaluated at the same
    state (two separate paths of the oracle), at a perturbed state."""
    prob = {"mms2d": lambda: synth.config1(n=16), "densitystep3d": lambda: synth.config3(n=8),
            "marshak3d": lambda: synth.config4(n=10)}[name]()
    ptr, idx, fz = _be_parts(prob)
    sysm = operator.assemble(prob, ptr, idx, fz)
    nin = prob.n_interior
    rng = np.random.default_rng(5)
    e = prob.e[:nin] * (1 + 0.01 * rng.standard_normal(nin))
    E = prob.E[:nin] * (1 + 0.01 * rng.standard_normal(nin))
    m, r = step.be_residual(prob, fz, ptr, idx, e, E)
    b = operator.rhs(prob, fz, sysm, e, E)
    ref = sysm.A @ E - b
    scale = np.abs(sysm.A).dot(np.abs(E)) + np.abs(b)
    assert np.max(np.abs(fz.V[:nin] * r - ref) / scale) <= 1e-13
    B = prob.a * (e / prob.cv[:nin]) ** 4
    m_ref = (prob.rho[:nin] / prob.dt * (e - prob.e[:nin])
             + prob.c * fz.sigma_a[:nin] * (B - E) - prob.Q_e[:nin])
    assert np.array_equal(m, m_ref)


def test_be_residual_small_after_algorithm_1():
    """Algorithm 1 iterated to a tight outer tolerance reaches the root of G:
    both residuals far below their terms, and far below those of the state
    after one outer iteration."""
    prob = synth.config1(n=16)
    ptr, idx, fz = _be_parts(prob)
    nin = prob.n_interior
    one = step.time_step(prob.copy(), ptr, idx, fixed_outer=1, solve_tol=1e-15)
    full = step.time_step(prob.copy(), ptr, idx, eps_e=1e-14, eps_E=1e-14, solve_tol=1e-15)
    m1, r1 = step.be_residual(prob, fz, ptr, idx, one.e, one.E)
    mf, rf = step.be_residual(prob, fz, ptr, idx, full.e, full.E)
    scale_r = np.max(np.abs(prob.E[:nin])) / prob.dt
    assert np.max(np.abs(rf)) <= 1e-9 * scale_r
    assert np.max(np.abs(rf)) <= 1e-3 * np.max(np.abs(r1))
    assert np.max(np.abs(mf)) <= 1e-9 * np.max(np.abs(prob.rho[:nin] * full.e / prob.dt))
