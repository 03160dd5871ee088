"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars: neighbour lists and CSR structure bit-exact; assembled values within
1e-13 of the row's largest entry; FP64 solves and Newton steps within 1e-12
relative, the mixed-precision path within 1e-10 relative in E and e.
"""
import numpy as np
import pytest

import synth
from gpu_common import gpu_system, oracle_system, rowwise_rel_err, say, small_cases
from oracle import linsolve, step as ostep

pytestmark = pytest.mark.gpu

CASES = small_cases()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_11606_amd import rt
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def systems():
    return {}


def _get(systems, name):
    if name not in systems:
        prob = CASES[name]()
        systems[name] = (prob, oracle_system(prob))
    return systems[name]


@pytest.mark.parametrize("name", list(CASES))
def test_neighbors_bit_exact(ctx, systems, name):
    prob, (ptr, idx, fz, sysm) = _get(systems, name)
    say(f"[neighbors] {name} n_total={prob.n_total} n_interior={prob.n_interior}")
    dp, nb, A = gpu_system(ctx, prob)
    gptr, gidx = ctx.export_neighbors(nb)
    assert nb.info.npairs == idx.shape[0]
    assert np.array_equal(gptr.cpu().numpy(), ptr)
    assert np.array_equal(gidx.cpu().numpy(), idx)


@pytest.mark.parametrize("name", list(CASES))
def test_matrix_parity(ctx, systems, name):
    prob, (ptr, idx, fz, sysm) = _get(systems, name)
    say(f"[assemble] {name}")
    dp, nb, A = gpu_system(ctx, prob)
    rp, col, val, g = [t.cpu().numpy() for t in ctx.export_matrix(A)]
    assert np.array_equal(rp, sysm.A.indptr.astype(np.int64))
    assert np.array_equal(col, sysm.A.indices.astype(np.int32))
    assert rowwise_rel_err(rp, val, sysm.A.data) <= 1e-13
    gs = np.max(np.abs(sysm.A.diagonal()))
    assert np.max(np.abs(g - sysm.g), initial=0.0) <= 1e-13 * gs


def _solve_case(ctx, systems, name, precision, precond, tol, amg=None):
    """One solve against the dense or oracle solution, scored by the max-norm
    relative error max|x - x_ref| / max|x_ref|: the right-hand side has mixed
    signs, so unknowns cross zero and a pointwise relative error is undefined
    there.  Pointwise relative errors over eight decades of positive unknowns
    are what test_solve_componentwise and the Newton-step tests hold."""
    from paper_2001_11606_amd import rt
    import torch
    prob, (ptr, idx, fz, sysm) = _get(systems, name)
    nin = prob.n_interior
    b = np.random.default_rng(17).standard_normal(nin) * sysm.A.diagonal()
    x_ref = linsolve.dense(sysm.A, b) if nin <= 5000 else linsolve.pcg_jacobi(sysm.A, b, tol=1e-15)[0]
    dp, nb, A = gpu_system(ctx, prob, amg=amg)
    bt = torch.tensor(b, device=ctx.device)
    xt = torch.zeros(nin, dtype=torch.float64, device=ctx.device)
    status, st = ctx.solve(A, bt, xt, rt.solve_opts(precision, precond, tol, 2000, 1e-4, 50))
    assert status == rt.RT_OK, rt.rt_last_error()
    x = xt.cpu().numpy()
    return np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref)), st


@pytest.mark.parametrize("name", ["mms2d_64", "densitystep3d_16", "marshak3d_16", "ensemble3d"])
@pytest.mark.parametrize("precond", [0, 1])
def test_solve_fp64(ctx, systems, name, precond):
    say(f"[solve fp64] {name} precond={precond}")
    err, st = _solve_case(ctx, systems, name, 0, precond, 1e-14)
    assert err <= 1e-12, (err, st.iterations)


@pytest.mark.parametrize("name", ["mms2d_64", "densitystep3d_16", "marshak3d_16", "ensemble3d"])
@pytest.mark.parametrize("precond", [0, 1])
def test_solve_mixed(ctx, systems, name, precond):
    say(f"[solve mixed] {name} precond={precond}")
    err, st = _solve_case(ctx, systems, name, 1, precond, 1e-12)
    assert err <= 1e-10, (err, st.iterations, st.refinements)
    assert st.refinements >= 1


@pytest.mark.parametrize("name", ["mms2d_64", "densitystep3d_16", "marshak3d_16", "wendland3d_9",
                                  "periodic3d_13"])
@pytest.mark.parametrize("degree", [2, 3])
def test_solve_chebyshev_vcycle(ctx, systems, name, degree):
    """The V-cycle with the Chebyshev smoother: FP64 and mixed solves reach the
    oracle's solution; the iteration counts are printed beside the l1-Jacobi
    V-cycle's."""
    from paper_2001_11606_amd import rt
    say(f"[solve chebyshev] {name} degree={degree}")
    cheb = rt.amg_opts(smoother=rt.RT_SMOOTHER_CHEBYSHEV, smoother_degree=degree)
    err, st = _solve_case(ctx, systems, name, 0, 1, 1e-14, amg=cheb)
    assert err <= 1e-12, (err, st.iterations)
    err32, st32 = _solve_case(ctx, systems, name, 1, 1, 1e-12, amg=cheb)
    assert err32 <= 1e-10, (err32, st32.iterations)
    _, st_l1 = _solve_case(ctx, systems, name, 0, 1, 1e-14)
    say(f"  iterations fp64: chebyshev {st.iterations}, l1-jacobi {st_l1.iterations}")


def _newton_case(ctx, name, precision, precond, outer):
    from paper_2001_11606_amd import driver, rt
    prob = CASES[name]()
    say(f"[newton] {name} precision={precision} precond={precond} outer={outer}")
    ref = ostep.time_step(prob.copy(), fixed_outer=outer, inner_tol_e=1e-14, solve_tol=1e-15)
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior, prob.kernel, period=dp.period)
    tol = 1e-14 if precision == 0 else 1e-12
    e, E, A, rep = driver.time_step(ctx, dp, nb, solve=rt.solve_opts(precision, precond, tol, 2000),
                                    fixed_outer=outer)
    assert rep.status == rt.RT_OK
    e, E = e.cpu().numpy(), E.cpu().numpy()
    err_e = np.max(np.abs(e - ref.e) / np.abs(ref.e))
    err_E = np.max(np.abs(E - ref.E) / np.abs(ref.E))
    return err_e, err_E, rep, ref


@pytest.mark.parametrize("name", ["marshak3d_16", "densitystep3d_16", "mms2d_64", "wendland3d_9",
                                  "densitystep3d_12_coldpatch"])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("precond", [0, 1])
def test_solve_componentwise(ctx, systems, name, precision, precond):
    """With the componentwise test every unknown is accurate, not only the
    largest: b = diag(A) 10^u with u uniform in [-8, 0] gives a positive
    solution spanning about eight decades, and the pointwise relative error
    against the oracle's solve (itself accurate per unknown) is held to
    1e-12 (FP64, tolerances 1e-14) or 1e-10 (mixed, tolerances 1e-12)."""
    import torch
    from paper_2001_11606_amd import rt
    prob, (ptr, idx, fz, sysm) = _get(systems, name)
    nin = prob.n_interior
    say(f"[solve componentwise] {name} precision={precision} precond={precond}")
    b = sysm.A.diagonal() * 10.0 ** np.random.default_rng(23).uniform(-8.0, 0.0, nin)
    x_ref = linsolve.solve(sysm.A, b, tol=1e-15)
    assert np.all(x_ref > 0.0)
    dp, nb, A = gpu_system(ctx, prob)
    tol, bar = (1e-14, 1e-12) if precision == 0 else (1e-12, 1e-10)
    bt = torch.tensor(b, device=ctx.device)
    xt = torch.zeros(nin, dtype=torch.float64, device=ctx.device)
    status, st = ctx.solve(A, bt, xt, rt.solve_opts(precision, precond, tol, 4000, 1e-4, 60, tol))
    assert status == rt.RT_OK, rt.rt_last_error()
    x = xt.cpu().numpy()
    err = np.max(np.abs(x - x_ref) / x_ref)
    assert st.cw_residual <= tol
    assert err <= bar, (err, st.iterations, st.refinements, st.cw_residual)


def test_componentwise_option_errors(ctx, systems):
    from paper_2001_11606_amd import rt
    import torch
    prob, _ = _get(systems, "marshak3d_16")
    dp, nb, A = gpu_system(ctx, prob)
    b = torch.ones(prob.n_interior, dtype=torch.float64, device=ctx.device)
    x = torch.zeros_like(b)
    for cw in (-1e-12, float("nan")):
        with pytest.raises(rt.RtError) as ei:
            ctx.solve(A, b, x, rt.solve_opts(0, 0, 1e-12, 100, 1e-4, 10, cw))
        assert ei.value.code == rt.RT_E_ARG


@pytest.mark.parametrize("name", ["marshak3d_16", "densitystep3d_16", "mms2d_64",
                                  "densitystep3d_12_coldpatch"])
@pytest.mark.parametrize("precision", [0, 1])
def test_newton_componentwise(ctx, name, precision):
    """Three outer iterations with the componentwise test on: pointwise
    relative errors in e and E against the oracle, 1e-12 (FP64) or 1e-10
    (mixed)."""
    from paper_2001_11606_amd import driver, rt
    prob = CASES[name]()
    say(f"[newton componentwise] {name} precision={precision}")
    ref = ostep.time_step(prob.copy(), fixed_outer=3, inner_tol_e=1e-14, solve_tol=1e-15)
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior, prob.kernel, period=dp.period)
    tol, bar = (1e-14, 1e-12) if precision == 0 else (1e-12, 1e-10)
    e, E, A, rep = driver.time_step(ctx, dp, nb,
                                    solve=rt.solve_opts(precision, 0, tol, 4000, 1e-4, 60, tol),
                                    fixed_outer=3)
    assert rep.status == rt.RT_OK
    e, E = e.cpu().numpy(), E.cpu().numpy()
    err_e = np.max(np.abs(e - ref.e) / np.abs(ref.e))
    err_E = np.max(np.abs(E - ref.E) / np.abs(ref.E))
    assert err_e <= bar and err_E <= bar, (err_e, err_E, rep.krylov, rep.refinements)


@pytest.mark.parametrize("name", ["mms2d_64", "mms3d_12", "densitystep3d_16", "marshak3d_16",
                                  "infinite3d_10", "densitystep3d_16_levermore", "wendland2d_24",
                                  "wendland3d_9", "periodic2d_16", "periodic3d_13",
                                  "periodicx_ghostsy2d_32"])
def test_newton_fp64(ctx, name):
    err_e, err_E, rep, ref = _newton_case(ctx, name, 0, 1, 3)
    assert err_e <= 1e-12 and err_E <= 1e-12, (err_e, err_E)
    # convergence measures and energy follow the oracle
    assert np.allclose(rep.delta_e, ref.delta_e, rtol=1e-6, atol=1e-14)
    assert rep.energy == pytest.approx(ref.energy_after, rel=1e-13)
    assert rep.energy_prev == pytest.approx(ref.energy_before, rel=1e-13)


@pytest.mark.parametrize("name", ["mms2d_64", "densitystep3d_16", "marshak3d_16"])
def test_newton_mixed(ctx, name):
    err_e, err_E, rep, ref = _newton_case(ctx, name, 1, 1, 3)
    assert err_e <= 1e-10 and err_E <= 1e-10, (err_e, err_E)


def test_deterministic(ctx):
    from paper_2001_11606_amd import driver, rt
    prob = CASES["densitystep3d_16"]()
    say("[determinism] densitystep3d_16 mixed AMG twice")
    outs = []
    for _ in range(2):
        dp = driver.upload(prob, ctx.device)
        nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior, prob.kernel)
        e, E, A, rep = driver.time_step(ctx, dp, nb, solve=rt.solve_opts(1, 1, 1e-10, 500),
                                        fixed_outer=2)
        outs.append((e.cpu().numpy().tobytes(), E.cpu().numpy().tobytes()))
    assert outs[0] == outs[1]


@pytest.mark.parametrize("name,strength", [("marshak3d_16", 0.0), ("diffusive3d_16", 0.25)])
def test_deep_hierarchy_repeated_setup(ctx, name, strength):
    """Several set-ups of a many-level hierarchy in one process (device memory
    recycled between them): every coarse level must be complete before it is
    coarsened again, and AMG-preconditioned solves must match the oracle.
    The Marshak rows are dominated by their diagonals, so the strength test
    would keep them on one level: there the aggregation is geometric."""
    import torch
    from paper_2001_11606_amd import rt
    prob = CASES[name]()
    ptr, idx, fz, sysm = oracle_system(prob)
    nin = prob.n_interior
    b = np.random.default_rng(5).standard_normal(nin) * sysm.A.diagonal()
    x_ref = linsolve.dense(sysm.A, b)
    for rep in range(3):
        say(f"[deep hierarchy] {name} strength {strength} set-up {rep}")
        dp, nb, A = gpu_system(ctx, prob, amg=rt.amg_opts(max_levels=8, coarse_size=8,
                                                          strength=strength))
        assert ctx.matrix_info(A).levels >= 4
        bt = torch.tensor(b, device=ctx.device)
        for prec, tol, bar in ((0, 1e-14, 1e-12), (1, 1e-12, 1e-10)):
            xt = torch.zeros(nin, dtype=torch.float64, device=ctx.device)
            status, st = ctx.solve(A, bt, xt, rt.solve_opts(prec, 1, tol, 2000, 1e-4, 50))
            assert status == rt.RT_OK
            err = np.max(np.abs(xt.cpu().numpy() - x_ref)) / np.max(np.abs(x_ref))
            assert err <= bar, (rep, prec, err)


@pytest.mark.parametrize("precision", [0, 1])
def test_newton_residual_carry(ctx, precision):
    """From the second outer iteration on, the initial residual of the solve
    is the last solve's residual plus the change of the right-hand side.  It
    is used only when E^l is bit for bit the last solution: with E perturbed
    between the calls, the step must equal one taken without carried state
    (matrix re-assembled first) bit for bit; unperturbed, it must agree with
    that one to the solve tolerance."""
    import torch
    from paper_2001_11606_amd import driver, rt
    say(f"[newton carry] precision={precision}")
    prob = synth.config4(n=12)
    nin = prob.n_interior
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, nin, prob.kernel)
    tol = 1e-14 if precision == 0 else 1e-12
    nopts = rt.newton_opts(rt.solve_opts(precision, 0, tol, 2000, 1e-4, 50))
    bump = torch.tensor(1.0 + 1e-3 * np.cos(np.arange(nin)), device=ctx.device)

    def run(perturb, fresh):
        A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                         dp.limiter_k, amg=rt.amg_opts(max_levels=1))
        e = dp.arrays["e"][:nin].clone()
        E = dp.arrays["E"][:nin].clone()
        s, _ = ctx.newton_step(A, e, E, 0, nopts)
        assert s == rt.RT_OK
        if perturb:
            E.mul_(bump)
        if fresh:   # re-assembly drops every carried residual
            ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                         dp.limiter_k, amg=rt.amg_opts(max_levels=1), A=A)
        s, st = ctx.newton_step(A, e, E, 1, nopts)
        assert s == rt.RT_OK
        out = (e.cpu().numpy(), E.cpu().numpy(), st.solve.rel_residual)
        rt.rt_matrix_free(A)
        ctx._owned = [o for o in ctx._owned if o[1] != A]
        return out

    e1, E1, r1 = run(True, False)
    e2, E2, r2 = run(True, True)
    assert np.array_equal(e1, e2) and np.array_equal(E1, E2)
    e3, E3, r3 = run(False, False)
    e4, E4, r4 = run(False, True)
    assert r3 <= tol and r4 <= tol
    bar = 1e-12 if precision == 0 else 1e-10
    assert np.max(np.abs(E3 - E4) / np.abs(E4)) <= bar
    assert np.max(np.abs(e3 - e4) / np.abs(e4)) <= bar


@pytest.mark.parametrize("name", ["mms2d_64", "densitystep3d_16", "marshak3d_16"])
@pytest.mark.parametrize("precond,restart,cheb", [(0, 30, False), (1, 30, False), (1, 5, False),
                                                  (1, 30, True)])
def test_gmres_unscaled_matches_oracle(ctx, systems, name, precond, restart, cheb):
    """GMRES on the paper's unscaled operator reaches the oracle's solution of
    the same system (the V-scaling does not change x), restarts included;
    cheb: the V-cycle with the Chebyshev smoother."""
    import torch
    from paper_2001_11606_amd import rt
    prob, (ptr, idx, fz, sysm) = _get(systems, name)
    say(f"[gmres] {name} precond={precond} restart={restart} chebyshev={cheb}")
    nin = prob.n_interior
    b = np.random.default_rng(29).standard_normal(nin) * sysm.A.diagonal()
    x_ref = linsolve.dense(sysm.A, b) if nin <= 5000 else linsolve.pcg_jacobi(sysm.A, b, tol=1e-15)[0]
    amg = rt.amg_opts(smoother=rt.RT_SMOOTHER_CHEBYSHEV, smoother_degree=2) if cheb else None
    dp, nb, A = gpu_system(ctx, prob, amg=amg)
    bt = torch.tensor(b, device=ctx.device)
    xt = torch.zeros(nin, dtype=torch.float64, device=ctx.device)
    s, st = ctx.solve_gmres(A, bt, xt, rt.gmres_opts(precond, 1e-13, 5000, restart))
    assert s == rt.RT_OK, rt.rt_last_error()
    x = xt.cpu().numpy()
    assert np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref)) <= 1e-10
    # the reported residual is that of the unscaled system, recomputed here
    V = fz.V[:nin]
    ru = (b - sysm.A @ x) / V
    assert np.linalg.norm(ru) / np.linalg.norm(b / V) <= 1.05e-13
    assert st.rel_residual <= 1e-13 and st.iterations > 0


def test_gmres_not_converged_and_errors(ctx, systems):
    import torch
    from paper_2001_11606_amd import rt
    prob, (ptr, idx, fz, sysm) = _get(systems, "mms2d_64")
    nin = prob.n_interior
    dp, nb, A = gpu_system(ctx, prob)
    bt = torch.ones(nin, dtype=torch.float64, device=ctx.device)
    xt = torch.zeros_like(bt)
    s, st = ctx.solve_gmres(A, bt, xt, rt.gmres_opts(0, 1e-14, 3, 30))
    assert s == rt.RT_NOT_CONVERGED and st.iterations == 3 and st.rel_residual > 1e-14
    for bad in (rt.gmres_opts(2, 1e-10, 10, 30), rt.gmres_opts(0, -1.0, 10, 30),
                rt.gmres_opts(0, 1e-10, 10, 0), rt.gmres_opts(0, 1e-10, 10, 65)):
        with pytest.raises(rt.RtError):
            ctx.solve_gmres(A, bt, xt, bad)
