"""rt_solve_noalloc (the solve for callers that cannot allocate) against
rt_solve through the C ABI: two calls in a row on one device, the second on a
smaller system, in FP64 and mixed precision, with the Jacobi and the V-cycle
preconditioner; the solutions agree to the parity bars (1e-12 FP64, 1e-10
mixed, relative to the largest unknown) and the iteration counts match.  A
system beyond the scratch array's limit is rejected with RT_E_ARG, and the
matrix's own carried residual is left alone."""
import numpy as np
import pytest

from gpu_common import gpu_system, say
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_11606_amd import rt
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rt.Context(0)
    yield c
    c.close()


def _rhs(n, seed, device):
    import torch
    rng = np.random.default_rng(seed)
    return torch.tensor(rng.uniform(0.5, 1.5, n) * 10.0 ** rng.uniform(-3.0, 0.0, n),
                        device=device)


@pytest.mark.parametrize("precision,precond", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_noalloc_matches_solve_twice(ctx, precision, precond):
    import torch
    from paper_2001_11606_amd import rt
    bar = 1e-12 if precision == 0 else 1e-10
    tol = 1e-13 if precision == 0 else 1e-11
    # the second call is on the smaller system
    for step, prob in enumerate((synth.config3(n=20), synth.config4(n=12))):
        say(f"[noalloc] call {step}: {prob.name} n={prob.n_interior} precision={precision} "
            f"precond={precond}")
        dp, nb, A = gpu_system(ctx, prob, amg=rt.amg_opts(max_levels=8, coarse_size=64))
        n = prob.n_interior
        b = _rhs(n, 100 + step, ctx.device)
        opts = rt.solve_opts(precision, precond, tol, 4000, 1e-4, 60, tol)
        x_ref = torch.zeros(n, dtype=torch.float64, device=ctx.device)
        s, st = ctx.solve(A, b, x_ref, opts)
        assert s == rt.RT_OK, rt.rt_last_error()
        x = torch.full((n,), 0.0, dtype=torch.float64, device=ctx.device)
        s2, st2 = rt.rt_solve_noalloc(ctx.handle, A, b.data_ptr(), x.data_ptr(), opts)
        torch.cuda.synchronize()
        assert s2 == rt.RT_OK, rt.rt_last_error()
        err = float((x - x_ref).abs().max() / x_ref.abs().max())
        assert err <= bar, (step, err)
        assert st2.iterations == st.iterations and st2.refinements == st.refinements
        assert st2.rel_residual <= tol and st2.cw_residual <= tol


def test_noalloc_rejects_too_large_and_keeps_carried_state(ctx):
    import torch
    from paper_2001_11606_amd import driver, rt
    prob = synth.config4(n=12)
    dp, nb, A = gpu_system(ctx, prob)
    n = prob.n_interior
    # outer iterations with the residual carried, with a no-allocation solve
    # in between on other data: the carried state must survive it
    e = dp.arrays["e"][:n].clone()
    E = dp.arrays["E"][:n].clone()
    opts = rt.newton_opts(rt.solve_opts(0, 0, 1e-13, 4000))
    ctx.newton_step(A, e, E, 0, opts)
    b = _rhs(n, 7, ctx.device)
    x = torch.zeros(n, dtype=torch.float64, device=ctx.device)
    rt.rt_solve_noalloc(ctx.handle, A, b.data_ptr(), x.data_ptr(), rt.solve_opts(0, 0, 1e-13, 4000))
    e1, E1 = e.clone(), E.clone()
    ctx.newton_step(A, e1, E1, 1, opts)
    A2 = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                      dp.limiter_k)
    e2, E2 = e.clone(), E.clone()
    ctx.newton_step(A2, e2, E2, 1, opts)   # a fresh matrix: no carried residual
    assert float(((E1 - E2).abs() / E2.abs()).max()) <= 1e-12


def test_noalloc_size_limit(ctx):
    """3,511,808 unknowns: within the FP64 limit (4,968,256), beyond the
    mixed-precision one (3,439,552)."""
    import torch
    from paper_2001_11606_amd import rt
    prob = synth.config3(n=152)
    say(f"[noalloc] size limit, n={prob.n_interior}")
    dp, nb, A = gpu_system(ctx, prob, amg=rt.amg_opts(max_levels=1))
    n = prob.n_interior
    b = _rhs(n, 3, ctx.device)
    x = torch.zeros(n, dtype=torch.float64, device=ctx.device)
    with pytest.raises(rt.RtError) as ei:
        rt.rt_solve_noalloc(ctx.handle, A, b.data_ptr(), x.data_ptr(),
                            rt.solve_opts(1, 0, 1e-10, 4000, 1e-4, 60))
    assert ei.value.code == rt.RT_E_ARG and "scratch" in str(ei.value)
    opts = rt.solve_opts(0, 0, 1e-10, 4000, 1e-4, 60, 1e-10)
    s, st = rt.rt_solve_noalloc(ctx.handle, A, b.data_ptr(), x.data_ptr(), opts)
    assert s == rt.RT_OK
    x_ref = torch.zeros_like(x)
    ctx.solve(A, b, x_ref, opts)
    assert float((x - x_ref).abs().max() / x_ref.abs().max()) <= 1e-12
