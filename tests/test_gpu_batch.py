"""Batched ensembles through the C ABI against the oracle, problem by problem.

An ensemble of independent problems (the 2-D / 3-D mix of the ensemble
workload, shrunk) is concatenated into one block-diagonal system.  Every
problem's solution must match its own oracle solve (FP64 to 1e-12, mixed to
1e-10, max-norm relative) whatever the graph replay length, and a batched
Newton step must match the oracle's time step per problem.  An ensemble of
diffusive problems with their own aggregation hierarchies does the same with
the batch's V-cycle (the problems' levels concatenated), whose iterations
replayed from graphs must give bitwise the iterates of eager launches.
"""
import numpy as np
import pytest

from gpu_common import gpu_system, oracle_system, say
from oracle import linsolve, step as ostep
import synth

pytestmark = pytest.mark.gpu

SIZES = (150.0, 2200.0, 90.0, 5000.0, 700.0, 12000.0, 64.0, 3000.0)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_11606_amd import rt
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ensemble(ctx):
    from paper_2001_11606_amd import rt
    probs = [synth.config5_member(q, s) for q, s in enumerate(SIZES)]
    systems = [gpu_system(ctx, pr, amg=rt.amg_opts(max_levels=1)) for pr in probs]
    B = rt.rt_batch_create(ctx.handle, [A for (_, _, A) in systems])
    yield probs, systems, B
    rt.rt_batch_free(B)


def _offsets(probs):
    return np.cumsum([0] + [pr.n_interior for pr in probs])


def _rhs(probs):
    rng = np.random.default_rng(31)
    bs, refs = [], []
    for pr in probs:
        A = oracle_system(pr)[3].A
        b = rng.standard_normal(pr.n_interior) * A.diagonal()
        bs.append(b)
        refs.append(linsolve.dense(A, b) if pr.n_interior <= 4000
                    else linsolve.pcg_jacobi(A, b, tol=1e-15)[0])
    return bs, refs


@pytest.mark.parametrize("precision,tol,bar", [(0, 1e-14, 1e-12), (1, 1e-12, 1e-10)])
@pytest.mark.parametrize("graph", [0, 4])
def test_batch_solve_matches_oracle(ctx, ensemble, precision, tol, bar, graph):
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, B = ensemble
    say(f"[batch solve] precision={precision} graph={graph} problems={len(probs)}")
    bs, refs = _rhs(probs)
    offs = _offsets(probs)
    b = torch.tensor(np.concatenate(bs), device=ctx.device)
    x = torch.zeros(offs[-1], dtype=torch.float64, device=ctx.device)
    s, st = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                              rt.solve_opts(precision, 0, tol, 4000, 1e-4, 50), graph)
    assert s == rt.RT_OK, rt.rt_last_error()
    xh = x.cpu().numpy()
    for q, pr in enumerate(probs):
        err = np.max(np.abs(xh[offs[q]:offs[q + 1]] - refs[q])) / np.max(np.abs(refs[q]))
        assert err <= bar, (q, err, st[q].iterations)
        assert st[q].rel_residual <= tol
        if precision == 1:
            assert st[q].refinements >= 1


def test_batch_solve_equals_single_solves(ctx, ensemble):
    """Each problem's batched FP64 solve reaches the same tolerance as its own
    rt_solve, and the problems converge independently (different counts)."""
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, B = ensemble
    bs, refs = _rhs(probs)
    offs = _offsets(probs)
    b = torch.tensor(np.concatenate(bs), device=ctx.device)
    x = torch.zeros(offs[-1], dtype=torch.float64, device=ctx.device)
    s, st = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                              rt.solve_opts(0, 0, 1e-12, 4000), 0)
    assert s == rt.RT_OK
    its_batch = [st[q].iterations for q in range(len(probs))]
    its_single = []
    for q, (dp, nb, A) in enumerate(systems):
        xq = torch.zeros(probs[q].n_interior, dtype=torch.float64, device=ctx.device)
        s1, st1 = ctx.solve(A, b[offs[q]:offs[q + 1]].clone(), xq, rt.solve_opts(0, 0, 1e-12, 4000))
        assert s1 == rt.RT_OK
        its_single.append(st1.iterations)
    say(f"[batch] iterations batched {its_batch} single {its_single}")
    # same algorithm; the reductions round differently, so allow one iteration either way
    assert all(abs(a - b) <= 1 for a, b in zip(its_batch, its_single))
    assert len(set(its_batch)) > 1


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_newton_matches_oracle(ctx, ensemble, precision):
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, B = ensemble
    say(f"[batch newton] precision={precision}")
    offs = _offsets(probs)
    e = torch.tensor(np.concatenate([pr.e[:pr.n_interior] for pr in probs]), device=ctx.device)
    E = torch.tensor(np.concatenate([pr.E[:pr.n_interior] for pr in probs]), device=ctx.device)
    tol = 1e-14 if precision == 0 else 1e-12
    nopts = rt.newton_opts(rt.solve_opts(precision, 0, tol, 4000, 1e-4, 50))
    for ell in range(3):
        s, st = rt.rt_batch_newton_step(ctx.handle, B, len(probs), e.data_ptr(), E.data_ptr(), ell,
                                        nopts, 4)
        assert s == rt.RT_OK, rt.rt_last_error()
    eh, Eh = e.cpu().numpy(), E.cpu().numpy()
    bar = 1e-12 if precision == 0 else 1e-10
    for q, pr in enumerate(probs):
        ref = ostep.time_step(pr.copy(), fixed_outer=3, inner_tol_e=1e-14, solve_tol=1e-15)
        err_e = np.max(np.abs(eh[offs[q]:offs[q + 1]] - ref.e) / np.abs(ref.e))
        err_E = np.max(np.abs(Eh[offs[q]:offs[q + 1]] - ref.E) / np.abs(ref.E))
        assert err_e <= bar and err_E <= bar, (q, err_e, err_E)
        if precision == 0:
            assert st[q].energy == pytest.approx(ref.energy_after, rel=1e-12)


def test_batch_tune_and_errors(ctx, ensemble):
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, B = ensemble
    rep = rt.rt_batch_tune(ctx.handle, B, 2)
    assert rep.levels == 1 and 0 <= rep.chosen[0][0] < rep.shapes
    offs = _offsets(probs)
    b = torch.ones(offs[-1], dtype=torch.float64, device=ctx.device)
    x = torch.zeros_like(b)
    # one-level matrices: the batch has no hierarchy and precond 1 is Jacobi
    s1, st1 = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                                rt.solve_opts(0, 1, 1e-10, 4000), 0)
    x.zero_()
    s0, st0 = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                                rt.solve_opts(0, 0, 1e-10, 4000), 0)
    assert s1 == s0 == rt.RT_OK
    assert [st1[q].iterations for q in range(len(probs))] == [st0[q].iterations
                                                               for q in range(len(probs))]
    with pytest.raises(rt.RtError):   # the componentwise test is not offered for batches
        rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                          rt.solve_opts(0, 0, 1e-10, 100, 1e-4, 60, 1e-10), 0)
    with pytest.raises(rt.RtError):
        rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                          rt.solve_opts(0, 0, 1e-10, 100), -1)
    with pytest.raises(rt.RtError):
        rt.rt_batch_create(ctx.handle, [])
    with pytest.raises(rt.RtError):   # negative depth
        rt.rt_batch_set_cycle_depth(B, -1)
    with pytest.raises(rt.RtError):   # the depth tuner times V-cycle solves only
        rt.rt_batch_tune_depth(ctx.handle, B, b.data_ptr(), x.data_ptr(),
                               rt.solve_opts(0, 0, 1e-10, 100), 0, 1)
    # a batch without a hierarchy: one depth, nothing to tune
    rep = rt.rt_batch_tune_depth(ctx.handle, B, b.data_ptr(), x.data_ptr(),
                                 rt.solve_opts(0, 1, 1e-10, 100), 0, 1)
    assert rep.depths == 1 and rep.chosen == 1


def test_full_ensemble_sampled_against_oracle(ctx):
    """The full 96-problem ensemble of the bench (11.8M particles, one batch,
    graph-replayed PCG): the batched Newton step's e and E of the smallest
    problems match the oracle's step to the mixed bar, and every problem's
    reported FP64 residual meets the tolerance."""
    import torch
    from paper_2001_11606_amd import driver, rt
    probs = synth.config5(96)
    say(f"[full ensemble] {sum(p.n_interior for p in probs)} particles")
    amg = rt.amg_opts(max_levels=1, build_fp32=1)
    handles = []
    for pr in probs:
        dp = driver.upload(pr, ctx.device)
        nb = ctx.build_neighbors(dp.pos, dp.h, dp.n_interior, dp.kernel)
        A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                         dp.limiter_k, amg=amg)
        handles.append((nb, A))
    B = rt.rt_batch_create(ctx.handle, [A for _, A in handles])
    try:
        offs = _offsets(probs)
        e = torch.tensor(np.concatenate([pr.e[:pr.n_interior] for pr in probs]), device=ctx.device)
        E = torch.tensor(np.concatenate([pr.E[:pr.n_interior] for pr in probs]), device=ctx.device)
        tol = 1e-12
        nopts = rt.newton_opts(rt.solve_opts(rt.RT_PREC_MIXED, 0, tol, 5000, 1e-4, 50))
        s, st = rt.rt_batch_newton_step(ctx.handle, B, len(probs), e.data_ptr(), E.data_ptr(), 0,
                                        nopts, 8)
        assert s == rt.RT_OK, rt.rt_last_error()
        assert all(st[q].solve.rel_residual <= tol for q in range(len(probs)))
        eh, Eh = e.cpu().numpy(), E.cpu().numpy()
        smallest = sorted(range(len(probs)), key=lambda q: probs[q].n_interior)[:3]
        for q in smallest:
            ref = ostep.time_step(probs[q].copy(), fixed_outer=1, inner_tol_e=1e-14,
                                  solve_tol=1e-15)
            err_e = np.max(np.abs(eh[offs[q]:offs[q + 1]] - ref.e) / np.abs(ref.e))
            err_E = np.max(np.abs(Eh[offs[q]:offs[q + 1]] - ref.E) / np.abs(ref.E))
            say(f"[full ensemble] problem {q} ({probs[q].n_interior} particles): "
                f"e {err_e:.1e} E {err_E:.1e}")
            assert err_e <= 1e-10 and err_E <= 1e-10, (q, err_e, err_E)
    finally:
        rt.rt_batch_free(B)
        for nb, A in handles:
            rt.rt_matrix_free(A)
            rt.rt_neighbors_free(nb.handle)
        ctx._owned.clear()


AMG_SIZES = (150.0, 2200.0, 700.0, 5000.0, 300.0)


@pytest.fixture(scope="module")
def ensemble_amg(ctx):
    from paper_2001_11606_amd import rt
    probs = []
    for q, size in enumerate(AMG_SIZES):
        pr = synth.config5_member(q, size)
        pr.dt = 0.1   # diffusion-dominated: the strength test coarsens the rows
        probs.append(pr)
    systems = [gpu_system(ctx, pr, amg=rt.amg_opts(max_levels=8, coarse_size=16)) for pr in probs]
    levels = [ctx.matrix_info(A).levels for (_, _, A) in systems]
    B = rt.rt_batch_create(ctx.handle, [A for (_, _, A) in systems])
    yield probs, systems, B, levels
    rt.rt_batch_free(B)


@pytest.mark.parametrize("precision,tol,bar", [(0, 1e-14, 1e-12), (1, 1e-12, 1e-10)])
def test_batch_amg_solve_matches_oracle(ctx, ensemble_amg, precision, tol, bar):
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, B, levels = ensemble_amg
    assert max(levels) >= 3, levels
    offs = _offsets(probs)
    bs, refs = _rhs(probs)
    b = torch.tensor(np.concatenate(bs), device=ctx.device)
    its, sols = {}, {}
    for precond, graph in ((1, 0), (0, 0), (1, 4)):
        x = torch.zeros_like(b)
        s, st = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                                  rt.solve_opts(precision, precond, tol, 4000, 1e-4, 60), graph)
        assert s == rt.RT_OK, rt.rt_last_error()
        its[(precond, graph)] = [st[q].iterations for q in range(len(probs))]
        xh = sols[(precond, graph)] = x.cpu().numpy()
        for q in range(len(probs)):
            err = np.max(np.abs(xh[offs[q]:offs[q + 1]] - refs[q])) / np.max(np.abs(refs[q]))
            assert err <= bar, (precond, graph, q, err)
    say(f"[batch amg] precision={precision} levels {levels}: iterations V-cycle {its[(1, 0)]}, "
        f"Jacobi {its[(0, 0)]}")
    assert sum(its[(1, 0)]) < sum(its[(0, 0)])
    # V-cycle iterations replayed from graphs: the same iterates as launched one by one
    assert its[(1, 4)] == its[(1, 0)]
    assert np.array_equal(sols[(1, 4)], sols[(1, 0)])


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_amg_newton_matches_oracle(ctx, ensemble_amg, precision):
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, B, levels = ensemble_amg
    offs = _offsets(probs)
    e = torch.tensor(np.concatenate([pr.e[:pr.n_interior] for pr in probs]), device=ctx.device)
    E = torch.tensor(np.concatenate([pr.E[:pr.n_interior] for pr in probs]), device=ctx.device)
    tol = 1e-14 if precision == 0 else 1e-12
    nopts = rt.newton_opts(rt.solve_opts(precision, 1, tol, 4000, 1e-4, 50))
    for ell in range(3):
        s, st = rt.rt_batch_newton_step(ctx.handle, B, len(probs), e.data_ptr(), E.data_ptr(), ell,
                                        nopts, 4 * (ell % 2))
        assert s == rt.RT_OK, rt.rt_last_error()
    eh, Eh = e.cpu().numpy(), E.cpu().numpy()
    bar = 1e-12 if precision == 0 else 1e-10
    for q, pr in enumerate(probs):
        ref = ostep.time_step(pr.copy(), fixed_outer=3, inner_tol_e=1e-14, solve_tol=1e-15)
        err_e = np.max(np.abs(eh[offs[q]:offs[q + 1]] - ref.e) / np.abs(ref.e))
        err_E = np.max(np.abs(Eh[offs[q]:offs[q + 1]] - ref.E) / np.abs(ref.E))
        assert err_e <= bar and err_E <= bar, (q, err_e, err_E)


def test_batch_amg_tune(ctx, ensemble_amg):
    from paper_2001_11606_amd import rt
    probs, systems, B, levels = ensemble_amg
    rep = rt.rt_batch_tune(ctx.handle, B, 2)
    assert rep.levels == max(levels)
    assert all(0 <= rep.chosen[l][0] < rep.shapes for l in range(rep.levels))


def test_batch_amg_depth_per_problem(ctx, ensemble_amg):
    """Each problem enters the batch's hierarchy with its own V-cycle depth
    (set on its matrix): the batch has as many levels as the deepest, every
    problem still matches the oracle, and with every depth 1 the batch has no
    hierarchy (precond 1 is Jacobi)."""
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, _, levels = ensemble_amg
    mats = [A for (_, _, A) in systems]
    depths = [1, 2, 0, 3, 2]   # 0: every level
    offs = _offsets(probs)
    bs, refs = _rhs(probs)
    b = torch.tensor(np.concatenate(bs), device=ctx.device)
    try:
        for A, d in zip(mats, depths):
            rt.rt_matrix_set_cycle_depth(A, d)
        B = rt.rt_batch_create(ctx.handle, mats)
        try:
            used = [levels[q] if d == 0 else min(d, levels[q]) for q, d in enumerate(depths)]
            assert rt.rt_batch_tune(ctx.handle, B, 1).levels == max(used)
            its = {}
            for precond in (1, 0):
                x = torch.zeros_like(b)
                s, st = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                                          rt.solve_opts(0, precond, 1e-14, 4000, 1e-4, 60), 0)
                assert s == rt.RT_OK, rt.rt_last_error()
                its[precond] = [st[q].iterations for q in range(len(probs))]
                xh = x.cpu().numpy()
                for q in range(len(probs)):
                    err = np.max(np.abs(xh[offs[q]:offs[q + 1]] - refs[q])) / np.max(np.abs(refs[q]))
                    assert err <= 1e-12, (precond, q, err)
            say(f"[batch depth] depths {used}: iterations V-cycle {its[1]}, Jacobi {its[0]}")
            # a problem of depth 1 takes two l1-Jacobi sweeps per application,
            # the deeper ones their coarse corrections: none more than Jacobi
            assert all(a <= j for a, j in zip(its[1], its[0]))
            assert sum(its[1]) < sum(its[0])
        finally:
            rt.rt_batch_free(B)
        for A in mats:
            rt.rt_matrix_set_cycle_depth(A, 1)
        B1 = rt.rt_batch_create(ctx.handle, mats)
        try:
            assert rt.rt_batch_tune(ctx.handle, B1, 1).levels == 1
        finally:
            rt.rt_batch_free(B1)
    finally:
        for A in mats:
            rt.rt_matrix_set_cycle_depth(A, 0)


@pytest.mark.parametrize("graph", [0, 4])
def test_batch_amg_zero_rhs_problem(ctx, ensemble_amg, graph):
    """A problem with b = 0 has stopped before the first V-cycle (the skipped
    rows of its levels are never written in the solve): its solution is
    exactly zero, and the other problems still match the oracle."""
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, B, levels = ensemble_amg
    offs = _offsets(probs)
    bs, refs = _rhs(probs)
    zero = 2
    bs[zero] = np.zeros_like(bs[zero])
    b = torch.tensor(np.concatenate(bs), device=ctx.device)
    for precision, tol, bar in ((0, 1e-14, 1e-12), (1, 1e-12, 1e-10)):
        x = torch.zeros_like(b)
        s, st = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                                  rt.solve_opts(precision, 1, tol, 4000, 1e-4, 60), graph)
        assert s == rt.RT_OK, rt.rt_last_error()
        xh = x.cpu().numpy()
        assert st[zero].iterations == 0
        assert not np.any(xh[offs[zero]:offs[zero + 1]])
        for q in range(len(probs)):
            if q == zero:
                continue
            err = np.max(np.abs(xh[offs[q]:offs[q + 1]] - refs[q])) / np.max(np.abs(refs[q]))
            assert err <= bar, (precision, q, err)


def test_full_ensemble_vcycle_sampled_against_oracle(ctx):
    """The full 96-problem ensemble of the bench, each problem assembled with
    its own aggregation hierarchy (1 to 7 levels, 2-D and 3-D mixed): one
    batched mixed Newton step with the batch's V-cycle meets the tolerance
    for every problem, and the three smallest problems match the oracle's
    step to the mixed bar."""
    import torch
    from paper_2001_11606_amd import driver, rt
    probs = synth.config5(96)
    amg = rt.amg_opts(build_fp32=1)
    handles = []
    for pr in probs:
        dp = driver.upload(pr, ctx.device)
        nb = ctx.build_neighbors(dp.pos, dp.h, dp.n_interior, dp.kernel)
        A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                         dp.limiter_k, amg=amg)
        handles.append((nb, A))
    levels = [ctx.matrix_info(A).levels for _, A in handles]
    B = rt.rt_batch_create(ctx.handle, [A for _, A in handles])
    try:
        say(f"[full ensemble V-cycle] levels {min(levels)}..{max(levels)}")
        assert max(levels) >= 3
        offs = _offsets(probs)
        e = torch.tensor(np.concatenate([pr.e[:pr.n_interior] for pr in probs]), device=ctx.device)
        E = torch.tensor(np.concatenate([pr.E[:pr.n_interior] for pr in probs]), device=ctx.device)
        tol = 1e-12
        nopts = rt.newton_opts(rt.solve_opts(rt.RT_PREC_MIXED, 1, tol, 5000, 1e-4, 50))
        s, st = rt.rt_batch_newton_step(ctx.handle, B, len(probs), e.data_ptr(), E.data_ptr(), 0,
                                        nopts, 0)
        assert s == rt.RT_OK, rt.rt_last_error()
        assert all(st[q].solve.rel_residual <= tol for q in range(len(probs)))
        eh, Eh = e.cpu().numpy(), E.cpu().numpy()
        smallest = sorted(range(len(probs)), key=lambda q: probs[q].n_interior)[:3]
        for q in smallest:
            ref = ostep.time_step(probs[q].copy(), fixed_outer=1, inner_tol_e=1e-14,
                                  solve_tol=1e-15)
            err_e = np.max(np.abs(eh[offs[q]:offs[q + 1]] - ref.e) / np.abs(ref.e))
            err_E = np.max(np.abs(Eh[offs[q]:offs[q + 1]] - ref.E) / np.abs(ref.E))
            say(f"[full ensemble V-cycle] problem {q} ({probs[q].n_interior} particles, "
                f"{levels[q]} levels): e {err_e:.1e} E {err_E:.1e}")
            assert err_e <= 1e-10 and err_E <= 1e-10, (q, err_e, err_E)
    finally:
        rt.rt_batch_free(B)
        ctx.free(*[h for nb, A in handles for h in (A, nb)])


def test_batch_tune_depth(ctx, ensemble_amg):
    """The batch's own depth tuner times the batched solve at every depth of
    the concatenated hierarchy (1: Jacobi); every depth, the tuned one
    included, solves to the oracle, and depth 1 takes Jacobi's iterations."""
    import torch
    from paper_2001_11606_amd import rt
    probs, systems, _, levels = ensemble_amg
    B = rt.rt_batch_create(ctx.handle, [A for (_, _, A) in systems])
    try:
        offs = _offsets(probs)
        bs, refs = _rhs(probs)
        b = torch.tensor(np.concatenate(bs), device=ctx.device)
        x0 = torch.zeros_like(b)
        opts = rt.solve_opts(0, 1, 1e-14, 4000, 1e-4, 60)
        rep = rt.rt_batch_tune_depth(ctx.handle, B, b.data_ptr(), x0.data_ptr(), opts, 4, 1)
        its = [rep.iterations[d] for d in range(rep.depths)]
        say(f"[batch depth tuner] depths {rep.depths}: ms "
            f"{[round(1e3 * rep.seconds[d], 2) for d in range(rep.depths)]}, iterations {its}, "
            f"chosen {rep.chosen}")
        assert rep.depths == max(levels) and 1 <= rep.chosen <= rep.depths
        assert all(rep.status[d] == rt.RT_OK for d in range(rep.depths))
        assert its[-1] < its[0]
        assert not np.any(x0.cpu().numpy())   # x0 is not changed
        x = torch.zeros_like(b)
        s, st = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                                  rt.solve_opts(0, 0, 1e-14, 4000, 1e-4, 60), 0)
        jac = [st[q].iterations for q in range(len(probs))]
        for d in list(range(1, rep.depths + 1)) + [0]:
            rt.rt_batch_set_cycle_depth(B, d)
            x = torch.zeros_like(b)
            s, st = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                                      opts, 0)
            assert s == rt.RT_OK, rt.rt_last_error()
            xh = x.cpu().numpy()
            for q in range(len(probs)):
                err = np.max(np.abs(xh[offs[q]:offs[q + 1]] - refs[q])) / np.max(np.abs(refs[q]))
                assert err <= 1e-12, (d, q, err)
            if d == 1:
                assert [st[q].iterations for q in range(len(probs))] == jac
    finally:
        rt.rt_batch_free(B)


@pytest.mark.parametrize("sizes", [(700.0,), (700.0, 16.0)])
def test_batch_amg_single_and_tiny(ctx, sizes):
    """A batch of one diffusive problem, and one that adds a 16-particle
    problem (a single level): the batched V-cycle solves each to the oracle."""
    import torch
    from paper_2001_11606_amd import rt
    probs = []
    for q, size in enumerate(sizes):
        pr = synth.config5_member(2 * q, size)   # even members are 2-D
        pr.dt = 0.1
        probs.append(pr)
    systems = [gpu_system(ctx, pr, amg=rt.amg_opts(max_levels=8, coarse_size=16)) for pr in probs]
    levels = [ctx.matrix_info(A).levels for (_, _, A) in systems]
    say(f"[batch amg edge] sizes {[pr.n_interior for pr in probs]} levels {levels}")
    B = rt.rt_batch_create(ctx.handle, [A for (_, _, A) in systems])
    try:
        offs = _offsets(probs)
        bs, refs = _rhs(probs)
        b = torch.tensor(np.concatenate(bs), device=ctx.device)
        for precision, tol, bar in ((0, 1e-14, 1e-12), (1, 1e-12, 1e-10)):
            for graph in (0, 3):
                x = torch.zeros_like(b)
                s, st = rt.rt_batch_solve(ctx.handle, B, len(probs), b.data_ptr(), x.data_ptr(),
                                          rt.solve_opts(precision, 1, tol, 4000, 1e-4, 60), graph)
                assert s == rt.RT_OK, rt.rt_last_error()
                xh = x.cpu().numpy()
                for q in range(len(probs)):
                    err = np.max(np.abs(xh[offs[q]:offs[q + 1]] - refs[q])) / np.max(np.abs(refs[q]))
                    assert err <= bar, (precision, graph, q, err)
    finally:
        rt.rt_batch_free(B)
        ctx.free(*[h for (_, nb, A) in systems for h in (A, nb)])
