"""GPU edge cases and the error contract of the C ABI."""
import numpy as np
import pytest

import synth
from gpu_common import oracle_system, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2001_11606_amd import rt
    c = rt.Context(0)
    yield c
    c.close()


def _t(ctx, x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).to(ctx.device)


def test_invalid_arguments(ctx):
    from paper_2001_11606_amd import rt
    say("[edges] invalid arguments")
    pos = _t(ctx, np.random.default_rng(0).uniform(0, 1, (3, 50)))
    h = _t(ctx, np.full(50, 0.1))
    with pytest.raises(rt.RtError) as ei:
        rt.rt_build_neighbors(ctx.handle, 4, 50, 50, pos.data_ptr(), h.data_ptr(), 0)
    assert ei.value.code == rt.RT_E_ARG
    with pytest.raises(rt.RtError):
        rt.rt_build_neighbors(ctx.handle, 3, 50, 60, pos.data_ptr(), h.data_ptr(), 0)
    bad = pos.clone()
    bad[1, 7] = float("nan")
    with pytest.raises(rt.RtError) as ei:
        ctx.build_neighbors(bad, h, 50)
    assert "non-finite" in str(ei.value)
    hz = h.clone()
    hz[3] = 0.0
    with pytest.raises(rt.RtError):
        ctx.build_neighbors(pos, hz, 50)


def test_periodic_axes_and_their_errors(ctx):
    """One periodic axis beside two open ones, random positions and smoothing
    lengths: lists equal the oracle's brute force with nearest images; a
    period under three supports, positions outside [0, L) and a negative
    period are rejected."""
    from paper_2001_11606_amd import rt
    from oracle import neighbors
    say("[edges] periodic x, open y and z")
    rng = np.random.default_rng(31)
    n = 3000
    pos_np = rng.uniform(0.0, 1.0, (3, n))
    h_np = rng.uniform(0.03, 0.06, n)
    ptr, idx = neighbors.brute_force(pos_np, h_np, 2.0, period=np.array([1.0, 0.0, 0.0]))
    pos, h = _t(ctx, pos_np), _t(ctx, h_np)
    nb = ctx.build_neighbors(pos, h, n, period=[1.0, 0.0, 0.0])
    gptr, gidx = ctx.export_neighbors(nb)
    assert np.array_equal(gptr.cpu().numpy(), ptr)
    assert np.array_equal(gidx.cpu().numpy(), idx)
    wraps = np.abs(pos_np[0, neighbors.pairs(ptr, idx)[0]] - pos_np[0, idx]) > 0.5
    assert wraps.any()   # the case reaches across the periodic boundary
    squeezed = pos.clone()
    squeezed[0] *= 0.29
    with pytest.raises(rt.RtError) as ei:
        ctx.build_neighbors(squeezed, h, n, period=[0.3, 0.0, 0.0])
    assert "three" in str(ei.value)
    with pytest.raises(rt.RtError) as ei:
        ctx.build_neighbors(pos, h, n, period=[0.0, 0.9, 0.0])
    assert "outside" in str(ei.value)
    with pytest.raises(rt.RtError):
        ctx.build_neighbors(pos, h, n, period=[-1.0, 0.0, 0.0])


def test_smoother_options_rejected(ctx):
    from paper_2001_11606_amd import driver, rt
    say("[edges] smoother options")
    prob = synth.config3(n=6)
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior, prob.kernel)
    for smoother, degree in ((2, 2), (rt.RT_SMOOTHER_CHEBYSHEV, 0), (rt.RT_SMOOTHER_CHEBYSHEV, 9)):
        with pytest.raises(rt.RtError) as ei:
            ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                         dp.limiter_k, amg=rt.amg_opts(smoother=smoother, smoother_degree=degree))
        assert ei.value.code == rt.RT_E_ARG and "smoother" in str(ei.value)


def test_mixed_needs_fp32_copy(ctx):
    from paper_2001_11606_amd import driver, rt
    import torch
    say("[edges] mixed solve without FP32 matrix")
    prob = synth.config1(n=12)
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior)
    A = ctx.assemble(nb, dp.arrays, dp.dt, amg=rt.amg_opts(build_fp32=0))
    b = torch.ones(prob.n_interior, dtype=torch.float64, device=ctx.device)
    x = torch.zeros_like(b)
    with pytest.raises(rt.RtError) as ei:
        ctx.solve(A, b, x, rt.solve_opts(rt.RT_PREC_MIXED))
    assert ei.value.code == rt.RT_E_STATE


def test_not_converged_reports_stats(ctx):
    from paper_2001_11606_amd import driver, rt
    import torch
    say("[edges] max_iter = 1")
    prob = synth.config3(n=10)
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior)
    A = ctx.assemble(nb, dp.arrays, dp.dt, limiter=prob.limiter)
    b = torch.ones(prob.n_interior, dtype=torch.float64, device=ctx.device)
    x = torch.zeros_like(b)
    status, st = ctx.solve(A, b, x, rt.solve_opts(0, 0, 1e-15, 1))
    assert status == rt.RT_NOT_CONVERGED
    assert st.iterations == 1 and st.rel_residual > 1e-15


def test_all_ghosts_and_single_particle(ctx):
    from paper_2001_11606_amd import rt
    import torch
    say("[edges] n_interior = 0 and n_total = 1")
    pos = _t(ctx, np.random.default_rng(1).uniform(0, 1, (2, 30)))
    h = _t(ctx, np.full(30, 0.2))
    nb = ctx.build_neighbors(pos, h, 0)
    assert nb.info.n_interior == 0
    ptr, idx = ctx.export_neighbors(nb)
    assert ptr[-1].item() == nb.info.npairs
    one = ctx.build_neighbors(_t(ctx, [[0.5], [0.5], [0.5]]), _t(ctx, [0.1]), 1)
    assert one.info.npairs == 0


def test_coincident_far_and_ragged(ctx):
    """Clustered particles with very different h (ragged rows, empty cells)."""
    from oracle import neighbors
    say("[edges] clustered, variable h")
    rng = np.random.default_rng(9)
    pos = np.concatenate([rng.uniform(0, 0.1, (3, 400)), rng.uniform(0.6, 1.0, (3, 300))], axis=1)
    h = np.concatenate([np.full(400, 0.01), rng.uniform(0.02, 0.09, 300)])
    nb = ctx.build_neighbors(_t(ctx, pos), _t(ctx, h), 650)
    gptr, gidx = ctx.export_neighbors(nb)
    ptr, idx = neighbors.brute_force(pos, h, 2.0)
    assert np.array_equal(gptr.cpu().numpy(), ptr) and np.array_equal(gidx.cpu().numpy(), idx)


def test_reassemble_reuses_matrix(ctx):
    from paper_2001_11606_amd import driver, rt
    import torch
    say("[edges] second step reuses the matrix object")
    prob = synth.config2_mms(n=8)
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior)
    e, E, A, rep = driver.time_step(ctx, dp, nb, fixed_outer=2)
    driver.advance(dp, e, E)
    prob.e[:prob.n_interior] = e.cpu().numpy()
    prob.E[:prob.n_interior] = E.cpu().numpy()
    prob.set_time(2 * prob.dt)
    dp2 = driver.upload(prob, ctx.device)
    A2 = ctx.assemble(nb, dp2.arrays, dp2.dt, opacity_exponent=prob.opacity_exponent, A=A)
    assert A2 == A
    rp, col, val, g = [t.cpu().numpy() for t in ctx.export_matrix(A)]
    ptr, idx, fz, sysm = oracle_system(prob)
    assert np.array_equal(col, sysm.A.indices)
    assert np.max(np.abs(val - sysm.A.data)) <= 1e-13 * np.max(np.abs(sysm.A.data))


def test_rebuild_from_cached_memory(ctx):
    """Freed handles leave their device blocks in the library's cache; a
    rebuild of the same problem takes them and must give the oracle's lists
    and matrix again; releasing the cache empties it."""
    from paper_2001_11606_amd import driver, rt
    say("[edges] rebuild from cached device memory")
    prob = synth.config4(n=12)
    ptr, idx, fz, sysm = oracle_system(prob)
    dp = driver.upload(prob, ctx.device)
    for rep in range(2):
        nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior, prob.kernel)
        A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                         dp.limiter_k, amg=rt.amg_opts(max_levels=1))
        gptr, gidx = [t.cpu().numpy() for t in ctx.export_neighbors(nb)]
        assert np.array_equal(gptr, ptr) and np.array_equal(gidx, idx), rep
        rp, col, val, g = [t.cpu().numpy() for t in ctx.export_matrix(A)]
        assert np.array_equal(rp, sysm.A.indptr) and np.array_equal(col, sysm.A.indices), rep
        assert np.max(np.abs(val - sysm.A.data)) <= 1e-13 * np.max(np.abs(sysm.A.data)), rep
        rt.rt_matrix_free(A)
        rt.rt_neighbors_free(nb.handle)
        ctx._owned = [o for o in ctx._owned if o[1] not in (A, nb.handle)]
        assert rt.rt_cached_bytes(ctx.handle) > 0
    freed = rt.rt_release_cached(ctx.handle)
    assert freed > 0 and rt.rt_cached_bytes(ctx.handle) == 0


def test_concurrent_contexts_on_their_own_streams():
    """Problems built from several host threads, each with its own context on
    its own stream, share the library's cache of device blocks (reuse across
    streams waits for the device): every matrix must equal the one built
    alone, bit for bit, over several rounds of builds and frees."""
    import threading
    import torch
    from paper_2001_11606_amd import driver, rt
    say("[edges] concurrent contexts")
    probs = [synth.config5_member(q, s) for q, s in enumerate((900.0, 3000.0, 400.0, 2000.0,
                                                                1500.0, 700.0))]
    main = rt.Context(0)
    dps = [driver.upload(pr, main.device) for pr in probs]
    torch.cuda.synchronize()
    ref = []
    for dp in dps:
        nb = main.build_neighbors(dp.pos, dp.h, dp.n_interior, dp.kernel)
        A = main.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                          dp.limiter_k, amg=rt.amg_opts(max_levels=1))
        ref.append([t.cpu().numpy() for t in main.export_matrix(A)])
    main.close()
    ctxs = []
    for _ in range(3):
        with torch.cuda.stream(torch.cuda.Stream()):
            ctxs.append(rt.Context(0))
    errors = []

    def work(w):
        try:
            c = ctxs[w]
            for rnd in range(3):
                for q in range(w, len(dps), len(ctxs)):
                    dp = dps[q]
                    nb = c.build_neighbors(dp.pos, dp.h, dp.n_interior, dp.kernel)
                    A = c.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent,
                                   dp.limiter, dp.limiter_k, amg=rt.amg_opts(max_levels=1))
                    got = [t.cpu().numpy() for t in c.export_matrix(A)]
                    if not all(np.array_equal(a, b) for a, b in zip(got, ref[q])):
                        errors.append((w, rnd, q))
                    rt.rt_matrix_free(A)
                    rt.rt_neighbors_free(nb.handle)
                    c._owned.clear()
        except Exception as exc:   # reported below, on the test's thread
            errors.append(repr(exc))

    threads = [threading.Thread(target=work, args=(w,)) for w in range(len(ctxs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for c in ctxs:
        c.close()
    assert not errors, errors
