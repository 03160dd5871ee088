"""Parity at the full benchmark sizes, in the configuration bench.py times
(Jacobi hierarchy, FP32 copies, tuned-shape-independent results).

The oracle cannot build these systems whole, so it checks sampled outputs
one by one -- neighbour lists of sampled particles (k-d tree candidates, then
the pair predicate), matrix rows of sampled particles (the per-row oracle)
and material updates of sampled particles -- and the solver is checked by a
property that holds at any size: the FP64 residual of the returned solution,
recomputed on the host from the exported matrix with scipy.
"""
import numpy as np
import pytest

from gpu_common import say
from oracle import material, neighbors, operator
import synth

pytestmark = pytest.mark.gpu

WORKLOADS = {
    "marshak3d_256": lambda: synth.config4(n=256),
    "densitystep3d_128": lambda: synth.config3(n=128),
}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_11606_amd import rt
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module", params=list(WORKLOADS))
def full(request, ctx):
    from paper_2001_11606_amd import driver, rt
    name = request.param
    say(f"[fullsize] generating {name}")
    prob = WORKLOADS[name]()
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior, prob.kernel)
    A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                     dp.limiter_k, amg=rt.amg_opts(max_levels=1))
    say(f"[fullsize] {name}: {prob.n_total} particles, {nb.info.npairs} pairs; k-d tree")
    sam = neighbors.Sampled(prob.pos, prob.h, 2.0)
    rng = np.random.default_rng(20011606)
    nin = prob.n_interior
    rows = sorted(set([0, nin - 1] + rng.integers(0, nin, 40).tolist()))
    ghosts = rng.integers(nin, prob.n_total, 6).tolist() if prob.n_total > nin else []
    yield name, prob, dp, nb, A, sam, rows, ghosts
    rt.rt_matrix_free(A)
    rt.rt_neighbors_free(nb.handle)
    ctx._owned = [o for o in ctx._owned if o[1] not in (A, nb.handle)]


def test_fullsize_neighbors_sampled(ctx, full):
    name, prob, dp, nb, A, sam, rows, ghosts = full
    say(f"[fullsize neighbors] {name}")
    ptr, idx = ctx.export_neighbors(nb)
    assert nb.info.npairs % 2 == 0   # the predicate is symmetric
    for i in rows + ghosts:
        lo, hi = int(ptr[i]), int(ptr[i + 1])
        got = idx[lo:hi].cpu().numpy()
        ref = sam.of(i)
        assert np.array_equal(got, ref), (name, i, got.size, ref.size)
    # two lists pinned by brute force (every particle tested)
    for i in rows[:2]:
        assert np.array_equal(sam.of(i), neighbors.neighbors_of(prob.pos, prob.h, i, 2.0))


def test_fullsize_matrix_rows_sampled(ctx, full):
    name, prob, dp, nb, A, sam, rows, ghosts = full
    say(f"[fullsize rows] {name}")
    rp, col, val, g = ctx.export_matrix(A)
    pick = rows[:12] if prob.limiter else rows
    ref = operator.rows_at(prob, pick, sam.of)
    gh = g.cpu().numpy()
    for i in pick:
        lo, hi = int(rp[i]), int(rp[i + 1])
        c = col[lo:hi].cpu().numpy()
        v = val[lo:hi].cpu().numpy()
        diag, cols, vals, gi = ref[i]
        off = c != i
        scale = max(np.max(np.abs(v)), abs(diag))
        assert np.array_equal(c[off], cols), (name, i)
        assert np.max(np.abs(v[off] - vals), initial=0.0) <= 1e-13 * scale, (name, i)
        assert abs(v[~off][0] - diag) <= 1e-13 * scale, (name, i)
        assert abs(gh[i] - gi) <= 1e-13 * max(scale, abs(gi)), (name, i)


@pytest.mark.parametrize("precision,tol", [(1, 1e-10), (0, 1e-10)])
def test_fullsize_solve_residual(ctx, full, precision, tol):
    import scipy.sparse as sp
    import torch
    from paper_2001_11606_amd import rt
    name, prob, dp, nb, A, sam, rows, ghosts = full
    say(f"[fullsize solve] {name} precision={precision}")
    nin = prob.n_interior
    rp, col, val, g = ctx.export_matrix(A)
    M = sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=(nin, nin))
    rng = np.random.default_rng(7)
    b = rng.standard_normal(nin) * M.diagonal()
    bt = torch.tensor(b, device=ctx.device)
    xt = torch.zeros(nin, dtype=torch.float64, device=ctx.device)
    s, st = ctx.solve(A, bt, xt, rt.solve_opts(precision, 0, tol, 5000, 1e-4, 30))
    assert s == rt.RT_OK, rt.rt_last_error()
    x = xt.cpu().numpy()
    rel = np.linalg.norm(b - M @ x) / np.linalg.norm(b)
    say(f"[fullsize solve] {name} precision={precision}: its={st.iterations} "
        f"refinements={st.refinements} residual={rel:.3e} (reported {st.rel_residual:.3e})")
    assert rel <= 1.05 * tol


_REF = {}


def _step(ctx, dp, nb, solve, outer):
    from paper_2001_11606_amd import driver, rt
    e, E, A, rep = driver.time_step(ctx, dp, nb, amg=rt.amg_opts(max_levels=1), solve=solve,
                                    fixed_outer=outer)
    rt.rt_matrix_free(A)
    ctx._owned = [o for o in ctx._owned if o[1] != A]
    return e, E, rep


@pytest.mark.parametrize("precision", [1, 0])
def test_fullsize_bench_accuracy(ctx, full, precision):
    """The step bench.py times (its outer iterations, preconditioner and both
    stopping tolerances, in either precision) against the same step solved to
    1e-14 in both measures in FP64: every particle's e and E within 1e-10
    relative."""
    import bench
    from paper_2001_11606_amd import rt
    name, prob, dp, nb, A, sam, rows, ghosts = full
    if name not in _REF:
        say(f"[fullsize accuracy] {name}: FP64 reference step to 1e-14")
        e, E, rep = _step(ctx, dp, nb, rt.solve_opts(0, 0, 1e-14, 20000, 1e-4, 60, 1e-14),
                          bench.BENCH_OUTER)
        assert rep.status == rt.RT_OK
        _REF[name] = (e, E)
    eR, ER = _REF[name]
    say(f"[fullsize accuracy] {name} precision={precision} at the bench's options")
    e, E, rep = _step(ctx, dp, nb, bench.bench_solve_opts(precision), bench.BENCH_OUTER)
    assert rep.status == rt.RT_OK
    dE = float(((E - ER).abs() / ER.abs()).max())
    de = float(((e - eR).abs() / eR.abs()).max())
    say(f"  krylov {rep.krylov} refinements {rep.refinements}: max rel diff E {dE:.2e} e {de:.2e}")
    assert dE <= 1e-10 and de <= 1e-10, (dE, de)


def test_fullsize_material_sampled(ctx, full):
    """After one outer iteration the material energies of sampled particles are
    the roots of their own material equations for the returned E."""
    from paper_2001_11606_amd import rt
    name, prob, dp, nb, A, sam, rows, ghosts = full
    say(f"[fullsize material] {name}")
    nin = prob.n_interior
    e = dp.arrays["e"][:nin].clone()
    E = dp.arrays["E"][:nin].clone()
    s, st = ctx.newton_step(A, e, E, 0,
                            rt.newton_opts(rt.solve_opts(1, 0, 1e-10, 5000, 1e-4, 30), 1e-14))
    assert s == rt.RT_OK, rt.rt_last_error()
    idx = np.array(rows)
    eh = e.cpu().numpy()[idx]
    Eh = E.cpu().numpy()[idx]
    fz = operator.frozen_at(prob, idx, sam.of)
    sa = np.array([fz[int(i)][0] for i in idx])
    P = prob.Q_e[idx] + prob.c * sa * Eh
    ref, its, nonphys = material.solve(prob.e[idx], P, prob.rho[idx], prob.cv[idx], sa, prob.dt,
                                       prob.c, prob.a, eh, tol=1e-14)
    assert not nonphys.any()
    assert np.max(np.abs(eh - ref) / np.abs(ref)) <= 1e-12
