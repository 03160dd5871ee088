"""Drive the CPU (AddressSanitizer) build of the library through the C ABI on
small seeded cases and compare with the oracle.  Run in a fresh process with
libasan preloaded (see tests/test_kernels_cpu_emulation.py).  Prints one
line per case; exits non-zero on the first mismatch, and ASan aborts the
process on any out-of-bounds access."""
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import synth  # noqa: E402
from oracle import linsolve, neighbors, operator, step as ostep  # noqa: E402
from gpu_common import (_cold_patch, _diffusive, _limited, _wendland, oracle_system,  # noqa: E402
                        rowwise_rel_err)
from paper_2001_11606_amd import rt  # noqa: E402

FIELDS = ("m", "rho", "cv", "sigma0_a", "sigma_s", "e", "E", "Q_e", "Q_E")
QUICK = os.environ.get("RT_CPU_QUICK") == "1"


def p(a):
    return a.ctypes.data


def say(*a):
    print(*a, flush=True)


class Case:
    def __init__(self, ctx, prob, amg=None):
        self.prob = prob
        self.pos = np.ascontiguousarray(prob.pos)
        self.h = np.ascontiguousarray(prob.h)
        self.arr = {k: np.ascontiguousarray(getattr(prob, k)).copy() for k in FIELDS}
        self.ctx = ctx
        self.nb = rt.rt_build_neighbors_periodic(ctx, prob.dim, prob.n_total, prob.n_interior,
                                                 p(self.pos), p(self.h), prob.kernel,
                                                 None if prob.period is None else list(prob.period))
        self.info = rt.rt_neighbors_get_info(self.nb)
        self.A = self.assemble(amg)

    def inputs(self):
        a = self.arr
        pr = self.prob
        return rt.rt_step_inputs(pr.dt, pr.c, pr.a, pr.opacity_exponent, pr.limiter, pr.limiter_k,
                                 *[p(a[k]) for k in FIELDS])

    def assemble(self, amg, A=0):
        return rt.rt_assemble(self.ctx, self.nb, self.inputs(), amg, A)

    def neighbors(self):
        ptr = np.zeros(self.info.n_total + 1, np.int64)
        idx = np.zeros(max(self.info.npairs, 1), np.int32)
        rt.rt_neighbors_export(self.ctx, self.nb, p(ptr), p(idx))
        return ptr, idx[:self.info.npairs]

    def matrix(self):
        info = rt.rt_matrix_get_info(self.A)
        rp = np.zeros(info.n + 1, np.int64)
        col = np.zeros(max(info.nnz, 1), np.int32)
        val = np.zeros(max(info.nnz, 1))
        g = np.zeros(max(info.n, 1))
        rt.rt_matrix_export(self.ctx, self.A, p(rp), p(col), p(val), p(g))
        return rp, col[:info.nnz], val[:info.nnz], g[:info.n], info

    def free(self):
        rt.rt_matrix_free(self.A)
        rt.rt_neighbors_free(self.nb)


def check_case(ctx, name, prob):
    ptr, idx, fz, sysm = oracle_system(prob)
    # a small coarsest size gives hierarchies of several levels even on tiny cases
    c = Case(ctx, prob, amg=rt.amg_opts(max_levels=8, coarse_size=8))
    gptr, gidx = c.neighbors()
    assert np.array_equal(gptr, ptr) and np.array_equal(gidx, idx), f"{name}: neighbours"
    rp, col, val, g, info = c.matrix()
    assert np.array_equal(rp, sysm.A.indptr) and np.array_equal(col, sysm.A.indices), f"{name}: CSR"
    err = rowwise_rel_err(rp, val, sysm.A.data)
    assert err <= 1e-13, f"{name}: values {err}"
    nin = prob.n_interior
    b = np.random.default_rng(3).standard_normal(nin) * sysm.A.diagonal()
    xref = linsolve.dense(sysm.A, b) if nin <= 3000 else linsolve.pcg_jacobi(sysm.A, b, tol=1e-15)[0]
    combos = ((0, 0, 1e-14, 1e-12), (0, 1, 1e-14, 1e-12), (1, 0, 1e-12, 1e-10), (1, 1, 1e-12, 1e-10))
    if QUICK:
        combos = ((0, 1, 1e-14, 1e-12), (1, 1, 1e-12, 1e-10))
    for prec, precond, tol, bar in combos:
        x = np.zeros(nin)
        s, st = rt.rt_solve(ctx, c.A, p(b), p(x), rt.solve_opts(prec, precond, tol, 3000, 1e-4, 50))
        e = np.max(np.abs(x - xref)) / np.max(np.abs(xref))
        assert s == 0 and e <= bar, f"{name}: solve prec={prec} precond={precond} err={e} its={st.iterations}"
    # the componentwise stopping test: a positive right-hand side over eight
    # decades, every unknown to the bar (relative), Jacobi FP64 and AMG mixed
    bpos = sysm.A.diagonal() * 10.0 ** np.random.default_rng(23).uniform(-8.0, 0.0, nin)
    xpos = linsolve.solve(sysm.A, bpos, tol=1e-15)
    for prec, precond, tol, bar in ((0, 0, 1e-14, 1e-12), (1, 1, 1e-12, 1e-10)):
        x = np.zeros(nin)
        s, st = rt.rt_solve(ctx, c.A, p(bpos), p(x),
                            rt.solve_opts(prec, precond, tol, 3000, 1e-4, 60, tol))
        e = np.max(np.abs(x - xpos) / xpos)
        assert s == 0 and e <= bar and st.cw_residual <= tol, \
            f"{name}: componentwise prec={prec} err={e} cw={st.cw_residual}"
    # the V-cycle with the Chebyshev smoother (degrees 2 and 3), FP64 and mixed
    cc = Case(ctx, prob, amg=rt.amg_opts(max_levels=8, coarse_size=8,
                                         smoother=rt.RT_SMOOTHER_CHEBYSHEV, smoother_degree=3))
    for prec, tol, bar in ((0, 1e-14, 1e-12), (1, 1e-12, 1e-10)):
        x = np.zeros(nin)
        s, st = rt.rt_solve(ctx, cc.A, p(b), p(x), rt.solve_opts(prec, 1, tol, 3000, 1e-4, 50))
        e = np.max(np.abs(x - xref)) / np.max(np.abs(xref))
        assert s == 0 and e <= bar, f"{name}: chebyshev prec={prec} err={e} its={st.iterations}"
    cc.free()
    # the W-cycle (two coarse corrections per level) with smoothed
    # aggregation, FP64 and mixed
    cw_ = Case(ctx, prob, amg=rt.amg_opts(max_levels=8, coarse_size=8, cycle=2,
                                          prolongation=rt.RT_PROLONG_SMOOTHED))
    winfo = rt.rt_matrix_get_info(cw_.A)
    assert winfo.levels == 1 or winfo.level_p_nnz[0] > 0, f"{name}: smoothed prolongation not built"
    for prec, tol, bar in ((0, 1e-14, 1e-12), (1, 1e-12, 1e-10)):
        x = np.zeros(nin)
        s, st = rt.rt_solve(ctx, cw_.A, p(b), p(x), rt.solve_opts(prec, 1, tol, 3000, 1e-4, 50))
        e = np.max(np.abs(x - xref)) / np.max(np.abs(xref))
        assert s == 0 and e <= bar, f"{name}: w-cycle sa prec={prec} err={e} its={st.iterations}"
    cw_.free()
    # the K-cycle (coarse corrections weighted by inner products), FP64 and
    # mixed, with the Chebyshev smoother
    kc_ = Case(ctx, prob, amg=rt.amg_opts(max_levels=8, coarse_size=8, cycle=rt.RT_CYCLE_K,
                                          smoother=rt.RT_SMOOTHER_CHEBYSHEV))
    for prec, tol, bar in ((0, 1e-14, 1e-12), (1, 1e-12, 1e-10)):
        x = np.zeros(nin)
        s, st = rt.rt_solve(ctx, kc_.A, p(b), p(x), rt.solve_opts(prec, 1, tol, 3000, 1e-4, 50))
        e = np.max(np.abs(x - xref)) / np.max(np.abs(xref))
        assert s == 0 and e <= bar, f"{name}: k-cycle prec={prec} err={e} its={st.iterations}"
    kc_.free()
    # the V-cycle on the first two levels only (the second smoothed, not
    # solved), then the depth tuner
    if info.levels >= 3:
        rt.rt_matrix_set_cycle_depth(c.A, 2)
        x = np.zeros(nin)
        s, st = rt.rt_solve(ctx, c.A, p(b), p(x), rt.solve_opts(0, 1, 1e-14, 3000, 1e-4, 50))
        e = np.max(np.abs(x - xref)) / np.max(np.abs(xref))
        assert s == 0 and e <= 1e-12, f"{name}: depth 2 err={e}"
        x0 = np.zeros(nin)
        rep = rt.rt_matrix_tune_depth(ctx, c.A, p(b), p(x0), rt.solve_opts(0, 1, 1e-14, 3000), 1)
        assert rep.depths == info.levels and 1 <= rep.chosen <= info.levels, f"{name}: depth tuner"
        rt.rt_matrix_set_cycle_depth(c.A, 0)
    # GMRES on the unscaled operator, Jacobi and AMG, with and without restarts
    for precond, restart in (((1, 4),) if QUICK else ((0, 30), (1, 30), (1, 4))):
        x = np.zeros(nin)
        s, st = rt.rt_solve_gmres(ctx, c.A, p(b), p(x), rt.gmres_opts(precond, 1e-13, 3000, restart))
        e = np.max(np.abs(x - xref)) / np.max(np.abs(xref))
        assert s == 0 and e <= 1e-10 and st.rel_residual <= 1e-13, \
            f"{name}: gmres precond={precond} restart={restart} err={e} its={st.iterations}"
    # every SpMV shape (forced on all levels), then the autotuner's choice
    nshapes = len(rt.rt_spmv_shapes())
    sweep = range(nshapes) if name in ("marshak3d_8", "mms2d_16") else (0, 7, nshapes - 1)
    # (the widest shapes are slow to emulate: every shuffle is a thread barrier here)
    for shape in (sweep if not QUICK else (0, 7)):
        for lvl in range(info.levels):
            for prec in (0, 1, 2):
                rt.rt_matrix_set_spmv_shape(c.A, lvl, prec, shape)
        for prec, tol, bar in ((0, 1e-14, 1e-12), (1, 1e-12, 1e-10)):
            x = np.zeros(nin)
            s, st = rt.rt_solve(ctx, c.A, p(b), p(x), rt.solve_opts(prec, 1, tol, 3000, 1e-4, 50))
            e = np.max(np.abs(x - xref)) / np.max(np.abs(xref))
            assert s == 0 and e <= bar, f"{name}: shape {shape} prec={prec} err={e}"
    if not QUICK:
        rep = rt.rt_matrix_tune(ctx, c.A, 1)
        assert rep.levels == info.levels and rep.shapes == nshapes, f"{name}: tune report"
    x = np.zeros(nin)
    s, st = rt.rt_solve(ctx, c.A, p(b), p(x), rt.solve_opts(1, 1, 1e-12, 3000, 1e-4, 50))
    e = np.max(np.abs(x - xref)) / np.max(np.abs(xref))
    assert s == 0 and e <= 1e-10, f"{name}: tuned solve err={e}"
    # Algorithm 1, three outer iterations, FP64 + AMG
    n_outer = 2 if QUICK else 3   # the second outer iteration carries the residual over
    ref = ostep.time_step(prob.copy(), fixed_outer=n_outer, solve_tol=1e-15)
    e_ = c.arr["e"][:nin].copy()
    E_ = c.arr["E"][:nin].copy()
    nopts = rt.newton_opts(rt.solve_opts(0, 1, 1e-14, 3000))
    for ell in range(n_outer):
        s, st = rt.rt_newton_step(ctx, c.A, p(e_), p(E_), ell, nopts)
        assert s == 0, f"{name}: newton status {s}"
    ee = np.max(np.abs(e_ - ref.e) / ref.e)
    eE = np.max(np.abs(E_ - ref.E) / ref.E)
    assert ee <= 1e-12 and eE <= 1e-12, f"{name}: newton {ee} {eE}"
    # the same steps with the state kept in the library's sorted order
    es = np.zeros(nin)
    Es = np.zeros(nin)
    e_in = c.arr["e"][:nin].copy()
    E_in = c.arr["E"][:nin].copy()
    rt.rt_to_sorted(ctx, c.nb, p(e_in), p(es))
    rt.rt_to_sorted(ctx, c.nb, p(E_in), p(Es))
    nso = rt.newton_opts(rt.solve_opts(0, 1, 1e-14, 3000), state_order=1)
    for ell in range(n_outer):
        s, st = rt.rt_newton_step(ctx, c.A, p(es), p(Es), ell, nso)
        assert s == 0, f"{name}: sorted newton status {s}"
    eu = np.zeros(nin)
    Eu = np.zeros(nin)
    rt.rt_to_user(ctx, c.nb, p(es), p(eu))
    rt.rt_to_user(ctx, c.nb, p(Es), p(Eu))
    assert np.max(np.abs(eu - e_) / e_) <= 1e-13 and np.max(np.abs(Eu - E_) / E_) <= 1e-13, \
        f"{name}: sorted-order state"
    # the backward-Euler residual G at the state reached, against the oracle's
    gres = rt.rt_newton_residual(ctx, c.A, p(e_), p(E_), 0)
    m_o, r_o = ostep.be_residual(prob, fz, ptr, idx, e_, E_)
    b_o = operator.rhs(prob, fz, sysm, e_, E_)
    rad = float(np.linalg.norm(fz.V[:nin] * r_o))
    mat = float(np.max(np.abs(m_o) / (prob.rho[:nin] / prob.dt * np.abs(e_))))
    bn = float(np.linalg.norm(b_o))
    assert abs(gres.rad_norm - rad) <= 1e-12 * bn and abs(gres.rad_rel - rad / bn) <= 1e-12 \
        and abs(gres.mat_rel - mat) <= 1e-12, f"{name}: residual {gres.rad_norm} {rad} {gres.mat_rel} {mat}"
    say(f"ok {name}: n={prob.n_total} pairs={info.nnz} levels={info.levels} "
        f"err(values)={err:.1e} newton=({ee:.1e},{eE:.1e})")
    c.free()


def check_cache(ctx):
    """Freed buffers go to the library's cache (filled with garbage bytes when
    reused in this build); a rebuild from cached blocks must still match the
    oracle, and releasing the cache empties it."""
    prob = synth.config4(n=6)
    ptr, idx, fz, sysm = oracle_system(prob)
    for rep in range(2):
        c = Case(ctx, prob, amg=rt.amg_opts(max_levels=1))
        gptr, gidx = c.neighbors()
        rp, col, val, g, info = c.matrix()
        assert np.array_equal(gptr, ptr) and np.array_equal(gidx, idx), f"cache rebuild {rep}: neighbours"
        assert np.array_equal(rp, sysm.A.indptr) and np.array_equal(col, sysm.A.indices), \
            f"cache rebuild {rep}: CSR"
        assert rowwise_rel_err(rp, val, sysm.A.data) <= 1e-13, f"cache rebuild {rep}: values"
        c.free()
        assert rt.rt_cached_bytes(ctx) > 0
    freed = rt.rt_release_cached(ctx)
    assert freed > 0 and rt.rt_cached_bytes(ctx) == 0
    say(f"ok cache: rebuilt from cached blocks, released {freed} bytes")


def check_batch(ctx):
    """An ensemble through the batched entry points against per-problem oracle results."""
    probs = [synth.config5_member(q, s) for q, s in enumerate((150.0, 300.0, 90.0, 700.0))]
    cases = [Case(ctx, pr, amg=rt.amg_opts(max_levels=1)) for pr in probs]
    B = rt.rt_batch_create(ctx, [c.A for c in cases])
    rows, nnz, tcols = rt.rt_batch_get_info(B)
    offs = np.cumsum([0] + [pr.n_interior for pr in probs])
    rng = np.random.default_rng(11)
    bs, xref = [], []
    for c, pr in zip(cases, probs):
        sysm = oracle_system(pr)[3]
        b = rng.standard_normal(pr.n_interior) * sysm.A.diagonal()
        bs.append(b)
        xref.append(linsolve.dense(sysm.A, b))
    bcat = np.concatenate(bs)
    for prec, tol, bar, graph in ((0, 1e-14, 1e-12, 0), (1, 1e-12, 1e-10, 0), (1, 1e-12, 1e-10, 3),
                                  (0, 1e-14, 1e-12, 2)):
        x = np.zeros(offs[-1])
        s, st = rt.rt_batch_solve(ctx, B, len(probs), p(bcat), p(x),
                                  rt.solve_opts(prec, 0, tol, 3000, 1e-4, 50), graph)
        assert s == 0, f"batch solve status {s}"
        for q in range(len(probs)):
            xq = x[offs[q]:offs[q + 1]]
            err = np.max(np.abs(xq - xref[q])) / np.max(np.abs(xref[q]))
            assert err <= bar, f"batch solve prec={prec} graph={graph} problem {q}: {err}"
    # three outer iterations of Algorithm 1 for every problem
    e = np.concatenate([pr.e[:pr.n_interior] for pr in probs]).copy()
    E = np.concatenate([pr.E[:pr.n_interior] for pr in probs]).copy()
    nopts = rt.newton_opts(rt.solve_opts(0, 0, 1e-14, 3000))
    for ell in range(3):
        s, st = rt.rt_batch_newton_step(ctx, B, len(probs), p(e), p(E), ell, nopts, 2)
        assert s == 0, f"batch newton status {s}"
    for q, pr in enumerate(probs):
        ref = ostep.time_step(pr.copy(), fixed_outer=3, solve_tol=1e-15)
        ee = np.max(np.abs(e[offs[q]:offs[q + 1]] - ref.e) / ref.e)
        eE = np.max(np.abs(E[offs[q]:offs[q + 1]] - ref.E) / ref.E)
        assert ee <= 1e-12 and eE <= 1e-12, f"batch newton problem {q}: {ee} {eE}"
        assert st[q].energy == pytest_approx(ref.energy_after), "batch energy"
    rt.rt_batch_free(B)
    for c in cases:
        c.free()
    say(f"ok batch: {len(probs)} problems, rows={rows} nnz={nnz} tile_cols={tcols}")


def check_batch_amg(ctx):
    """An ensemble of diffusive problems with their own aggregation
    hierarchies: batched V-cycle solves and Newton steps against the oracle."""
    probs = []
    for q, s_ in enumerate((150.0, 300.0, 700.0)):
        pr = synth.config5_member(q, s_)
        pr.dt = 0.1
        probs.append(pr)
    cases = [Case(ctx, pr, amg=rt.amg_opts(max_levels=8, coarse_size=16)) for pr in probs]
    levels = [rt.rt_matrix_get_info(c.A).levels for c in cases]
    assert max(levels) >= 3, f"batch amg: hierarchies {levels}"
    B = rt.rt_batch_create(ctx, [c.A for c in cases])
    offs = np.cumsum([0] + [pr.n_interior for pr in probs])
    rng = np.random.default_rng(13)
    bs, xref = [], []
    for pr in probs:
        sysm = oracle_system(pr)[3]
        b = rng.standard_normal(pr.n_interior) * sysm.A.diagonal()
        bs.append(b)
        xref.append(linsolve.dense(sysm.A, b))
    bcat = np.concatenate(bs)
    its, sols = {}, {}
    for prec, precond, tol, bar, graph in ((0, 1, 1e-14, 1e-12, 0), (1, 1, 1e-12, 1e-10, 0),
                                           (0, 0, 1e-14, 1e-12, 0), (0, 1, 1e-14, 1e-12, 3),
                                           (1, 1, 1e-12, 1e-10, 3)):
        x = np.zeros(offs[-1])
        s, st = rt.rt_batch_solve(ctx, B, len(probs), p(bcat), p(x),
                                  rt.solve_opts(prec, precond, tol, 3000, 1e-4, 50), graph)
        assert s == 0, f"batch amg solve status {s}"
        its[(prec, precond, graph)] = [st[q].iterations for q in range(len(probs))]
        sols[(prec, precond, graph)] = x.copy()
        if graph:   # replayed V-cycle iterations: the same iterates as launched one by one
            assert its[(prec, precond, graph)] == its[(prec, precond, 0)], its
            assert np.array_equal(x, sols[(prec, precond, 0)]), f"graph {graph} prec {prec}"
        for q in range(len(probs)):
            xq = x[offs[q]:offs[q + 1]]
            err = np.max(np.abs(xq - xref[q])) / np.max(np.abs(xref[q]))
            assert err <= bar, f"batch amg solve prec={prec} precond={precond} problem {q}: {err}"
    e = np.concatenate([pr.e[:pr.n_interior] for pr in probs]).copy()
    E = np.concatenate([pr.E[:pr.n_interior] for pr in probs]).copy()
    nopts = rt.newton_opts(rt.solve_opts(0, 1, 1e-14, 3000))
    for ell in range(2):
        s, st = rt.rt_batch_newton_step(ctx, B, len(probs), p(e), p(E), ell, nopts, 2 * ell)
        assert s == 0, f"batch amg newton status {s}"
    for q, pr in enumerate(probs):
        ref = ostep.time_step(pr.copy(), fixed_outer=2, solve_tol=1e-15)
        ee = np.max(np.abs(e[offs[q]:offs[q + 1]] - ref.e) / ref.e)
        eE = np.max(np.abs(E[offs[q]:offs[q + 1]] - ref.E) / ref.E)
        assert ee <= 1e-12 and eE <= 1e-12, f"batch amg newton problem {q}: {ee} {eE}"
    rt.rt_batch_free(B)
    # a problem with b = 0 stops before the first V-cycle: exactly zero
    bz = bcat.copy()
    bz[offs[1]:offs[2]] = 0.0
    x = np.zeros(offs[-1])
    s, st = rt.rt_batch_solve(ctx, B2 := rt.rt_batch_create(ctx, [c.A for c in cases]),
                              len(probs), p(bz), p(x), rt.solve_opts(0, 1, 1e-14, 3000, 1e-4, 50), 2)
    assert s == 0 and st[1].iterations == 0, f"batch amg zero rhs: {s}"
    assert not np.any(x[offs[1]:offs[2]]), "batch amg zero rhs: nonzero solution"
    for q in (0, 2):
        err = np.max(np.abs(x[offs[q]:offs[q + 1]] - xref[q])) / np.max(np.abs(xref[q]))
        assert err <= 1e-12, f"batch amg zero rhs problem {q}: {err}"
    rt.rt_batch_free(B2)
    # the batch's own depth tuner: every depth timed, the chosen one solves
    B3 = rt.rt_batch_create(ctx, [c.A for c in cases])
    x0 = np.zeros(offs[-1])
    rep = rt.rt_batch_tune_depth(ctx, B3, p(bcat), p(x0), rt.solve_opts(0, 1, 1e-14, 3000, 1e-4, 50),
                                 2, 1)
    assert 1 <= rep.chosen <= rep.depths == max(levels), f"batch depth tuner: {rep.chosen}"
    assert not np.any(x0), "batch depth tuner changed x0"
    x = np.zeros(offs[-1])
    s, st = rt.rt_batch_solve(ctx, B3, len(probs), p(bcat), p(x),
                              rt.solve_opts(0, 1, 1e-14, 3000, 1e-4, 50), 0)
    assert s == 0, f"batch tuned depth solve status {s}"
    for q in range(len(probs)):
        err = np.max(np.abs(x[offs[q]:offs[q + 1]] - xref[q])) / np.max(np.abs(xref[q]))
        assert err <= 1e-12, f"batch tuned depth problem {q}: {err}"
    rt.rt_batch_free(B3)
    # each problem with its own V-cycle depth (0: every level)
    for c, d in zip(cases, (1, 0, 2)):
        rt.rt_matrix_set_cycle_depth(c.A, d)
    B = rt.rt_batch_create(ctx, [c.A for c in cases])
    x = np.zeros(offs[-1])
    s, st = rt.rt_batch_solve(ctx, B, len(probs), p(bcat), p(x),
                              rt.solve_opts(0, 1, 1e-14, 3000, 1e-4, 50), 0)
    assert s == 0, f"batch amg depth solve status {s}"
    for q in range(len(probs)):
        err = np.max(np.abs(x[offs[q]:offs[q + 1]] - xref[q])) / np.max(np.abs(xref[q]))
        assert err <= 1e-12, f"batch amg depth problem {q}: {err}"
    rt.rt_batch_free(B)
    for c in cases:
        c.free()
    say(f"ok batch amg: levels {levels}, iterations {its}")


def pytest_approx(v, rel=1e-12):
    class _A:
        def __eq__(self, o):
            return abs(o - v) <= rel * abs(v)
    return _A()


def _levermore(prob):
    prob.limiter = synth.LIMITER_LEVERMORE
    return prob


def main():
    rt.load(os.environ["RT_CPU_LIB"])
    ctx = rt.rt_create(0, 0)
    cases = {
        "mms2d_16": synth.config1(n=16),
        "mms3d_6": synth.config2_mms(n=6),
        "densitystep3d_8": synth.config3(n=8),
        "levermore3d_8": _levermore(synth.config3(n=8)),
        "wendland2d_12": _wendland(2, 12),
        "wendland3d_6": _wendland(3, 6),
        "levermore2d_16": _limited(synth.config1(n=16), synth.LIMITER_LEVERMORE),
        "larsen_wendland2d_12": _limited(_wendland(2, 12), synth.LIMITER_LARSEN),
        "levermore_wendland3d_6": _limited(_wendland(3, 6), synth.LIMITER_LEVERMORE),
        "coldpatch3d_8": _cold_patch(8),
        "diffusive2d_16": _diffusive(synth.config1(n=16), 0.1),
        "diffusive3d_8": _diffusive(synth.config3(n=8), 0.1),
        "periodic2d_16": synth.periodic_wendland(2, 16),
        "marshak3d_8": synth.config4(n=8),
        "ensemble2d": synth.config5_member(0, 400.0),
        "infinite3d_5": synth.config2_infinite(1.0, 0.01, n=5),
    }
    only = os.environ.get("RT_CPU_CASES")
    for name, prob in cases.items():
        if only and name not in only.split(","):
            continue
        check_case(ctx, name, prob)
    if not only or "batch" in only.split(","):
        check_batch(ctx)
    if not only or "batch_amg" in only.split(","):
        check_batch_amg(ctx)
    check_cache(ctx)
    # error contract on the host
    pos = np.random.default_rng(0).uniform(0, 1, (3, 40))
    h = np.full(40, 0.2)
    try:
        rt.rt_build_neighbors(ctx, 4, 40, 40, p(pos), p(h), 0)
        raise AssertionError("dim=4 accepted")
    except rt.RtError as e:
        assert e.code == rt.RT_E_ARG
    # periodic axes: a period under three supports, positions outside [0, L)
    for period, word in (([0.5, 0.0, 0.0], "three"), ([0.0, 0.9, 0.0], "outside")):
        sq = pos.copy()
        sq[0] *= 0.49
        try:
            rt.rt_build_neighbors_periodic(ctx, 3, 40, 40, p(sq), p(h), 0, period)
            raise AssertionError(f"period {period} accepted")
        except rt.RtError as e:
            assert e.code == rt.RT_E_ARG and word in str(e), str(e)
    # empty interior, single particle
    nb = rt.rt_build_neighbors(ctx, 3, 40, 0, p(pos), p(h), 0)
    rt.rt_neighbors_free(nb)
    one = np.array([[0.5], [0.5], [0.5]])
    nb = rt.rt_build_neighbors(ctx, 3, 1, 1, p(one), p(np.array([0.1])), 0)
    rt.rt_neighbors_free(nb)
    if not QUICK or (only and "crowded" in only.split(",")):
        # one crowded cell: more candidates and more rows than one LDS pass holds,
        # and more particles in one cell than the counting sort takes (split sort)
        rng = np.random.default_rng(5)
        crowd = rng.uniform(0.0, 0.1, (3, 1100))
        hc = rng.uniform(0.05, 0.1, 1100)
        nb = rt.rt_build_neighbors(ctx, 3, 1100, 1050, p(crowd), p(hc), 0)
        info = rt.rt_neighbors_get_info(nb)
        gptr = np.zeros(1101, dtype=np.int64)
        gidx = np.zeros(max(info.npairs, 1), dtype=np.int32)
        rt.rt_neighbors_export(ctx, nb, p(gptr), p(gidx))
        rptr, ridx = neighbors.brute_force(crowd, hc, 2.0)
        assert np.array_equal(gptr, rptr) and np.array_equal(gidx[:info.npairs], ridx), "crowded cell"
        rt.rt_neighbors_free(nb)
        say(f"ok crowded cell: pairs={info.npairs}")
    rt.rt_destroy(ctx)
    say("all cases ok")


if __name__ == "__main__":
    main()
