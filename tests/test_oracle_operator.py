"""Pins for the oracle's Brookshaw operator and assembled system (CPU).

Independent facts checked:

* continuum identities of the second derivative (Sec. 2.3): on an unjittered
  lattice, away from the edges, the operator annihilates constants and linear
  fields exactly (by lattice symmetry) and maps |x|^2 to 2 d k C where the
  lattice-sum factor C tends to 1 as the support grows (C within 1e-4 of 1 at
  h = 2 spacings for the cubic spline) -- a dropped factor 1/2, a sign or a
  wrong kernel derivative fails this;
* second-order consistency: the error of the operator against C*Laplacian of a
  smooth field falls ~4x when the spacing halves;
* the SPH first derivative of a linear field equals C times its slope;
* the assembled V-scaled matrix is bitwise symmetric, an M-matrix, its
  Laplacian part has zero row sums away from ghosts, and it agrees with the
  paper's pair sum evaluated without a matrix;
* flux limiters have the diffusion and free-streaming limits of Sec. 2.1.
"""
import numpy as np
import pytest

import synth
from oracle import kernels, neighbors, operator


def _lattice_problem(dim, n, eta, kernel=kernels.CUBIC_SPLINE, jitter=0.0, seed=0):
    pos, nin = synth.jittered_lattice(dim, n, jitter, 0, np.random.default_rng(seed))
    N = pos.shape[1]
    dx = 1.0 / n
    return synth.Problem(name="lat", dim=dim, pos=pos, h=np.full(N, eta * dx), n_interior=N,
                         m=np.full(N, dx ** dim), rho=np.ones(N), cv=np.ones(N),
                         sigma0_a=np.ones(N), sigma_s=np.zeros(N), opacity_exponent=0.0,
                         e=np.ones(N), E=np.ones(N), Q_e=np.zeros(N), Q_E=np.zeros(N),
                         dt=1e-3, kernel=kernel)


def _center(p, n):
    c = np.argmin(np.sum((p.pos - 0.5) ** 2, axis=0))
    return c


@pytest.mark.parametrize("dim,eta,kernel", [(2, 2.0, kernels.CUBIC_SPLINE),
                                            (3, 2.0, kernels.CUBIC_SPLINE),
                                            (2, 4.0, kernels.WENDLAND_C4),
                                            (3, 4.0, kernels.WENDLAND_C4)])
def test_lattice_identities(dim, eta, kernel):
    n = 16 if dim == 3 else 24
    p = _lattice_problem(dim, n, eta, kernel)
    ptr, idx = neighbors.build(p.pos, p.h, kernels.KAPPA[kernel])
    c = _center(p, n)
    k = np.ones(p.n_total)
    L1 = operator.brookshaw(p, ptr, idx, k, np.ones(p.n_total))
    Lx = operator.brookshaw(p, ptr, idx, k, p.pos[0] * 3.0 - p.pos[-1])
    Lr2 = operator.brookshaw(p, ptr, idx, k, np.sum(p.pos ** 2, axis=0))
    assert L1[c] == 0.0
    scale = abs(Lr2[c])
    assert abs(Lx[c]) < 1e-12 * scale
    # <d(k d|x|^2)> = 2 d k C(eta), here k = 1 (k_i + k_j = 2)
    C = Lr2[c] / (2.0 * dim)
    assert abs(C - 1.0) < 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_second_order_consistency(dim):
    eta = 1.3 if dim == 2 else 1.2
    errs = []
    for n in ((16, 32, 64) if dim == 2 else (8, 16, 32)):
        p = _lattice_problem(dim, n, eta)
        ptr, idx = neighbors.build(p.pos, p.h, 2.0)
        k = np.full(p.n_total, 0.5)       # k_i + k_j = 1
        c = _center(p, n)
        Lr2 = operator.brookshaw(p, ptr, idx, k, np.sum(p.pos ** 2, axis=0))
        C = Lr2[c] / (2.0 * dim)
        g = np.prod(np.sin(np.pi * p.pos + 0.3), axis=0)
        lap = -dim * np.pi ** 2 * g
        Lg = operator.brookshaw(p, ptr, idx, k, g)
        errs.append(abs(Lg[c] - C * lap[c]) / abs(lap[c]))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.0 < r < 5.5 for r in ratios), (errs, ratios)


def test_gradient_of_linear_field():
    dim, eta, n = 3, 1.2, 14
    p = _lattice_problem(dim, n, eta)
    ptr, idx = neighbors.build(p.pos, p.h, 2.0)
    c = _center(p, n)
    slope = np.array([0.7, -1.1, 0.4])
    g = operator.grad_E(p, ptr, idx, slope @ p.pos)
    # with k_i + k_j = 1 the second derivative of |x|^2 is d * C
    Lr2 = operator.brookshaw(p, ptr, idx, np.full(p.n_total, 0.5), np.sum(p.pos ** 2, axis=0))
    C = Lr2[c] / dim
    assert np.allclose(g[:, c], C * slope, rtol=1e-12, atol=1e-12)


def _system(prob):
    ptr, idx = neighbors.build(prob.pos, prob.h, 2.0)
    fz = operator.frozen(prob, ptr, idx)
    return ptr, idx, fz, operator.assemble(prob, ptr, idx, fz)


def test_matrix_structure_config1():
    p = synth.config1(n=24)
    ptr, idx, fz, s = _system(p)
    A = s.A
    assert abs(A - A.T).max() == 0.0
    off = A - __import__("scipy.sparse", fromlist=["diags"]).diags(A.diagonal())
    assert off.max() <= 0.0
    assert np.all(A.diagonal() > 0)
    nin = p.n_interior
    mass = fz.V[:nin] * (1.0 / p.dt + p.c * fz.sigma_a[:nin] * fz.f[:nin])
    lap_rowsum = np.asarray(A.sum(axis=1)).ravel() - mass
    I, J = neighbors.pairs(ptr, idx)
    touches_ghost = np.zeros(nin, bool)
    touches_ghost[I[(I < nin) & (J >= nin)]] = True
    scale = A.diagonal() - mass
    assert np.all(np.abs(lap_rowsum[~touches_ghost]) <= 1e-13 * scale[~touches_ghost])
    assert np.all(lap_rowsum[touches_ghost] > 0)


def test_matrix_matches_pair_sum():
    p = synth.config3(n=10)
    p.E = p.E * (1.0 + 0.1 * np.random.default_rng(1).standard_normal(p.n_total))
    ptr, idx, fz, s = _system(p)
    x = np.random.default_rng(2).uniform(0.5, 1.5, p.n_total)
    nin = p.n_interior
    lhs = s.A @ x[:nin] - s.g
    direct = fz.V[:nin] * operator.apply_unscaled(p, ptr, idx, fz, np.concatenate([x[:nin], p.E[nin:]]))
    assert np.allclose(lhs, direct, rtol=1e-12, atol=1e-12 * np.abs(direct).max())


def test_matrix_with_ghosts_matches_pair_sum():
    p = synth.config1(n=20)
    ptr, idx, fz, s = _system(p)
    nin = p.n_interior
    x = np.random.default_rng(4).uniform(0.5, 1.5, nin)
    lhs = s.A @ x - s.g
    direct = fz.V[:nin] * operator.apply_unscaled(p, ptr, idx, fz, np.concatenate([x, p.E[nin:]]))
    assert np.allclose(lhs, direct, rtol=1e-12, atol=1e-12 * np.abs(direct).max())


# Lattice-sum factor C(eta) = -(1/d) sum_{j != i} V_j W'(r_ij) r_ij of the
# cubic spline on an unjittered lattice at the configurations' own smoothing
# lengths (2-D h = 1.3 spacings, 3-D h = 1.2), evaluated to 30 digits by
# summing the closed-form kernel derivative over the lattice offsets.
LATTICE_C = {(2, 1.3): 1.0105429572533936, (3, 1.2): 0.98168856707997002}


@pytest.mark.parametrize("dim,eta", sorted(LATTICE_C))
def test_lattice_constant_at_config_eta(dim, eta):
    """<d(k d|x|^2)> at an interior lattice point is 2 d k C(eta) exactly (up to
    rounding): pins sigma_d, W' and the 1/2 of the symmetrised gradient at the
    smoothing lengths the workloads use, to 1e-12."""
    n = 12 if dim == 3 else 20
    p = _lattice_problem(dim, n, eta)
    ptr, idx = neighbors.build(p.pos, p.h, 2.0)
    c = _center(p, n)
    Lr2 = operator.brookshaw(p, ptr, idx, np.ones(p.n_total), np.sum(p.pos ** 2, axis=0))
    C = Lr2[c] / (2.0 * dim)
    assert abs(C - LATTICE_C[(dim, eta)]) < 1e-12 * LATTICE_C[(dim, eta)], C


def test_levermore_between_limits():
    """Levermore's lambda = (2 + R)/(6 + 3R + R^2) (Sec. 2.1) at hand-evaluated
    points between its limits, and its large-R form without overflow."""
    lev = lambda R: operator.flux_limiter(np.array([R], float), operator.LIMITER_LEVERMORE, 0.0)[0]
    assert lev(1.0) == pytest.approx(3.0 / 10.0, rel=1e-15)
    assert lev(2.0) == pytest.approx(1.0 / 4.0, rel=1e-15)
    assert lev(3.0) == pytest.approx(5.0 / 24.0, rel=1e-15)
    assert lev(0.5) == pytest.approx(2.5 / 7.75, rel=1e-15)
    assert lev(10.0) == pytest.approx(12.0 / 136.0, rel=1e-15)
    # far beyond where R^2 overflows: lambda R -> 1, lambda(inf) = 0
    assert lev(1e200) * 1e200 == pytest.approx(1.0, rel=1e-12)
    assert lev(np.inf) == 0.0
    # continuous across the switch to the reciprocal form at R = 1
    assert lev(np.nextafter(1.0, 2.0)) == pytest.approx(lev(1.0), rel=1e-15)
    # Larsen k = 2 at R = 4: 1/5
    assert operator.flux_limiter(np.array([4.0]), operator.LIMITER_LARSEN, 2.0)[0] == \
        pytest.approx(0.2, rel=1e-15)


def test_limiter_ratio_degenerate_cases():
    """R = |grad E|/(sigma_t E): zero gradient is the diffusion limit (also at
    E = 0), a gradient at E = 0 the free-streaming limit."""
    R = operator.limiter_ratio(np.array([0.0, 0.0, 2.0, 3.0]), np.array([1.0, 1.0, 1.0, 2.0]),
                               np.array([1.0, 0.0, 0.0, 0.5]))
    assert R[0] == 0.0 and R[1] == 0.0 and np.isinf(R[2]) and R[3] == 3.0
    for kind in (operator.LIMITER_LARSEN, operator.LIMITER_LEVERMORE):
        lam = operator.flux_limiter(R, kind, 2.0)
        assert lam[0] == pytest.approx(1.0 / 3.0) and lam[2] == 0.0 and np.all(np.isfinite(lam))


def test_flux_limiter_limits():
    R = np.array([0.0, 1e-8, 1e6])
    for kind, k in ((operator.LIMITER_LARSEN, 2.0), (operator.LIMITER_LARSEN, 3.0),
                    (operator.LIMITER_LEVERMORE, 0.0)):
        lam = operator.flux_limiter(R, kind, k)
        assert lam[0] == pytest.approx(1.0 / 3.0, rel=1e-14)
        assert lam[1] == pytest.approx(1.0 / 3.0, rel=1e-6)
        assert lam[2] * R[2] == pytest.approx(1.0, rel=1e-5)   # |F| -> c E
    # Larsen k = 2 is 1/sqrt(9 + R^2)
    R = np.linspace(0, 10, 11)
    assert np.allclose(operator.flux_limiter(R, operator.LIMITER_LARSEN, 2.0),
                       1.0 / np.sqrt(9.0 + R * R), rtol=1e-15)


def test_fleck_factor_limits():
    p = _lattice_problem(2, 6, 1.3)
    ptr, idx = neighbors.build(p.pos, p.h, 2.0)
    p.sigma0_a[:] = 0.0
    with np.errstate(divide="ignore"):   # D = c lambda / sigma_t is infinite here, f is not
        assert np.all(operator.frozen(p, ptr, idx).f == 1.0)
    p.sigma0_a[:] = 1e30
    assert np.all(operator.frozen(p, ptr, idx).f < 1e-25)


def test_fleck_factor_is_schur_complement_of_jacobian():
    """Sec. 2.2: with the Jacobian entries J_me = rho/dt + (c/c_v) sigma_a dB/dT and
    J_re = -(c/c_v) sigma_a dB/dT (dB/dT = 4 a T^3), the Schur-complement factor
    J_re J_me^-1 equals f - 1."""
    p = synth.config3(n=6)
    p.dt = 0.37
    ptr, idx = neighbors.build(p.pos, p.h, 2.0)
    fz = operator.frozen(p, ptr, idx)
    dBdT = 4.0 * p.a * fz.T ** 3
    J_me = p.rho / p.dt + p.c / p.cv * fz.sigma_a * dBdT
    J_re = -p.c / p.cv * fz.sigma_a * dBdT
    assert np.allclose(J_re / J_me, fz.f - 1.0, rtol=1e-13, atol=1e-15)


def test_sampled_rows_match_full_assembly():
    """The per-row oracle (used at full sizes) equals the full assembly on a
    problem with ghosts and one with the flux limiter; its neighbour lists
    equal the brute-force ones."""
    import synth
    from oracle import neighbors, operator
    for prob in (synth.config4(n=10), synth.config3(n=10)):
        kappa = 2.0
        ptr, idx = neighbors.brute_force(prob.pos, prob.h, kappa)
        sam = neighbors.Sampled(prob.pos, prob.h, kappa)
        for i in range(0, prob.n_total, 37):
            assert np.array_equal(sam.of(i), idx[ptr[i]:ptr[i + 1]])
        fz = operator.frozen(prob, ptr, idx)
        sysm = operator.assemble(prob, ptr, idx, fz)
        rows = list(range(0, prob.n_interior, 17))
        got = operator.rows_at(prob, rows, sam.of)
        A = sysm.A
        for i in rows:
            diag, cols, vals, g = got[i]
            lo, hi = A.indptr[i], A.indptr[i + 1]
            c_ref, v_ref = A.indices[lo:hi], A.data[lo:hi]
            off = c_ref != i
            scale = np.max(np.abs(v_ref))
            assert np.array_equal(cols, c_ref[off])
            assert np.max(np.abs(vals - v_ref[off]), initial=0.0) <= 1e-14 * scale
            assert abs(diag - v_ref[~off][0]) <= 1e-14 * scale
            assert abs(g - sysm.g[i]) <= 1e-14 * max(abs(sysm.g[i]), scale)
