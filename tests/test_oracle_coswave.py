"""Pins for the cos-wave manufactured problem of Sec. 4.3 and the oracle's
run of it (CPU).

* the analytic time derivatives and Laplacian of the manufactured fields
  agree with central finite differences (a dropped factor, sign or the wrong
  phase of the two waves fails this), and the lattice sum of the total source
  vanishes on the periodic box;
* one full cycle at 16^2 points (the paper's 256-point case): the energy of
  the periodic system returns to its start within the radiation-solve
  tolerance (the paper prints a relative change of 6.35e-14 at this size),
  every step needs at most the paper's two outer iterations plus one check,
  and the solution returns to the initial condition;
* second-order convergence in space of the radiation energy (Sec. 4.3);
* first-order convergence in time of both energies (Sec. 4.3).
"""
import numpy as np
import pytest

import synth
from oracle import kernels, neighbors, step


def _run(prob, nsteps, tol_outer=1e-8, tol_inner=1e-12):
    """nsteps backward-Euler steps of Algorithm 1 with the tolerances the
    paper lists for this problem; returns (t, per-step outer counts, energy
    at the start)."""
    ptr, idx = neighbors.build(prob.pos, prob.h, kernels.KAPPA[prob.kernel], prob.period)
    e_start = step.energy(prob, prob.e, prob.E)
    t, outer = 0.0, []
    for _ in range(nsteps):
        t += prob.dt
        prob.set_time(t)
        r = step.time_step(prob, ptr, idx, eps_e=tol_outer, eps_E=tol_outer,
                           inner_tol_e=tol_inner, solve_tol=tol_inner)
        step.advance(prob, r)
        outer.append(r.outer)
    return t, outer, e_start


def _l1(num, exact):
    return float(np.sum(np.abs(num - exact)) / np.sum(exact))


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_fields_match_finite_differences(dim):
    rng = np.random.default_rng(5)
    pos = rng.uniform(0.0, 5.0, (dim, 40))
    args = (1.3, 2.1, 5.0e9, 5.0, 1.0 / 16.0)
    t, dt = 3.0e-10, 1.0e-15
    e, E, de, dE, lap = synth.cos_wave_fields(pos, t, *args)
    ep, Ep, *_ = synth.cos_wave_fields(pos, t + dt, *args)
    em, Em, *_ = synth.cos_wave_fields(pos, t - dt, *args)
    scale_t = 2.0 * np.pi * 5.0e9 / 5.0
    assert np.max(np.abs((ep - em) / (2 * dt) - de)) <= 1e-6 * 1.3 * scale_t
    assert np.max(np.abs((Ep - Em) / (2 * dt) - dE)) <= 1e-6 * 2.1 * scale_t
    hx = 1e-4
    fd = np.zeros(pos.shape[1])
    for a in range(dim):
        off = np.zeros((dim, 1))
        off[a] = hx
        Ea = synth.cos_wave_fields(pos + off, t, *args)[1]
        Eb = synth.cos_wave_fields(pos - off, t, *args)[1]
        fd += (Ea - 2.0 * E + Eb) / hx ** 2
    assert np.max(np.abs(fd - lap)) <= 1e-5 * 2.1 * (2.0 * np.pi / 5.0) ** 2 * dim


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 13)])
def test_total_source_vanishes(dim, n):
    p = synth.cos_wave_mms(dim, n)
    V = p.m / p.rho
    for t in (p.dt, 0.37e-9):
        _, _, Qe, QE = p.mms(t)
        total = np.sum(V * (Qe + QE))
        assert abs(total) <= 1e-13 * np.sum(V * (np.abs(Qe) + np.abs(QE)))


def test_full_cycle_16x16_vs_paper():
    p = synth.cos_wave_mms(2, 16)
    e0, E0 = p.e.copy(), p.E.copy()
    t, outer, start = _run(p, p.meta["steps"])
    assert t == pytest.approx(p.meta["t_end"], rel=1e-12)
    drift = abs(step.energy(p, p.e, p.E) - start) / start
    assert drift <= 1e-12, drift
    assert max(outer) <= 3, np.bincount(outer)
    # one cycle brings the waves back to the initial condition; the error at
    # this coarse spacing (support h = 1.25 cm of a 5 cm wave) is a few percent
    em, Em, _, _ = p.mms(t)
    assert np.allclose(em, e0, rtol=1e-12) and np.allclose(Em, E0, rtol=1e-12)
    assert _l1(p.e, em) < 0.03 and _l1(p.E, Em) < 0.04


def test_radiation_energy_second_order_in_space():
    errs = []
    for n in (16, 32):
        p = synth.cos_wave_mms(2, n)
        t, _, _ = _run(p, 100)
        errs.append(_l1(p.E, p.mms(t)[1]))
    assert 3.0 < errs[0] / errs[1] < 5.5, errs


def test_first_order_in_time():
    """At fixed particles, successive differences of the state at t = 1e-10 s
    (a tenth of the cycle) for dt, dt/2, dt/4, dt/8 halve with the step
    (backward Euler is first order in time, Sec. 4.3); the spatial error
    cancels in the differences."""
    states = []
    for nsteps in (25, 50, 100, 200):
        p = synth.cos_wave_mms(2, 16, steps=10 * nsteps)   # dt = t_end / (10 nsteps)
        t, _, _ = _run(p, nsteps, tol_outer=1e-12, tol_inner=1e-14)
        assert t == pytest.approx(1e-10, rel=1e-12)
        states.append((p.e.copy(), p.E.copy()))
    for k in (0, 1):
        d = [np.max(np.abs(states[i + 1][k] - states[i][k])) for i in range(3)]
        ratios = [d[i] / d[i + 1] for i in range(2)]
        assert all(1.8 < r < 2.2 for r in ratios), (k, d, ratios)
