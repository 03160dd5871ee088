"""Multi-step runs with the Sec. 3.3 step control through the C ABI, against
the oracle's run of the same controller: the paper's two infinite-medium
cases (Sec. 4.1: hot material from dt = 1e-20, hot radiation from dt = 1e-7,
both to t = 10), where the oracle takes 780 and 156 steps (the paper prints
779 and 155, tests/golden/infinite_medium_sec4_1.json).  The GPU run must
take the same steps and end in the same state."""
import numpy as np
import pytest

from gpu_common import say
import synth
from oracle import step as ostep, timestep

pytestmark = pytest.mark.gpu


CASES = {"hot_material": (1.0, 1e-16, 1e-20), "hot_radiation": (1e-4, 1.0, 1e-7)}


def _problem(case):
    e0, E0, dt0 = CASES[case]
    prob = synth.config2_infinite(e0, E0, n=2, sigma0=1.0, dt=dt0)
    prob.opacity_exponent = 0.0
    return prob


def _oracle_run(prob, t_end):
    nin = prob.n_interior
    V = prob.m[:nin] / prob.rho[:nin]
    t, dt, ts = 0.0, prob.dt, []
    while t < t_end * (1.0 - 1e-14):
        dt = min(dt, t_end - t)
        prob.dt = dt
        e_old, E_old = prob.e[:nin].copy(), prob.E[:nin].copy()
        r = ostep.time_step(prob, eps_e=1e-12, eps_E=1e-12, inner_tol_e=1e-14, solve_tol=1e-14)
        ostep.advance(prob, r)
        t += dt
        ts.append(t)
        dt = timestep.next_dt(dt, r.e, e_old, r.E, E_old, V, eta_target=0.05, dt_max=0.1,
                              max_growth=10.0)
    return np.array(ts), prob.e[:nin].copy(), prob.E[:nin].copy()


@pytest.mark.parametrize("case", list(CASES))
def test_adaptive_infinite_medium_matches_oracle(case):
    from paper_2001_11606_amd import driver, rt
    e0, E0, dt0 = CASES[case]
    ctx = rt.Context(0)
    try:
        t_end = 10.0
        ts_ref, e_ref, E_ref = _oracle_run(_problem(case), t_end)
        prob = _problem(case)
        dp = driver.upload(prob, ctx.device)
        say(f"[adaptive] {case}: oracle steps {len(ts_ref)}")
        steps, hist = driver.run_adaptive(
            ctx, dp, t_end, dt0, eta_target=0.05, dt_max=0.1, max_growth=10.0,
            amg=rt.amg_opts(max_levels=1), solve=rt.solve_opts(0, 0, 1e-14, 100),
            eps_e=1e-12, eps_E=1e-12, material_tol=1e-14)
        ts = np.array([h[0] for h in hist])
        say(f"[adaptive] GPU steps {steps}")
        assert steps == len(ts_ref)
        assert np.max(np.abs(ts - ts_ref) / ts_ref) <= 1e-9
        e = dp.arrays["e"][:prob.n_interior].cpu().numpy()
        E = dp.arrays["E"][:prob.n_interior].cpu().numpy()
        assert np.max(np.abs(e - e_ref) / e_ref) <= 1e-10
        assert np.max(np.abs(E - E_ref) / E_ref) <= 1e-10
        assert abs(float(e[0] + E[0]) - (e0 + E0)) <= 1e-12   # energy conserved
    finally:
        ctx.close()
