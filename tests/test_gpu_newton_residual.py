"""The residual of the backward-Euler system (Sec. 2.2), G = [m, r], through
the C ABI (rt_newton_residual) against the oracle's direct evaluation
(oracle.step.be_residual: the diffusion term as the pair sum, not the
assembled matrix), at the state two outer iterations reach and at a
perturbed state far from the root; and the starting residual each
rt_newton_step solve reports, which is the same norm for the state the call
starts from.
"""
import numpy as np
import pytest

from gpu_common import gpu_system, oracle_system, say, small_cases
from oracle import operator, step as ostep

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


def _oracle_norms(prob, parts, e, E):
    ptr, idx, fz, sysm = parts
    nin = prob.n_interior
    m, r = ostep.be_residual(prob, fz, ptr, idx, e, E)
    b = operator.rhs(prob, fz, sysm, e, E)
    rad = float(np.linalg.norm(fz.V[:nin] * r))
    mat = float(np.max(np.abs(m) / (prob.rho[:nin] / prob.dt * np.abs(e))))
    return rad, float(np.linalg.norm(b)), mat


@pytest.mark.parametrize("name", ["mms2d_64", "densitystep3d_16", "marshak3d_16", "wendland3d_9",
                                  "diffusive3d_16", "periodic3d_13"])
def test_newton_residual_matches_oracle(ctx, name):
    import torch
    from paper_2001_11606_amd import rt
    prob = CASES[name]()
    parts = oracle_system(prob)
    nin = prob.n_interior
    dp, nb, A = gpu_system(ctx, prob, amg=rt.amg_opts(max_levels=1))
    e = dp.arrays["e"][:nin].clone()
    E = dp.arrays["E"][:nin].clone()
    nopts = rt.newton_opts(rt.solve_opts(0, 0, 1e-14, 4000, 1e-4, 60, 1e-14))
    starts = []
    for ell in range(3):
        e_in, E_in = e.cpu().numpy(), E.cpu().numpy()
        s, st = ctx.newton_step(A, e, E, ell, nopts)
        assert s == rt.RT_OK, rt.rt_last_error()
        starts.append((e_in, E_in, st.solve.init_rel_residual))
    rng = np.random.default_rng(11)
    states = [("after 3 outer iterations", e.cpu().numpy(), E.cpu().numpy()),
              ("perturbed", e.cpu().numpy() * (1 + 1e-3 * rng.standard_normal(nin)),
               E.cpu().numpy() * (1 + 1e-3 * rng.standard_normal(nin)))]
    for label, eh, Eh in states:
        et = torch.tensor(eh, device=ctx.device)
        Et = torch.tensor(Eh, device=ctx.device)
        g = ctx.newton_residual(A, et, Et)
        rad, bn, mat = _oracle_norms(prob, parts, eh, Eh)
        say(f"[G] {name} {label}: |Vr| {g.rad_norm:.6e} (oracle {rad:.6e}), rel {g.rad_rel:.3e}, "
            f"material {g.mat_rel:.3e} (oracle {mat:.3e})")
        assert abs(g.rad_norm - rad) <= 1e-12 * bn, (label, g.rad_norm, rad, bn)
        assert abs(g.rad_rel - rad / bn) <= 1e-12
        assert abs(g.mat_rel - mat) <= 1e-12 * max(1.0, mat), (label, g.mat_rel, mat)
    # the starting residual of the second and third calls is the state's rad_rel
    for ell in (1, 2):
        eh, Eh, init = starts[ell]
        rad, bn, _ = _oracle_norms(prob, parts, eh, Eh)
        assert abs(init - rad / bn) <= 1e-12, (ell, init, rad / bn)
