"""SpMV row-group shapes and the shape autotuner, through the C ABI.

Every shape must give the oracle's solution (FP64 to 1e-12, mixed to 1e-10
relative, AMG-preconditioned so that the coarse levels use the forced shape
too), including shapes whose one pass covers fewer entries than the longest
row (several passes per row).  rt_matrix_tune must time every shape on every
level and keep a valid choice.
"""
import numpy as np
import pytest

from gpu_common import gpu_system, oracle_system, say, small_cases
from oracle import linsolve

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
def built(ctx):
    out = {}
    for name in ("marshak3d_16", "mms2d_64"):
        prob = CASES[name]()
        sysm = oracle_system(prob)[3]
        b = np.random.default_rng(23).standard_normal(prob.n_interior) * sysm.A.diagonal()
        x_ref = linsolve.dense(sysm.A, b)
        out[name] = (prob, b, x_ref, gpu_system(ctx, prob))
    return out


def _solve(ctx, A, b, precision, tol):
    import torch
    from paper_2001_11606_amd import rt
    bt = torch.tensor(b, device=ctx.device)
    xt = torch.zeros(b.shape[0], dtype=torch.float64, device=ctx.device)
    status, st = ctx.solve(A, bt, xt, rt.solve_opts(precision, 1, tol, 2000, 1e-4, 50))
    assert status == rt.RT_OK, rt.rt_last_error()
    return xt.cpu().numpy()


@pytest.mark.parametrize("name", ["marshak3d_16", "mms2d_64"])
@pytest.mark.parametrize("shape", range(18))
def test_every_shape_solves(ctx, built, name, shape):
    from paper_2001_11606_amd import rt
    shapes = rt.rt_spmv_shapes()
    assert len(shapes) == 18
    prob, b, x_ref, (dp, nb, A) = built[name]
    info = ctx.matrix_info(A)
    assert info.level_tile_cols[0] > 0, "the fine level of these cases is tiled"
    say(f"[shape] {name} shape={shapes[shape]} levels={info.levels} "
        f"tiled={[info.level_tile_cols[l] > 0 for l in range(info.levels)]}")
    for lvl in range(info.levels):
        for prec in (rt.RT_PREC_FP64, rt.RT_PREC_MIXED, rt.RT_PRODUCT_RESIDUAL):
            rt.rt_matrix_set_spmv_shape(A, lvl, prec, shape)
    try:
        scale = np.max(np.abs(x_ref))
        x64 = _solve(ctx, A, b, rt.RT_PREC_FP64, 1e-14)
        assert np.max(np.abs(x64 - x_ref)) / scale <= 1e-12
        x32 = _solve(ctx, A, b, rt.RT_PREC_MIXED, 1e-12)
        assert np.max(np.abs(x32 - x_ref)) / scale <= 1e-10
    finally:
        for lvl in range(info.levels):
            for prec in (rt.RT_PREC_FP64, rt.RT_PREC_MIXED, rt.RT_PRODUCT_RESIDUAL):
                rt.rt_matrix_set_spmv_shape(A, lvl, prec, -1)


def test_tune_reports_and_keeps_choice(ctx, built):
    from paper_2001_11606_amd import rt
    prob, b, x_ref, (dp, nb, A) = built["marshak3d_16"]
    info = ctx.matrix_info(A)
    rep = ctx.tune(A, reps=3)
    say(f"[tune] chosen {rep['chosen']}")
    assert len(rep["us"]) == info.levels
    for lvl in range(info.levels):
        tiled = info.level_tile_cols[lvl] > 0
        # FP64 and FP32 products on every level, the FP64 residual on the fine one
        for p in (range(3) if lvl == 0 else range(2)):
            for s, t in enumerate(rep["us"][lvl][p]):
                assert (t > 0) if (tiled or not rep["shapes"][s][2]) else (t == 0)
            c = rep["chosen"][lvl][p]
            assert 0 <= c < len(rep["shapes"])
            assert rep["us"][lvl][p][c] == min(t for t in rep["us"][lvl][p] if t > 0)
        if lvl > 0:
            assert rep["chosen"][lvl][2] == -1
    x = _solve(ctx, A, b, rt.RT_PREC_MIXED, 1e-12)
    assert np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref)) <= 1e-10


def test_shape_arguments_rejected(ctx, built):
    from paper_2001_11606_amd import rt
    A = built["mms2d_64"][3][2]
    for args in ((99, rt.RT_PREC_FP64, 0), (0, 7, 0), (0, rt.RT_PREC_FP64, 18),
                 (0, rt.RT_PREC_FP64, -2), (0, 3, 0)):
        with pytest.raises(rt.RtError):
            rt.rt_matrix_set_spmv_shape(A, *args)
