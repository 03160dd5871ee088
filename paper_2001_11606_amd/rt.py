"""ctypes binding of the C ABI declared in ``include/rt.h``.

Argument marshalling only: every computation runs in ``librt.so`` on the GPU.
Functions keep the C names (``rt_build_neighbors``, ``rt_assemble``,
``rt_solve``, ``rt_newton_step`` ...) and take device pointers as integers;
``Context`` wraps them for torch tensors (PyTorch is used for device memory
and streams only).  Importing this module does not need a GPU; loading the
library does, and fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librt.so")

RT_OK = 0
RT_NOT_CONVERGED = 1
RT_NONPHYSICAL = 2
RT_E_ARG = -1
RT_E_OOM = -2
RT_E_DEVICE = -3
RT_E_STATE = -4

RT_KERNEL_CUBIC_SPLINE = 0
RT_KERNEL_WENDLAND_C4 = 1
RT_LIMITER_NONE = 0
RT_LIMITER_LARSEN = 1
RT_LIMITER_LEVERMORE = 2
RT_PREC_FP64 = 0
RT_PREC_MIXED = 1
PRECOND_JACOBI = 0
PRECOND_AMG = 1

c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_int = ctypes.c_int
c_vp = ctypes.c_void_p


class rt_neighbors_info(ctypes.Structure):
    _fields_ = [("dim", c_int), ("kernel", c_int), ("n_total", c_i64), ("n_interior", c_i64),
                ("npairs", c_i64), ("ncells", c_i64), ("cell_size", c_dbl)]


class rt_step_inputs(ctypes.Structure):
    _fields_ = [("dt", c_dbl), ("c", c_dbl), ("a", c_dbl), ("opacity_exponent", c_dbl),
                ("limiter", c_int), ("limiter_k", c_dbl),
                ("m", c_vp), ("rho", c_vp), ("cv", c_vp), ("sigma0_a", c_vp), ("sigma_s", c_vp),
                ("e", c_vp), ("E", c_vp), ("Q_e", c_vp), ("Q_E", c_vp)]


class rt_amg_opts(ctypes.Structure):
    _fields_ = [("max_levels", c_int), ("coarse_size", c_int), ("strength", c_dbl),
                ("build_fp32", c_int), ("tiled_spmv", c_int), ("smoother", c_int),
                ("smoother_degree", c_int), ("cycle", c_int), ("prolongation", c_int)]


class rt_matrix_info(ctypes.Structure):
    _fields_ = [("n", c_i64), ("nnz", c_i64), ("levels", c_int),
                ("level_n", c_i64 * 16), ("level_nnz", c_i64 * 16),
                ("level_tile_cols", c_i64 * 16),
                ("level_p_nnz", c_i64 * 16)]


class rt_depth_report(ctypes.Structure):
    _fields_ = [("depths", c_int), ("seconds", c_dbl * 16), ("iterations", c_int * 16),
                ("status", c_int * 16), ("chosen", c_int)]


class rt_solve_opts(ctypes.Structure):
    _fields_ = [("precision", c_int), ("precond", c_int), ("tol", c_dbl), ("max_iter", c_int),
                ("inner_tol", c_dbl), ("max_refine", c_int), ("cw_tol", c_dbl)]


class rt_gmres_opts(ctypes.Structure):
    _fields_ = [("precond", c_int), ("tol", c_dbl), ("max_iter", c_int), ("restart", c_int)]


class rt_solve_stats(ctypes.Structure):
    _fields_ = [("iterations", c_int), ("refinements", c_int), ("rel_residual", c_dbl),
                ("seconds", c_dbl), ("spmv_calls", c_int), ("spmv_seconds", c_dbl),
                ("spmv32_calls", c_int), ("spmv32_seconds", c_dbl), ("cw_residual", c_dbl),
                ("resid_calls", c_int), ("resid_seconds", c_dbl),
                ("init_rel_residual", c_dbl), ("replacements", c_int)]


class rt_newton_opts(ctypes.Structure):
    _fields_ = [("solve", rt_solve_opts), ("material_tol", c_dbl), ("material_max_iter", c_int),
                ("state_order", c_int), ("recompute_residual", c_int)]


class rt_be_residual(ctypes.Structure):
    _fields_ = [("rad_norm", c_dbl), ("rad_rel", c_dbl), ("mat_rel", c_dbl)]


class rt_newton_stats(ctypes.Structure):
    _fields_ = [("delta_e", c_dbl), ("delta_E", c_dbl), ("energy", c_dbl), ("energy_prev", c_dbl),
                ("material_iterations", c_int), ("nonphysical", c_i64), ("solve", rt_solve_stats),
                ("seconds", c_dbl)]


RT_MAX_LEVELS = 16
RT_MAX_SHAPES = 24
RT_PRODUCT_RESIDUAL = 2


class rt_tune_report(ctypes.Structure):
    _fields_ = [("levels", c_int), ("shapes", c_int),
                ("us", ((c_dbl * RT_MAX_SHAPES) * 3) * RT_MAX_LEVELS),
                ("chosen", (c_int * 3) * RT_MAX_LEVELS)]


# name -> (restype, argtypes)
_SIGS = {
    "rt_create": (c_int, [ctypes.POINTER(c_vp), c_int, c_vp]),
    "rt_destroy": (None, [c_vp]),
    "rt_set_stream": (c_int, [c_vp, c_vp]),
    "rt_set_profiling": (c_int, [c_vp, c_int]),
    "rt_cached_bytes": (c_int, [c_vp, ctypes.POINTER(c_i64)]),
    "rt_release_cached": (c_int, [c_vp, ctypes.POINTER(c_i64)]),
    "rt_last_error": (ctypes.c_char_p, []),
    "rt_version": (ctypes.c_char_p, []),
    "rt_build_neighbors": (c_int, [c_vp, c_int, c_i64, c_i64, c_vp, c_vp, c_int,
                                   ctypes.POINTER(c_vp)]),
    "rt_build_neighbors_periodic": (c_int, [c_vp, c_int, c_i64, c_i64, c_vp, c_vp, c_int,
                                            ctypes.POINTER(c_dbl), ctypes.POINTER(c_vp)]),
    "rt_neighbors_get_info": (c_int, [c_vp, ctypes.POINTER(rt_neighbors_info)]),
    "rt_neighbors_export": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "rt_neighbors_order": (c_int, [c_vp, c_vp, c_vp]),
    "rt_neighbors_free": (None, [c_vp]),
    "rt_assemble": (c_int, [c_vp, c_vp, ctypes.POINTER(rt_step_inputs),
                            ctypes.POINTER(rt_amg_opts), ctypes.POINTER(c_vp)]),
    "rt_matrix_get_info": (c_int, [c_vp, ctypes.POINTER(rt_matrix_info)]),
    "rt_matrix_export": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "rt_matrix_free": (None, [c_vp]),
    "rt_spmv_shapes": (c_int, [ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                               ctypes.POINTER(c_int), c_int]),
    "rt_matrix_tune": (c_int, [c_vp, c_vp, c_int, ctypes.POINTER(rt_tune_report)]),
    "rt_matrix_set_spmv_shape": (c_int, [c_vp, c_int, c_int, c_int]),
    "rt_to_sorted": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "rt_to_user": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "rt_fractional_change": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_dbl, c_dbl,
                                     ctypes.POINTER(c_dbl)]),
    "rt_batch_create": (c_int, [c_vp, c_int, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp)]),
    "rt_batch_free": (None, [c_vp]),
    "rt_batch_get_info": (c_int, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                                  ctypes.POINTER(c_i64)]),
    "rt_batch_tune": (c_int, [c_vp, c_vp, c_int, ctypes.POINTER(rt_tune_report)]),
    "rt_batch_set_spmv_shape": (c_int, [c_vp, c_int, c_int]),
    "rt_batch_solve": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(rt_solve_opts), c_int,
                               ctypes.POINTER(rt_solve_stats)]),
    "rt_batch_newton_step": (c_int, [c_vp, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(rt_newton_opts),
                                     c_int, ctypes.POINTER(rt_newton_stats)]),
    "rt_solve": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(rt_solve_opts),
                         ctypes.POINTER(rt_solve_stats)]),
    "rt_solve_noalloc": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(rt_solve_opts),
                                 ctypes.POINTER(rt_solve_stats)]),
    "rt_solve_gmres": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(rt_gmres_opts),
                               ctypes.POINTER(rt_solve_stats)]),
    "rt_newton_step": (c_int, [c_vp, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(rt_newton_opts),
                               ctypes.POINTER(rt_newton_stats)]),
    "rt_newton_residual": (c_int, [c_vp, c_vp, c_vp, c_vp, c_int,
                                   ctypes.POINTER(rt_be_residual)]),
    "rt_matrix_tune_depth": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(rt_solve_opts),
                                     c_int, ctypes.POINTER(rt_depth_report)]),
    "rt_matrix_set_cycle_depth": (c_int, [c_vp, c_int]),
    "rt_batch_tune_depth": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(rt_solve_opts), c_int,
                                    c_int, ctypes.POINTER(rt_depth_report)]),
    "rt_batch_set_cycle_depth": (c_int, [c_vp, c_int]),
}

EXPORTED = tuple(_SIGS)

_lib = None


class RtError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librt.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2001_11606_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(fn: str, status: int) -> int:
    if status < 0:
        raise RtError(fn, status, load().rt_last_error().decode())
    return status


def rt_last_error() -> str:
    return load().rt_last_error().decode()


def rt_version() -> str:
    return load().rt_version().decode()


def rt_create(device: int = 0, stream: int = 0) -> int:
    ctx = c_vp()
    _check("rt_create", load().rt_create(ctypes.byref(ctx), device, stream or None))
    return ctx.value


def rt_destroy(ctx: int) -> None:
    load().rt_destroy(ctx)


def rt_set_stream(ctx: int, stream: int) -> None:
    _check("rt_set_stream", load().rt_set_stream(ctx, stream or None))


def rt_set_profiling(ctx: int, on: bool) -> None:
    _check("rt_set_profiling", load().rt_set_profiling(ctx, int(bool(on))))


def rt_cached_bytes(ctx: int) -> int:
    out = c_i64(0)
    _check("rt_cached_bytes", load().rt_cached_bytes(ctx, ctypes.byref(out)))
    return out.value


def rt_release_cached(ctx: int) -> int:
    out = c_i64(0)
    _check("rt_release_cached", load().rt_release_cached(ctx, ctypes.byref(out)))
    return out.value


def rt_build_neighbors(ctx: int, dim: int, n_total: int, n_interior: int, pos: int, h: int,
                       kernel: int) -> int:
    out = c_vp()
    _check("rt_build_neighbors", load().rt_build_neighbors(ctx, dim, n_total, n_interior, pos, h,
                                                           kernel, ctypes.byref(out)))
    return out.value


def rt_build_neighbors_periodic(ctx: int, dim: int, n_total: int, n_interior: int, pos: int,
                                h: int, kernel: int, period) -> int:
    """period: dim lengths (0 leaves an axis open) or None (no periodic axis)."""
    out = c_vp()
    arr = None
    if period is not None:
        if len(period) != dim:
            raise ValueError(f"period needs {dim} entries, got {len(period)}")
        arr = (c_dbl * dim)(*[float(v) for v in period])
    _check("rt_build_neighbors_periodic",
           load().rt_build_neighbors_periodic(ctx, dim, n_total, n_interior, pos, h, kernel, arr,
                                              ctypes.byref(out)))
    return out.value


def rt_neighbors_get_info(nb: int) -> rt_neighbors_info:
    info = rt_neighbors_info()
    _check("rt_neighbors_get_info", load().rt_neighbors_get_info(nb, ctypes.byref(info)))
    return info


def rt_neighbors_export(ctx: int, nb: int, nbr_ptr: int, nbr_idx: int) -> None:
    _check("rt_neighbors_export", load().rt_neighbors_export(ctx, nb, nbr_ptr, nbr_idx))


def rt_neighbors_order(ctx: int, nb: int, perm: int) -> None:
    _check("rt_neighbors_order", load().rt_neighbors_order(ctx, nb, perm))


def rt_neighbors_free(nb: int) -> None:
    load().rt_neighbors_free(nb)


def rt_assemble(ctx: int, nb: int, inputs: rt_step_inputs, amg: Optional[rt_amg_opts],
                A: int = 0) -> int:
    out = c_vp(A or None)
    _check("rt_assemble", load().rt_assemble(ctx, nb, ctypes.byref(inputs),
                                             ctypes.byref(amg) if amg is not None else None,
                                             ctypes.byref(out)))
    return out.value


def rt_matrix_get_info(A: int) -> rt_matrix_info:
    info = rt_matrix_info()
    _check("rt_matrix_get_info", load().rt_matrix_get_info(A, ctypes.byref(info)))
    return info


def rt_matrix_export(ctx: int, A: int, row_ptr: int, col: int, val: int, ghost_rhs: int) -> None:
    _check("rt_matrix_export", load().rt_matrix_export(ctx, A, row_ptr, col, val, ghost_rhs or None))


def rt_matrix_free(A: int) -> None:
    load().rt_matrix_free(A)


def rt_spmv_shapes() -> list:
    """[(G lanes per row, E entries per lane, tiled)] for every product shape."""
    g = (c_int * RT_MAX_SHAPES)()
    e = (c_int * RT_MAX_SHAPES)()
    t = (c_int * RT_MAX_SHAPES)()
    n = load().rt_spmv_shapes(g, e, t, RT_MAX_SHAPES)
    return [(g[i], e[i], bool(t[i])) for i in range(min(n, RT_MAX_SHAPES))]


def rt_matrix_tune(ctx: int, A: int, reps: int) -> rt_tune_report:
    rep = rt_tune_report()
    _check("rt_matrix_tune", load().rt_matrix_tune(ctx, A, reps, ctypes.byref(rep)))
    return rep


def rt_matrix_set_spmv_shape(A: int, level: int, precision: int, shape: int) -> None:
    _check("rt_matrix_set_spmv_shape", load().rt_matrix_set_spmv_shape(A, level, precision, shape))


def rt_to_sorted(ctx: int, nb: int, user: int, sorted_: int) -> None:
    _check("rt_to_sorted", load().rt_to_sorted(ctx, nb, user, sorted_))


def rt_to_user(ctx: int, nb: int, sorted_: int, user: int) -> None:
    _check("rt_to_user", load().rt_to_user(ctx, nb, sorted_, user))


def rt_fractional_change(ctx: int, A: int, e_new: int, e_old: int, E_new: int, E_old: int,
                         eta_target: float, tiny: float = 1e-15) -> tuple:
    eta = (c_dbl * 2)()
    _check("rt_fractional_change", load().rt_fractional_change(ctx, A, e_new, e_old, E_new, E_old,
                                                               eta_target, tiny, eta))
    return eta[0], eta[1]


def rt_batch_create(ctx: int, mats: list) -> int:
    arr = (c_vp * len(mats))(*mats)
    out = c_vp()
    _check("rt_batch_create", load().rt_batch_create(ctx, len(mats), arr, ctypes.byref(out)))
    return out.value


def rt_batch_free(B: int) -> None:
    load().rt_batch_free(B)


def rt_batch_get_info(B: int) -> tuple:
    rows, nnz, tc = c_i64(), c_i64(), c_i64()
    _check("rt_batch_get_info", load().rt_batch_get_info(B, ctypes.byref(rows), ctypes.byref(nnz),
                                                         ctypes.byref(tc)))
    return rows.value, nnz.value, tc.value


def rt_batch_tune(ctx: int, B: int, reps: int) -> rt_tune_report:
    rep = rt_tune_report()
    _check("rt_batch_tune", load().rt_batch_tune(ctx, B, reps, ctypes.byref(rep)))
    return rep


def rt_batch_set_spmv_shape(B: int, precision: int, shape: int) -> None:
    _check("rt_batch_set_spmv_shape", load().rt_batch_set_spmv_shape(B, precision, shape))


def rt_batch_solve(ctx: int, B: int, nprob: int, b: int, x: int, opts: rt_solve_opts,
                   graph_iters: int = 0) -> tuple:
    st = (rt_solve_stats * nprob)()
    s = _check("rt_batch_solve", load().rt_batch_solve(ctx, B, b, x, ctypes.byref(opts),
                                                       graph_iters, st))
    return s, list(st)


def rt_batch_newton_step(ctx: int, B: int, nprob: int, e: int, E: int, ell: int,
                         opts: rt_newton_opts, graph_iters: int = 0) -> tuple:
    st = (rt_newton_stats * nprob)()
    s = _check("rt_batch_newton_step", load().rt_batch_newton_step(ctx, B, e, E, ell,
                                                                   ctypes.byref(opts),
                                                                   graph_iters, st))
    return s, list(st)


def rt_solve(ctx: int, A: int, b: int, x: int, opts: rt_solve_opts) -> tuple:
    st = rt_solve_stats()
    s = _check("rt_solve", load().rt_solve(ctx, A, b, x, ctypes.byref(opts), ctypes.byref(st)))
    return s, st


def rt_solve_noalloc(ctx: int, A: int, b: int, x: int, opts: rt_solve_opts) -> tuple:
    st = rt_solve_stats()
    s = _check("rt_solve_noalloc", load().rt_solve_noalloc(ctx, A, b, x, ctypes.byref(opts),
                                                           ctypes.byref(st)))
    return s, st


def rt_solve_gmres(ctx: int, A: int, b: int, x: int, opts: rt_gmres_opts) -> tuple:
    st = rt_solve_stats()
    s = _check("rt_solve_gmres", load().rt_solve_gmres(ctx, A, b, x, ctypes.byref(opts),
                                                       ctypes.byref(st)))
    return s, st


def gmres_opts(precond=PRECOND_JACOBI, tol=1e-10, max_iter=1000, restart=30) -> rt_gmres_opts:
    return rt_gmres_opts(precond, tol, max_iter, restart)


def rt_matrix_tune_depth(ctx: int, A: int, b: int, x0: int, opts: rt_solve_opts,
                         reps: int = 3) -> rt_depth_report:
    rep = rt_depth_report()
    _check("rt_matrix_tune_depth", load().rt_matrix_tune_depth(ctx, A, b, x0, ctypes.byref(opts),
                                                               reps, ctypes.byref(rep)))
    return rep


def rt_matrix_set_cycle_depth(A: int, depth: int) -> None:
    _check("rt_matrix_set_cycle_depth", load().rt_matrix_set_cycle_depth(A, depth))


def rt_batch_tune_depth(ctx: int, B: int, b: int, x0: int, opts: rt_solve_opts, graph_iters: int,
                        reps: int) -> rt_depth_report:
    rep = rt_depth_report()
    _check("rt_batch_tune_depth", load().rt_batch_tune_depth(ctx, B, b, x0, ctypes.byref(opts),
                                                             graph_iters, reps, ctypes.byref(rep)))
    return rep


def rt_batch_set_cycle_depth(B: int, depth: int) -> None:
    _check("rt_batch_set_cycle_depth", load().rt_batch_set_cycle_depth(B, depth))


def rt_newton_residual(ctx: int, A: int, e: int, E: int, state_order: int = 0) -> rt_be_residual:
    out = rt_be_residual()
    _check("rt_newton_residual", load().rt_newton_residual(ctx, A, e, E, state_order,
                                                           ctypes.byref(out)))
    return out


def rt_newton_step(ctx: int, A: int, e: int, E: int, ell: int, opts: rt_newton_opts) -> tuple:
    st = rt_newton_stats()
    s = _check("rt_newton_step", load().rt_newton_step(ctx, A, e, E, ell, ctypes.byref(opts),
                                                       ctypes.byref(st)))
    return s, st


# ---------------------------------------------------------------------------
# torch-tensor convenience layer (still marshalling only)
# ---------------------------------------------------------------------------

def _ptr(t, dtype=None) -> int:
    import torch
    if t is None:
        return 0
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


def solve_opts(precision=RT_PREC_FP64, precond=PRECOND_JACOBI, tol=1e-10, max_iter=1000,
               inner_tol=1e-4, max_refine=20, cw_tol=0.0) -> rt_solve_opts:
    return rt_solve_opts(precision, precond, tol, max_iter, inner_tol, max_refine, cw_tol)


RT_SMOOTHER_L1_JACOBI, RT_SMOOTHER_CHEBYSHEV = 0, 1


RT_PROLONG_PIECEWISE, RT_PROLONG_SMOOTHED = 0, 1
RT_CYCLE_V, RT_CYCLE_W, RT_CYCLE_K = 1, 2, 3


def amg_opts(max_levels=8, coarse_size=256, strength=0.25, build_fp32=1,
             tiled_spmv=1, smoother=RT_SMOOTHER_L1_JACOBI, smoother_degree=2,
             cycle=1, prolongation=RT_PROLONG_PIECEWISE) -> rt_amg_opts:
    return rt_amg_opts(max_levels, coarse_size, strength, build_fp32, tiled_spmv, smoother,
                       smoother_degree, cycle, prolongation)


def newton_opts(solve: rt_solve_opts, material_tol=1e-14, material_max_iter=100,
                state_order=0, recompute_residual=0) -> rt_newton_opts:
    return rt_newton_opts(solve, material_tol, material_max_iter, state_order,
                          recompute_residual)


@dataclass
class Neighbors:
    handle: int
    info: rt_neighbors_info


class Context:
    """A library context bound to torch's current stream on ``device``."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.handle = rt_create(device, stream)
        self._owned = []

    def close(self):
        lib = load()
        for kind, h in reversed(self._owned):
            (lib.rt_matrix_free if kind == "A" else lib.rt_neighbors_free)(h)
        self._owned.clear()
        if self.handle:
            rt_destroy(self.handle)
            self.handle = 0

    def free(self, *handles):
        """Release matrices and neighbour lists of this context before close()."""
        lib = load()
        drop = {h.handle if isinstance(h, Neighbors) else h for h in handles}
        for kind, h in [o for o in self._owned if o[1] in drop]:
            (lib.rt_matrix_free if kind == "A" else lib.rt_neighbors_free)(h)
        self._owned = [o for o in self._owned if o[1] not in drop]

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_profiling(self, on: bool):
        rt_set_profiling(self.handle, on)

    def build_neighbors(self, pos, h, n_interior: int, kernel: int = RT_KERNEL_CUBIC_SPLINE,
                        period=None):
        torch = self.torch
        dim, n = pos.shape
        if period is None:
            nb = rt_build_neighbors(self.handle, dim, n, n_interior, _ptr(pos, torch.float64),
                                    _ptr(h, torch.float64), kernel)
        else:
            nb = rt_build_neighbors_periodic(self.handle, dim, n, n_interior,
                                             _ptr(pos, torch.float64), _ptr(h, torch.float64),
                                             kernel, list(period))
        self._owned.append(("N", nb))
        return Neighbors(nb, rt_neighbors_get_info(nb))

    def export_neighbors(self, nb: Neighbors):
        torch = self.torch
        ptr = torch.empty(nb.info.n_total + 1, dtype=torch.int64, device=self.device)
        idx = torch.empty(max(nb.info.npairs, 1), dtype=torch.int32, device=self.device)
        rt_neighbors_export(self.handle, nb.handle, ptr.data_ptr(), idx.data_ptr())
        return ptr, idx[:nb.info.npairs]

    def order(self, nb: Neighbors):
        torch = self.torch
        perm = torch.empty(nb.info.n_total, dtype=torch.int32, device=self.device)
        rt_neighbors_order(self.handle, nb.handle, perm.data_ptr())
        return perm

    def assemble(self, nb: Neighbors, arrays: dict, dt: float, c: float = 1.0, a: float = 1.0,
                 opacity_exponent: float = 0.0, limiter: int = RT_LIMITER_NONE,
                 limiter_k: float = 2.0, amg: Optional[rt_amg_opts] = None, A: int = 0) -> int:
        torch = self.torch
        p = lambda k: _ptr(arrays.get(k), torch.float64) if arrays.get(k) is not None else None
        inp = rt_step_inputs(dt, c, a, opacity_exponent, limiter, limiter_k,
                             p("m"), p("rho"), p("cv"), p("sigma0_a"), p("sigma_s"), p("e"),
                             p("E"), p("Q_e"), p("Q_E"))
        new = rt_assemble(self.handle, nb.handle, inp, amg, A)
        if not A:
            self._owned.append(("A", new))
        return new

    def matrix_info(self, A: int) -> rt_matrix_info:
        return rt_matrix_get_info(A)

    def export_matrix(self, A: int):
        torch = self.torch
        info = rt_matrix_get_info(A)
        rp = torch.empty(info.n + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(info.nnz, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(info.nnz, 1), dtype=torch.float64, device=self.device)
        g = torch.empty(max(info.n, 1), dtype=torch.float64, device=self.device)
        rt_matrix_export(self.handle, A, rp.data_ptr(), col.data_ptr(), val.data_ptr(), g.data_ptr())
        return rp, col[:info.nnz], val[:info.nnz], g[:info.n]

    def tune(self, A: int, reps: int = 5) -> dict:
        """Time every SpMV shape on every level; keeps the fastest per level and
        product.  Returns {"shapes": [(G, E, tiled)], "us": [[fp64 list, fp32
        list, fp64 residual list]], "chosen": [[fp64, fp32, fp64 residual]]}
        (-1 / zero timings: not timed)."""
        rep = rt_matrix_tune(self.handle, A, reps)
        return {"shapes": rt_spmv_shapes()[:rep.shapes],
                "us": [[list(rep.us[l][p][:rep.shapes]) for p in range(3)]
                       for l in range(rep.levels)],
                "chosen": [[rep.chosen[l][p] for p in range(3)] for l in range(rep.levels)]}

    def solve(self, A: int, b, x, opts: rt_solve_opts):
        torch = self.torch
        return rt_solve(self.handle, A, _ptr(b, torch.float64), _ptr(x, torch.float64), opts)

    def solve_gmres(self, A: int, b, x, opts: rt_gmres_opts):
        torch = self.torch
        return rt_solve_gmres(self.handle, A, _ptr(b, torch.float64), _ptr(x, torch.float64),
                              opts)

    def tune_depth(self, A: int, b, x0, opts: rt_solve_opts, reps: int = 3) -> rt_depth_report:
        torch = self.torch
        return rt_matrix_tune_depth(self.handle, A, _ptr(b, torch.float64),
                                    _ptr(x0, torch.float64), opts, reps)

    def newton_residual(self, A: int, e, E, state_order: int = 0) -> rt_be_residual:
        torch = self.torch
        return rt_newton_residual(self.handle, A, _ptr(e, torch.float64), _ptr(E, torch.float64),
                                  state_order)

    def newton_step(self, A: int, e, E, ell: int, opts: rt_newton_opts):
        torch = self.torch
        return rt_newton_step(self.handle, A, _ptr(e, torch.float64), _ptr(E, torch.float64), ell,
                              opts)
