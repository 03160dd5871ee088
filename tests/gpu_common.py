"""Shared helpers of the GPU parity tests: run a seeded problem through the
C ABI and through the oracle on identical inputs."""
import sys

import numpy as np

import synth
from oracle import kernels, neighbors, operator


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _levermore(prob):
    """The density-step problem with the Levermore limiter of Sec. 2.1 in
    place of Larsen's."""
    prob.limiter = synth.LIMITER_LEVERMORE
    return prob


def _limited(prob, kind, k=2.0):
    """A workload with the flux limiter of Sec. 2.1 switched on (kind: Larsen
    or Levermore), so that the limiter's gradient runs on its row lengths and
    dimension."""
    prob.limiter = kind
    prob.limiter_k = k
    return prob


def _cold_patch(n):
    """The density-step recipe with the Levermore limiter and E = 0 on the
    particles with x < 0.3: inside the patch the gradient vanishes (R = 0,
    the diffusion limit), on its edge it does not while E = 0 (R infinite,
    the free-streaming limit)."""
    prob = _levermore(synth.config3(n=n))
    prob.E = np.where(prob.pos[0] < 0.3, 0.0, prob.E)
    return prob


def _diffusive(prob, dt):
    """A workload with a longer time step, so that diffusion dominates the
    diagonal (the coupling of a row grows with dt) and the strength-based
    aggregation coarsens it; a manufactured problem takes the sources and
    ghost values of its new first step."""
    prob.dt = dt
    prob.set_time(dt)
    return prob


def _wendland(dim, n):
    """The paper's Wendland kernel at h = 4 spacings (synth.wendland_lattice)."""
    return synth.wendland_lattice(dim, n)


def _periodic_x_ghosts_y(n):
    """The 2-D manufactured recipe (fields periodic in x) with the ghost
    layers beyond the y faces kept as Dirichlet boundaries and those beyond
    the x faces removed; x is periodic with period 1."""
    prob = synth.config1(n=n)
    nin = prob.n_interior
    x = prob.pos[0]
    N = prob.n_total
    keep = np.ones(N, bool)
    keep[nin:] = (x[nin:] > 0.0) & (x[nin:] < 1.0)
    for k, v in list(prob.__dict__.items()):
        if isinstance(v, np.ndarray) and v.shape[-1] == N:
            setattr(prob, k, np.ascontiguousarray(v[..., keep]))
    prob.mms = None
    prob.period = np.array([1.0, 0.0])
    return prob


def small_cases():
    """Seeded problems of every workload family, sized so the oracle finishes in
    seconds while still spanning many rows per block and ragged tails."""
    return {
        "mms2d_64": lambda: synth.config1(n=64),
        "mms3d_12": lambda: synth.config2_mms(n=12),
        "densitystep3d_16": lambda: synth.config3(n=16),
        "densitystep3d_16_levermore": lambda: _levermore(synth.config3(n=16)),
        "wendland2d_24": lambda: _wendland(2, 24),
        "wendland3d_9": lambda: _wendland(3, 9),
        "periodic2d_16": lambda: synth.periodic_wendland(2, 16),
        "periodic3d_13": lambda: synth.periodic_wendland(3, 13),
        "periodicx_ghostsy2d_32": lambda: _periodic_x_ghosts_y(32),
        "mms2d_32_levermore": lambda: _limited(synth.config1(n=32), synth.LIMITER_LEVERMORE),
        "wendland2d_24_larsen": lambda: _limited(_wendland(2, 24), synth.LIMITER_LARSEN),
        "wendland3d_9_levermore": lambda: _limited(_wendland(3, 9), synth.LIMITER_LEVERMORE),
        "densitystep3d_12_coldpatch": lambda: _cold_patch(12),
        "diffusive2d_48": lambda: _diffusive(synth.config1(n=48), 0.1),
        "diffusive3d_16": lambda: _diffusive(synth.config3(n=16), 0.1),
        "marshak3d_16": lambda: synth.config4(n=16),
        "infinite3d_10": lambda: synth.config2_infinite(1.0, 0.01, n=10),
        "ensemble2d": lambda: synth.config5_member(0, 2500.0),
        "ensemble3d": lambda: synth.config5_member(1, 5000.0),
    }


def oracle_system(prob):
    ptr, idx = neighbors.build(prob.pos, prob.h, kernels.KAPPA[prob.kernel], prob.period)
    fz = operator.frozen(prob, ptr, idx)
    sysm = operator.assemble(prob, ptr, idx, fz)
    return ptr, idx, fz, sysm


def gpu_system(ctx, prob, amg=None):
    from paper_2001_11606_amd import driver
    dp = driver.upload(prob, ctx.device)
    nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior, prob.kernel, period=dp.period)
    A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                     dp.limiter_k, amg=amg)
    return dp, nb, A


def rowwise_rel_err(rp, val_a, val_b):
    """max over rows of max|a - b| / max|b| within the row."""
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    scale = np.zeros(n)
    np.maximum.at(scale, rows, np.abs(val_b))
    err = np.zeros(n)
    np.maximum.at(err, rows, np.abs(val_a - val_b))
    return float(np.max(err / np.where(scale > 0, scale, 1.0))) if n else 0.0
