"""Seeded synthetic particle problems for the implicit SPH radiation-diffusion path.

This module only *places particles and fills in per-particle data*: positions,
smoothing lengths, masses, densities, opacity coefficients, initial energies,
boundary (ghost) values and manufactured sources.  It contains none of the
method's arithmetic (no SPH kernel, no neighbour predicate, no operator, no
solver, no material update).  Both the CPU oracle and the GPU path read the
arrays produced here, so they always see bit-identical inputs.

Conventions shared by every problem:

* positions are SoA, ``pos[alpha, i]`` (float64, shape ``(dim, n_total)``);
* interior particles come first, ``[0, n_interior)``; constant-value (Dirichlet)
  ghost particles follow, ``[n_interior, n_total)`` -- the ghost treatment of the
  paper's meshless implementation (Sec. 3.1);
* per-particle arrays have length ``n_total``; ghost entries of ``e``/``E`` hold
  the boundary data of the step, ghost entries of ``Q_e``/``Q_E`` are zero;
* the opacity model is a power law evaluated by the method at the start of the
  step, ``sigma_a = sigma0_a * T**opacity_exponent`` (Sec. 3.2: material data is
  frozen per time step), ``sigma_t = sigma_a + sigma_s``;
* dimensionless units, ``c = a = 1`` unless stated.

Seeds follow ``11606000 + config`` (ensemble member ``p`` uses ``11606500 + p``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

KERNEL_CUBIC_SPLINE = 0
KERNEL_WENDLAND_C4 = 1

LIMITER_NONE = 0
LIMITER_LARSEN = 1
LIMITER_LEVERMORE = 2

SEED_BASE = 11606000
SEED_ENSEMBLE = 11606500


@dataclass
class Problem:
    name: str
    dim: int
    pos: np.ndarray            # (dim, n_total) float64
    h: np.ndarray              # (n_total,)
    n_interior: int
    m: np.ndarray
    rho: np.ndarray
    cv: np.ndarray
    sigma0_a: np.ndarray
    sigma_s: np.ndarray
    opacity_exponent: float
    e: np.ndarray              # e^{n-1} (interior) / boundary data (ghosts)
    E: np.ndarray              # E^{n-1} (interior) / boundary data (ghosts)
    Q_e: np.ndarray
    Q_E: np.ndarray
    dt: float
    c: float = 1.0
    a: float = 1.0
    kernel: int = KERNEL_CUBIC_SPLINE
    limiter: int = LIMITER_NONE
    limiter_k: float = 2.0
    t: float = 0.0
    # Optional manufactured solution: mms(t) -> (e_exact, E_exact, Q_e, Q_E)
    # evaluated at every particle position (sources are zeroed on ghosts).
    mms: Optional[Callable[[float], tuple]] = None
    # Optional periodic box: period[a] > 0 makes axis a periodic with that
    # length (positions in [0, period[a])); 0 leaves it open.
    period: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n_total(self) -> int:
        return int(self.h.shape[0])

    @property
    def n_ghost(self) -> int:
        return self.n_total - self.n_interior

    def set_time(self, t_new: float) -> None:
        """Load the sources and the ghost boundary data of the step ending at ``t_new``."""
        if self.mms is None:
            return
        e_x, E_x, Qe, QE = self.mms(t_new)
        g = slice(self.n_interior, self.n_total)
        self.e[g] = e_x[g]
        self.E[g] = E_x[g]
        self.Q_e[:] = Qe
        self.Q_E[:] = QE
        self.Q_e[g] = 0.0
        self.Q_E[g] = 0.0

    def copy(self) -> "Problem":
        out = Problem(**{k: (v.copy() if isinstance(v, np.ndarray) else v)
                         for k, v in self.__dict__.items() if k != "meta"})
        out.meta = dict(self.meta)
        return out


# ---------------------------------------------------------------------------
# particle placement
# ---------------------------------------------------------------------------

def jittered_lattice(dim: int, n: int, jitter: float, ghost_layers: int,
                     rng: np.random.Generator):
    """Points at ``(i + 1/2) * spacing`` of an ``n**dim`` lattice on the unit
    box, each coordinate jittered by ``U(-jitter, +jitter) * spacing``, plus
    ``ghost_layers`` extra lattice layers outside every face.

    Returns ``(pos, n_interior)`` with interior points first (lattice order,
    x fastest) followed by the ghost layers (same order)."""
    spacing = 1.0 / n
    idx = np.arange(-ghost_layers, n + ghost_layers)
    grids = np.meshgrid(*([idx] * dim), indexing="ij")
    # lattice order with x fastest: reverse axes so that axis 0 (x) varies fastest
    coords = [g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids]
    lat = np.stack(coords)                          # (dim, M) integer sites
    inside = np.all((lat >= 0) & (lat < n), axis=0)
    order = np.concatenate([np.nonzero(inside)[0], np.nonzero(~inside)[0]])
    lat = lat[:, order]
    jit = rng.uniform(-jitter, jitter, size=lat.shape)
    pos = (lat + 0.5 + jit) * spacing
    return np.ascontiguousarray(pos), int(inside.sum())


def _greedy_hard_core(cand: np.ndarray, prio: np.ndarray, r_min: float,
                      cell: float) -> np.ndarray:
    """Greedy dart-throwing over a stratified candidate grid.

    ``cand`` has shape ``(GX, GY, GZ, 3)`` with one candidate per grid cell of
    width ``cell``; candidates are visited in increasing ``prio`` and a
    candidate is accepted iff no already-accepted candidate lies closer than
    ``r_min``.  Requires ``r_min < cell`` so that only the 26 adjacent cells
    can conflict.  The sequential greedy result is computed exactly with the
    round-based "lexicographically first independent set" formulation:
    a candidate is accepted once every lower-priority conflicting candidate
    has been rejected; a candidate is rejected once a conflicting candidate
    has been accepted.  Returns a boolean acceptance grid."""
    assert r_min < cell
    shape = cand.shape[:3]
    offsets = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
               if (a, b, c) != (0, 0, 0)]

    def shifted(arr, off, fill):
        """out[i] = arr[i + off] where in range, else fill."""
        out = np.full(arr.shape, fill, dtype=arr.dtype)
        src = tuple(slice(max(o, 0), s + min(o, 0)) for o, s in zip(off, shape))
        dst = tuple(slice(max(-o, 0), s + min(-o, 0)) for o, s in zip(off, shape))
        out[dst] = arr[src]
        return out

    r2 = r_min * r_min
    conflict = []
    for off in offsets:
        d2 = np.zeros(shape)
        for ax in range(3):
            other = shifted(cand[..., ax], off, np.inf)
            diff = cand[..., ax] - other
            d2 += diff * diff
        conflict.append(d2 < r2)

    UNDECIDED, ACCEPTED, REJECTED = 0, 1, 2
    state = np.zeros(shape, dtype=np.int8)
    big = np.iinfo(prio.dtype).max
    while True:
        und = state == UNDECIDED
        if not und.any():
            break
        prio_und = np.where(und, prio, big)
        ok = und.copy()
        for off, cf in zip(offsets, conflict):
            nb = shifted(prio_und, off, big)
            ok &= ~(cf & (nb < prio))
        state[ok] = ACCEPTED
        acc = state == ACCEPTED
        rej = np.zeros(shape, dtype=bool)
        for off, cf in zip(offsets, conflict):
            rej |= cf & shifted(acc, off, False)
        state[und & ~ok & rej] = REJECTED
    return state == ACCEPTED


# Calibrated once on a 70^3 candidate grid: with r_min = 0.6 candidate cells the
# greedy sampler keeps ~0.80 of the candidates, above the (n/ceil(1.1 n))^3
# <= 1/1.1^3 = 0.751 (0.748 for n = 256) needed to draw n^3 points.
DART_RMIN_OVER_CELL = 0.60


def dart_throwing_points(n: int, rng: np.random.Generator, ghost_slab: float = 3.0):
    """``n**3`` quasi-uniform points in the unit cube by greedy rejection on a
    jittered candidate grid ``ceil(1.1 n)`` per side, plus a ghost slab of
    thickness ``ghost_slab / n`` at ``x < 0`` drawn by the same process.

    Returns ``(pos, n_interior)``: interior points in visit order, then ghosts
    in visit order."""
    G = int(math.ceil(1.1 * n))
    cell = 1.0 / G
    spacing = 1.0 / n
    gx0 = -int(math.ceil(ghost_slab * spacing / cell))     # extra x cells for the slab
    GX = G - gx0
    ix = np.arange(gx0, G)
    iy = np.arange(G)
    cand = np.empty((GX, G, G, 3))
    cand[..., 0] = ix[:, None, None]
    cand[..., 1] = iy[None, :, None]
    cand[..., 2] = iy[None, None, :]
    cand += 0.5 + rng.uniform(-0.5, 0.5, size=cand.shape)
    cand *= cell
    prio = rng.permutation(cand.shape[0] * G * G).astype(np.int64).reshape(GX, G, G)
    acc = _greedy_hard_core(cand, prio, DART_RMIN_OVER_CELL * cell, cell)
    x = cand[..., 0]
    interior = acc & (x >= 0.0)
    ghost = acc & (x < 0.0) & (x >= -ghost_slab * spacing)
    N = n ** 3
    int_prio = prio[interior]
    if int_prio.size < N:
        raise RuntimeError(f"dart throwing accepted {int_prio.size} < {N} points")
    order = np.argsort(int_prio, kind="stable")[:N]
    p_int = cand[interior][order]
    g_prio = prio[ghost]
    p_gh = cand[ghost][np.argsort(g_prio, kind="stable")]
    pos = np.concatenate([p_int, p_gh]).T
    return np.ascontiguousarray(pos), N


def _filled(n_total: int, value: float) -> np.ndarray:
    return np.full(n_total, float(value))


# ---------------------------------------------------------------------------
# manufactured solution T = 1 + 0.1 prod sin(pi x_a) exp(-t), E = a T^4
# (closed-form sources of the continuous equations, flux limiter fixed at 1/3)
# ---------------------------------------------------------------------------

def _mms_sinusoid(pos: np.ndarray, dim: int, rho: np.ndarray, cv: np.ndarray,
                  c: float, a: float, sigma_of_T: Callable, dsigma_dT: Callable,
                  sigma_grad_explicit: Optional[Callable] = None):
    """Closed-form manufactured sources for T(x,t)=1+0.1*prod_a sin(pi x_a)*exp(-t),
    e = cv*T, E = a*T^4.  The material equation gives Q_e = rho*cv*dT/dt (the
    emission and absorption terms cancel because E = aT^4); the diffusion
    equation with D = c/(3 sigma_t) gives Q_E = dE/dt - div(D grad E)."""
    x = pos
    sins = np.sin(np.pi * x)
    coss = np.cos(np.pi * x)
    s = np.prod(sins, axis=0)

    def f(t):
        et = math.exp(-t)
        T = 1.0 + 0.1 * s * et
        dTdt = -0.1 * s * et
        gT = np.empty_like(x)
        for al in range(dim):
            others = np.prod(np.delete(sins, al, axis=0), axis=0) if dim > 1 else 1.0
            gT[al] = 0.1 * np.pi * et * coss[al] * others
        lapT = -dim * np.pi ** 2 * 0.1 * s * et
        E = a * T ** 4
        gE = 4.0 * a * T ** 3 * gT
        lapE = 4.0 * a * (3.0 * T ** 2 * np.sum(gT * gT, axis=0) + T ** 3 * lapT)
        sig = sigma_of_T(T)
        if sigma_grad_explicit is not None:
            gsig = sigma_grad_explicit()
        else:
            gsig = dsigma_dT(T) * gT
        D = c / (3.0 * sig)
        gD = -c * gsig / (3.0 * sig ** 2)
        Qe = rho * cv * dTdt
        QE = 4.0 * a * T ** 3 * dTdt - (np.sum(gD * gE, axis=0) + D * lapE)
        return cv * T, E, Qe, QE

    return f


def config1(n: int = 64, seed: Optional[int] = None) -> Problem:
    """2D manufactured problem: n x n jittered lattice (+-0.1 spacing), 3 ghost
    layers, cubic spline with h = 1.3 spacing, sigma = 10(1 + 0.5 sin 2pi x sin 2pi y),
    one backward-Euler step of dt = 1e-3."""
    rng = np.random.default_rng(SEED_BASE + 1 if seed is None else seed)
    dim = 2
    dx = 1.0 / n
    pos, nin = jittered_lattice(dim, n, 0.1, 3, rng)
    N = pos.shape[1]
    rho = _filled(N, 1.0)
    cv = _filled(N, 1.0)
    sig0 = 10.0 * (1.0 + 0.5 * np.sin(2 * np.pi * pos[0]) * np.sin(2 * np.pi * pos[1]))

    def gsig():
        return np.stack([10.0 * np.pi * np.cos(2 * np.pi * pos[0]) * np.sin(2 * np.pi * pos[1]),
                         10.0 * np.pi * np.sin(2 * np.pi * pos[0]) * np.cos(2 * np.pi * pos[1])])

    mms = _mms_sinusoid(pos, dim, rho, cv, 1.0, 1.0, lambda T: sig0, None, gsig)
    e0, E0, _, _ = mms(0.0)
    prob = Problem(name="mms2d", dim=dim, pos=pos, h=_filled(N, 1.3 * dx), n_interior=nin,
                   m=_filled(N, dx * dx), rho=rho, cv=cv, sigma0_a=sig0,
                   sigma_s=np.zeros(N), opacity_exponent=0.0, e=e0.copy(), E=E0.copy(),
                   Q_e=np.zeros(N), Q_E=np.zeros(N), dt=1e-3, mms=mms,
                   meta=dict(config=1, n=n, spacing=dx))
    prob.set_time(prob.dt)
    return prob


def config2_mms(n: int = 64, seed: Optional[int] = None) -> Problem:
    """3D manufactured problem: n^3 jittered lattice (+-0.1), 3 ghost layers,
    h = 1.2 spacing, sigma_a = sigma_t = 10 T^-3 (frozen at the step start),
    dt = 1e-3.  Call ``set_time`` before each step."""
    rng = np.random.default_rng(SEED_BASE + 2 if seed is None else seed)
    dim = 3
    dx = 1.0 / n
    pos, nin = jittered_lattice(dim, n, 0.1, 3, rng)
    N = pos.shape[1]
    rho = _filled(N, 1.0)
    cv = _filled(N, 1.0)
    mms = _mms_sinusoid(pos, dim, rho, cv, 1.0, 1.0,
                        lambda T: 10.0 * T ** -3.0, lambda T: -30.0 * T ** -4.0)
    e0, E0, _, _ = mms(0.0)
    prob = Problem(name="mms3d", dim=dim, pos=pos, h=_filled(N, 1.2 * dx), n_interior=nin,
                   m=_filled(N, dx ** 3), rho=rho, cv=cv, sigma0_a=_filled(N, 10.0),
                   sigma_s=np.zeros(N), opacity_exponent=-3.0, e=e0.copy(), E=E0.copy(),
                   Q_e=np.zeros(N), Q_E=np.zeros(N), dt=1e-3, mms=mms,
                   meta=dict(config=2, n=n, spacing=dx))
    prob.set_time(prob.dt)
    return prob


def config2_infinite(T0: float, E0: float, n: int = 64, seed: Optional[int] = None,
                     sigma0: float = 10.0, dt: float = 1e-3) -> Problem:
    """3D infinite medium on the config-2 particles: uniform (T0, E0), no sources,
    no ghosts (a uniform field feels no diffusion), sigma_a = sigma0 T^-3."""
    rng = np.random.default_rng(SEED_BASE + 2 if seed is None else seed)
    dim = 3
    dx = 1.0 / n
    pos, nin = jittered_lattice(dim, n, 0.1, 0, rng)
    N = pos.shape[1]
    return Problem(name="infinite3d", dim=dim, pos=pos, h=_filled(N, 1.2 * dx), n_interior=nin,
                   m=_filled(N, dx ** 3), rho=_filled(N, 1.0), cv=_filled(N, 1.0),
                   sigma0_a=_filled(N, sigma0), sigma_s=np.zeros(N), opacity_exponent=-3.0,
                   e=_filled(N, T0), E=_filled(N, E0), Q_e=np.zeros(N), Q_E=np.zeros(N),
                   dt=dt, meta=dict(config=2, n=n, spacing=dx, T0=T0, E0=E0))


def _smooth_gaussian_field(shape, rng: np.random.Generator, radius: int = 2) -> np.ndarray:
    """Unit-variance Gaussian field on a periodic lattice: i.i.d. N(0,1) values
    filtered separably with a binomial window of half-width ``radius`` lattice
    sites and rescaled so each value is again N(0,1)."""
    z = rng.standard_normal(shape)
    w = np.array([math.comb(2 * radius, k) for k in range(2 * radius + 1)], dtype=float)
    w /= w.sum()
    for ax in range(len(shape)):
        acc = np.zeros(shape)
        for k, wk in enumerate(w):
            acc += wk * np.roll(z, k - radius, axis=ax)
        z = acc
    return z / math.sqrt(float(np.sum(w * w)) ** len(shape))


def config3(n: int = 128, seed: Optional[int] = None) -> Problem:
    """3D density step: n^3 jittered lattice (+-0.2), equal masses, rho = 1 for
    x < 0.5 and 4 for x >= 0.5, h = 1.2 (m/rho)^(1/3), lognormal opacity
    (mu = ln 10, s = 1) with a ~2h correlation length, Larsen k = 2 flux
    limiter, T0 = 1 + 0.1 prod sin(pi x_a), E0 = (0.9 T0)^4, free boundaries."""
    rng = np.random.default_rng(SEED_BASE + 3 if seed is None else seed)
    dim = 3
    dx = 1.0 / n
    pos, nin = jittered_lattice(dim, n, 0.2, 0, rng)
    N = pos.shape[1]
    m = _filled(N, dx ** 3)
    rho = np.where(pos[0] < 0.5, 1.0, 4.0)
    h = 1.2 * np.cbrt(m / rho)
    z = _smooth_gaussian_field((n, n, n), rng).reshape(-1)   # lattice order, x fastest
    sig = np.exp(math.log(10.0) + z)
    T0 = 1.0 + 0.1 * np.prod(np.sin(np.pi * pos), axis=0)
    cv = _filled(N, 1.0)
    return Problem(name="densitystep3d", dim=dim, pos=pos, h=h, n_interior=nin, m=m, rho=rho,
                   cv=cv, sigma0_a=sig, sigma_s=np.zeros(N), opacity_exponent=0.0,
                   e=cv * T0, E=(0.9 * T0) ** 4, Q_e=np.zeros(N), Q_E=np.zeros(N), dt=1e-3,
                   limiter=LIMITER_LARSEN, limiter_k=2.0,
                   meta=dict(config=3, n=n, spacing=dx))


def wendland_lattice(dim: int, n: int, seed: Optional[int] = None) -> Problem:
    """The paper's own kernel regime (Sec. 2.3, Sec. 3.1): a jittered n^dim
    lattice (+-0.1 spacing) with two ghost layers, the Wendland kernel at
    h = 4 spacings (support h: about 50 neighbours in 2-D, 250 in 3-D),
    m = spacing^dim, rho = c_v = 1, T = 1 + 0.2 prod sin(pi x_a), E = (0.9 T)^4,
    sigma_a = 10 T^-3, dt = 1e-3."""
    rng = np.random.default_rng(SEED_BASE + 700 + dim if seed is None else seed)
    pos, nin = jittered_lattice(dim, n, 0.1, 2, rng)
    N = pos.shape[1]
    dx = 1.0 / n
    T = 1.0 + 0.2 * np.prod(np.sin(np.pi * np.clip(pos, 0.0, 1.0)), axis=0)
    return Problem(name=f"wendland{dim}d", dim=dim, pos=pos, h=_filled(N, 4.0 * dx),
                   n_interior=nin, m=_filled(N, dx ** dim), rho=_filled(N, 1.0),
                   cv=_filled(N, 1.0), sigma0_a=_filled(N, 10.0), sigma_s=np.zeros(N),
                   opacity_exponent=-3.0, e=T.copy(), E=(0.9 * T) ** 4, Q_e=np.zeros(N),
                   Q_E=np.zeros(N), dt=1e-3, kernel=KERNEL_WENDLAND_C4)


def periodic_wendland(dim: int, n: int, seed: Optional[int] = None) -> Problem:
    """The geometry of the paper's periodic manufactured problem (Sec. 4.3):
    a jittered n^dim lattice (+-0.1 spacing) on the unit box, periodic on
    every axis (jittered points wrapped back into [0, 1)), the Wendland kernel
    at h = 4 spacings; m = spacing^dim, rho = c_v = 1,
    T = 1 + 0.2 prod cos(2 pi x_a), E = (0.9 T)^4, sigma_a = 10 T^-3, dt = 1e-3."""
    rng = np.random.default_rng(SEED_BASE + 800 + dim if seed is None else seed)
    pos, nin = jittered_lattice(dim, n, 0.1, 0, rng)
    pos = np.mod(pos, 1.0)
    N = pos.shape[1]
    dx = 1.0 / n
    T = 1.0 + 0.2 * np.prod(np.cos(2.0 * np.pi * pos), axis=0)
    return Problem(name=f"periodic{dim}d", dim=dim, pos=pos, h=_filled(N, 4.0 * dx),
                   n_interior=nin, m=_filled(N, dx ** dim), rho=_filled(N, 1.0),
                   cv=_filled(N, 1.0), sigma0_a=_filled(N, 10.0), sigma_s=np.zeros(N),
                   opacity_exponent=-3.0, e=T.copy(), E=(0.9 * T) ** 4, Q_e=np.zeros(N),
                   Q_E=np.zeros(N), dt=1e-3, kernel=KERNEL_WENDLAND_C4,
                   period=np.ones(dim))


# cgs constants of the cos-wave manufactured problem (Sec. 4.3)
CGS_C = 2.99792458e10            # speed of light, cm/s
CGS_A = 7.565723e-15             # radiation constant a = 4 sigma_SB / c, erg cm^-3 K^-4
CGS_KB = 1.380649e-16            # Boltzmann constant, erg/K
CGS_MP = 1.67262192e-24          # proton mass, g


def cos_wave_fields(pos, t: float, e0: float, E0: float, v: float, d: float, omega: float,
                    xp=np):
    """The manufactured solution of Sec. 4.3 and its derivatives at time t:
    e_m = e0 [1.2 + prod_a cos th_a],  th_a = 2 pi (x_a - v t)/d,
    E_m = E0 [1.2 + prod_a cos ph_a],  ph_a = 2 pi (x_a + v t)/d - omega.
    Returns (e_m, E_m, de_m/dt, dE_m/dt, Laplacian of E_m).  ``xp`` is the
    array module of ``pos`` (numpy, or torch for device arrays)."""
    k = 2.0 * np.pi / d
    dim = pos.shape[0]
    th = [k * (pos[a] - v * t) for a in range(dim)]
    ph = [k * (pos[a] + v * t) - omega for a in range(dim)]
    ce, cE = [xp.cos(u) for u in th], [xp.cos(u) for u in ph]

    def prod(fs, skip=-1):
        out = None
        for a, f in enumerate(fs):
            if a != skip:
                out = f if out is None else out * f
        return 1.0 if out is None else out

    # d/dt prod_a cos(u_a) = sum_a (-sin u_a) du_a/dt prod_{b != a} cos u_b
    de = 0.0
    dE = 0.0
    for a in range(dim):
        de = de + xp.sin(th[a]) * (k * v) * prod(ce, a)
        dE = dE - xp.sin(ph[a]) * (k * v) * prod(cE, a)
    Pe, PE = prod(ce), prod(cE)
    return (e0 * (1.2 + Pe), E0 * (1.2 + PE), e0 * de, E0 * dE, -dim * k * k * E0 * PE)


class CosWaveSources:
    """Sources of the step ending at t for the cos-wave problem (see
    ``cos_wave_mms``), evaluated with the array module of ``pos``."""

    def __init__(self, pos, consts: dict, xp=np):
        self.pos, self.c, self.xp = pos, consts, xp

    def __call__(self, t: float):
        c = self.c
        e_m, E_m, de, dE, lapE = cos_wave_fields(self.pos, t, c["e0"], c["E0"], c["v"], c["d"],
                                                 c["omega"], self.xp)
        x = c["c"] * c["sigma_a"] * (c["a"] * (e_m / c["cv"]) ** 4 - E_m)   # emission - absorption
        return e_m, E_m, c["rho"] * de + x, dE - c["D"] * lapE - x


def cos_wave_mms(dim: int, n: int, steps: int = 1000) -> Problem:
    """The paper's manufactured problem for material-radiation coupling
    (Sec. 4.3): an unjittered n^dim lattice on the periodic box [0, d_m)^dim,
    d_m = 5 cm (one wavelength per axis), the Wendland kernel at h = 4
    spacings, e0 = 1e13 erg/g, E0 = 7 a (e0/c_v)^4, v_m = 5e9 cm/s,
    omega_m = 1/16, sigma_a = 0.05 and sigma_s = 0.95 per cm (constant), the
    ideal gas c_v = k_B/(mu (gamma - 1) m_p) with gamma = 5/3 and mu = 1, one
    cycle t_end = d_m/v_m in ``steps`` steps of dt = t_end/steps.
    Readings (the paper leaves them open): rho = E0/e0, so that the material
    and radiation energy densities, and with them the terms of both
    equations, are of one magnitude; no flux limiter (lambda = 1/3, so
    D = c/(3 sigma_t) is constant); the sources of the step ending at t are
    the manufactured residuals at t (backward Euler):
    Q_e = rho de_m/dt + c sigma_a (a T_m^4 - E_m),
    Q_E = dE_m/dt - D lap E_m - c sigma_a (a T_m^4 - E_m),  T_m = e_m/c_v.
    Call ``set_time`` before each step."""
    d, v, omega = 5.0, 5.0e9, 1.0 / 16.0
    e0 = 1.0e13
    gamma, mu = 5.0 / 3.0, 1.0
    cv = CGS_KB / (mu * (gamma - 1.0) * CGS_MP)
    E0 = 7.0 * CGS_A * (e0 / cv) ** 4
    rho = E0 / e0
    sa, ss = 0.05, 0.95
    D = CGS_C / (3.0 * (sa + ss))
    dx = d / n
    pos, nin = jittered_lattice(dim, n, 0.0, 0, np.random.default_rng(0))
    pos = pos * d
    N = pos.shape[1]

    consts = dict(e0=e0, E0=E0, v=v, d=d, omega=omega, c=CGS_C, a=CGS_A, cv=cv, rho=rho,
                  sigma_a=sa, D=D)
    mms = CosWaveSources(pos, consts)
    t_end = d / v
    e_i, E_i, _, _ = mms(0.0)
    prob = Problem(name=f"coswave{dim}d", dim=dim, pos=pos, h=_filled(N, 4.0 * dx),
                   n_interior=nin, m=_filled(N, rho * dx ** dim), rho=_filled(N, rho),
                   cv=_filled(N, cv), sigma0_a=_filled(N, sa), sigma_s=_filled(N, ss),
                   opacity_exponent=0.0, e=e_i.copy(), E=E_i.copy(), Q_e=np.zeros(N),
                   Q_E=np.zeros(N), dt=t_end / steps, c=CGS_C, a=CGS_A,
                   kernel=KERNEL_WENDLAND_C4, mms=mms, period=np.full(dim, d),
                   meta=dict(n=n, spacing=dx, t_end=t_end, steps=steps, consts=consts))
    prob.set_time(prob.dt)
    return prob


def config4(n: int = 256, seed: Optional[int] = None) -> Problem:
    """3D Marshak-like front on a non-lattice point set: n^3 points by greedy
    dart throwing on a jittered ceil(1.1 n)^3 candidate grid, V = 1/n^3,
    h = 1.2 V^(1/3); T = 0.01 inside, Dirichlet ghost slab x in [-3/n, 0) at
    T = 1; sigma_a = T^-3; dt = 1e-3."""
    rng = np.random.default_rng(SEED_BASE + 4 if seed is None else seed)
    pos, nin = dart_throwing_points(n, rng)
    N = pos.shape[1]
    V = 1.0 / n ** 3
    T = np.where(np.arange(N) < nin, 0.01, 1.0)
    return Problem(name="marshak3d", dim=3, pos=pos, h=_filled(N, 1.2 * V ** (1.0 / 3.0)),
                   n_interior=nin, m=_filled(N, V), rho=_filled(N, 1.0), cv=_filled(N, 1.0),
                   sigma0_a=_filled(N, 1.0), sigma_s=np.zeros(N), opacity_exponent=-3.0,
                   e=T.copy(), E=T ** 4, Q_e=np.zeros(N), Q_E=np.zeros(N), dt=1e-3,
                   meta=dict(config=4, n=n, outer_iterations=5))


def ensemble_sizes(nprob: int = 96, lo: int = 8000, hi: int = 500000,
                   seed: int = SEED_ENSEMBLE) -> np.ndarray:
    """Particle-count targets drawn log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=nprob))


def config5_member(p: int, target: float) -> Problem:
    """Ensemble member p: even p -> 2D lattice n = round(sqrt(target)), h = 1.3
    spacing; odd p -> 3D lattice n = round(cbrt(target)), h = 1.2 spacing;
    jitter +-0.15; sigma0 ~ U[1,100], sigma_a = sigma0 T^-3; dt ~ U[1e-4, 1e-2];
    T0 and E0 as in the density-step problem; free boundaries."""
    rng = np.random.default_rng(SEED_ENSEMBLE + p)
    dim = 2 if p % 2 == 0 else 3
    n = int(round(target ** (1.0 / dim)))
    n = max(n, 4)
    dx = 1.0 / n
    pos, nin = jittered_lattice(dim, n, 0.15, 0, rng)
    N = pos.shape[1]
    sigma0 = rng.uniform(1.0, 100.0)
    dt = rng.uniform(1e-4, 1e-2)
    T0 = 1.0 + 0.1 * np.prod(np.sin(np.pi * pos), axis=0)
    cv = _filled(N, 1.0)
    return Problem(name=f"ensemble{p}", dim=dim, pos=pos,
                   h=_filled(N, (1.3 if dim == 2 else 1.2) * dx), n_interior=nin,
                   m=_filled(N, dx ** dim), rho=_filled(N, 1.0), cv=cv,
                   sigma0_a=_filled(N, sigma0), sigma_s=np.zeros(N), opacity_exponent=-3.0,
                   e=cv * T0, E=(0.9 * T0) ** 4, Q_e=np.zeros(N), Q_E=np.zeros(N), dt=dt,
                   meta=dict(config=5, member=p, n=n, sigma0=sigma0))


def config5(nprob: int = 96, scale: float = 1.0) -> list:
    """The ensemble: ``nprob`` independent problems with log-uniform sizes
    (``scale`` shrinks every member, for tests)."""
    sizes = ensemble_sizes(nprob)
    return [config5_member(p, max(64.0, s * scale)) for p, s in enumerate(sizes)]
