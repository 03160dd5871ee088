"""Adaptive time-step choice of Sec. 3.3 (oracle, FP64).

eta_e = max_i |e_i^n - e_i^{n-1}| / (e_i^n + eta_target * ebar^n + tiny), with
ebar^n the volume-weighted mean of e^n; proposed dt_e = dt^n (eta_target/eta_e)^(1/2).
The same is done for E and the smaller proposal is taken, clipped to the
user's [dt_min, dt_max] and to at most ``max_growth`` times the previous step
(Sec. 4.1 allows one order of magnitude per step).
"""
from __future__ import annotations

import numpy as np


def fractional_change(new, old, V, eta_target: float, tiny: float = 1e-15) -> float:
    bar = float(np.sum(new * V) / np.sum(V))
    return float(np.max(np.abs(new - old) / (new + eta_target * bar + tiny)))


def next_dt(dt: float, e_new, e_old, E_new, E_old, V, eta_target: float = 0.05,
            dt_min: float = 0.0, dt_max: float = np.inf, max_growth: float = 10.0) -> float:
    props = []
    for new, old in ((e_new, e_old), (E_new, E_old)):
        eta = fractional_change(new, old, V, eta_target)
        props.append(np.inf if eta == 0.0 else dt * (eta_target / eta) ** 0.5)
    out = min(props)
    out = min(out, max_growth * dt, dt_max)
    return max(out, dt_min)
