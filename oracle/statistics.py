"""Time means of long runs (Sec. 5.1; oracle, test infrastructure only).

The paper's one-layer experiments average the flow over t in [10, 50] after
the spin-up (Sec. 5.1, from 20 thousand snapshots).  With steps of varying
size the time mean of omega over the steps n0 < n <= n1 is taken here as the
rectangle rule on the step grid,

    <omega> = sum_n dt_n omega_n / sum_n dt_n,

omega_n the state after step n and dt_n that step's size.  The elliptic map
psi = A_l omega is linear, so <psi> = A_l <omega>; the potential vorticity
q = Ro omega + y (vorticity form, R3) has <q> = Ro <omega> + y.
"""
from __future__ import annotations

import numpy as np

from . import cfl as cfl_mod
from . import model
from .grid import Grid


def time_mean(omega0, forcing, grid: Grid, level: int, phys: model.Physics, cfl: float,
              dt_max: float, n_spin: int, n_avg: int, nlayers: int = 1, route: str = "dst"):
    """Run n_spin steps, then n_avg steps accumulating dt_n omega_n.  Returns
    (<omega>, <psi>, sum of dt_n over the window, final state)."""
    acc = np.zeros_like(np.asarray(omega0, dtype=np.float64))
    tsum = [0.0]

    def cb(n, w, dt):
        if n > n_spin:
            acc[...] += dt * w
            tsum[0] += dt

    w_end, _ = cfl_mod.run_adaptive(omega0, forcing, grid, level, phys, cfl, dt_max,
                                    n_spin + n_avg, nlayers=nlayers, route=route, callback=cb)
    mean_w = acc / tsum[0]
    if nlayers == 1:
        mean_psi = model.cgp_psi(mean_w, grid, level, route)
    else:
        mean_psi = model.cgp_psi_two_layer(mean_w, grid, level, phys, route)
    return mean_w, mean_psi, tsum[0], w_end
