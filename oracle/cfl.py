"""Adaptive CFL time step of Sec. 4.2 (oracle; test infrastructure only).

Sec. 4.2 sets the step size from the CFL number c after every time step:

    dt = c min(dx, dy) / max{ |d psi_i/dx|, |d psi_i/dy| },

the maximum taken over the grid and the layers.  The paper leaves three
things open; the readings used here (and by the GPU path) are:

* the derivatives are centred differences at the interior nodes,
  (psi_{i+1,j} - psi_{i-1,j}) / (2 dx) and (psi_{i,j+1} - psi_{i,j-1}) / (2 dy);
* "at the end of each time step" uses the stream function in hand at that
  point of the CGPRK3 step (Sec. 3.2 listing): the prolonged psi of the
  step's third stage, psi = A_l w2;
* the step size never exceeds dt_max, the configured step, which is also the
  size of the first step (the paper's runs start from rest, where the CFL
  bound is infinite); a state with psi = 0 everywhere takes dt_max.
"""
from __future__ import annotations

import numpy as np

from . import model
from .grid import Grid


def max_velocity(psi, grid: Grid) -> float:
    """max over interior nodes (and layers) of |psi_x| and |psi_y|, centred differences."""
    p = np.asarray(psi, dtype=np.float64)
    if p.ndim == 2:
        p = p[None]
    vx = np.abs(p[:, 1:-1, 2:] - p[:, 1:-1, :-2]) / (2.0 * grid.dx)
    vy = np.abs(p[:, 2:, 1:-1] - p[:, :-2, 1:-1]) / (2.0 * grid.dy)
    return float(max(vx.max(initial=0.0), vy.max(initial=0.0)))


def cfl_dt(psi, grid: Grid, cfl: float, dt_max: float) -> float:
    """The Sec. 4.2 step size from psi, capped at dt_max."""
    m = max_velocity(psi, grid)
    if m == 0.0:
        return dt_max
    return min(dt_max, cfl * min(grid.dx, grid.dy) / m)


def run_adaptive(omega0, forcing, grid: Grid, level: int, phys: model.Physics, cfl: float,
                 dt_max: float, nsteps: int, nlayers: int = 1, route: str = "dst",
                 callback=None):
    """Advance nsteps with adaptive steps (cfl <= 0: every step dt_max).  Returns
    (state, list of the dt of every step).  callback(n, state, dt) after every
    step if given."""
    w = np.array(omega0, dtype=np.float64)
    dt = dt_max
    dts = []
    for n in range(nsteps):
        if nlayers == 1:
            w, stages = model.step(w, forcing, grid, level, phys, dt, route, return_stages=True)
        else:
            w, stages = model.step_two_layer(w, forcing, grid, level, phys, dt, route,
                                             return_stages=True)
        dts.append(dt)
        if callback is not None:
            callback(n + 1, w, dt)
        dt = cfl_dt(stages[2][1], grid, cfl, dt_max) if cfl > 0 else dt_max
    return w, dts
