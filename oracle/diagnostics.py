"""Basin diagnostics (oracle; test infrastructure only).

Kinetic energy: eq. 26, E = 1/2 integral (psi_x^2 + psi_y^2) dx dy, discretised
with forward differences on every grid link (x-links on interior rows, y-links
on interior columns; links on the walls carry psi = 0 at both ends) and divided
by the basin area so that it is a domain average.  Enstrophy (not defined in
the paper; added as the companion statistic): Z = 1/2 <omega^2>, same average.
For two layers E_i uses psi_i and Z_i uses Q_i.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


def energy(psi, grid: Grid) -> float:
    dx, dy = grid.dx, grid.dy
    area = grid.lx * grid.ly
    ex = ((psi[1:-1, 1:] - psi[1:-1, :-1]) / dx) ** 2    # i = 0..nx-1, j = 1..ny-1
    ey = ((psi[1:, 1:-1] - psi[:-1, 1:-1]) / dy) ** 2    # i = 1..nx-1, j = 0..ny-1
    return float(dx * dy / (2.0 * area) * (ex.sum() + ey.sum()))


def enstrophy(omega, grid: Grid) -> float:
    area = grid.lx * grid.ly
    return float(grid.dx * grid.dy / (2.0 * area) * np.sum(omega[1:-1, 1:-1] ** 2))
