"""Geometric multigrid for the coarse Dirichlet problem (oracle; test infrastructure only).

CGP treats the coarse elliptic solve as a black box (Sec. 3: any solver of
the coarse problem can be wrapped; the introduction expects larger savings
with slower solvers than the fast Poisson solver the paper uses).  This is a
textbook V(2,2) cycle for Lap_h u = f (5-point Laplacian, spacings dx, dy,
u = 0 on the ring of an nx x ny interval grid):

* smoother: red-black Gauss-Seidel, red = interior nodes with i + j even;
  pre-smoothing red then black, post-smoothing black then red;
* transfers: full weighting of the residual and bilinear interpolation of the
  correction (the Sec. 3.1 operators of transfer.py);
* coarsening while both interval counts are even and at least 8; the
  coarsest grid is solved exactly (dense inverse of its 5-point matrix);
* a solve runs `cycles` V-cycles from u = 0.
"""
from __future__ import annotations

import numpy as np

from . import transfer

NU1 = 2
NU2 = 2


def laplacian_matrix(nx: int, ny: int, dx: float, dy: float) -> np.ndarray:
    """Dense 5-point Laplacian on the interior nodes, row-major (j, i)."""
    n = (nx - 1) * (ny - 1)
    A = np.zeros((n, n))
    ax, ay = 1.0 / dx ** 2, 1.0 / dy ** 2
    for j in range(1, ny):
        for i in range(1, nx):
            k = (j - 1) * (nx - 1) + (i - 1)
            A[k, k] = -2.0 * ax - 2.0 * ay
            if i > 1:
                A[k, k - 1] = ax
            if i < nx - 1:
                A[k, k + 1] = ax
            if j > 1:
                A[k, k - (nx - 1)] = ay
            if j < ny - 1:
                A[k, k + (nx - 1)] = ay
    return A


def coarsest(nx: int, ny: int) -> bool:
    return nx % 2 == 1 or ny % 2 == 1 or nx < 8 or ny < 8


def rb_sweep(u: np.ndarray, f: np.ndarray, dx: float, dy: float, color: int) -> None:
    """One half sweep of Gauss-Seidel on the nodes of one colour (in place)."""
    ny, nx = u.shape[0] - 1, u.shape[1] - 1
    ax, ay = 1.0 / dx ** 2, 1.0 / dy ** 2
    J, I = np.meshgrid(np.arange(1, ny), np.arange(1, nx), indexing="ij")
    mask = (I + J) % 2 == color
    nb = ax * (u[1:-1, 2:] + u[1:-1, :-2]) + ay * (u[2:, 1:-1] + u[:-2, 1:-1])
    new = (nb - f[1:-1, 1:-1]) / (2.0 * ax + 2.0 * ay)
    inner = u[1:-1, 1:-1]
    inner[mask] = new[mask]


def residual(u: np.ndarray, f: np.ndarray, dx: float, dy: float) -> np.ndarray:
    """f - Lap_h u at interior nodes, 0 on the ring."""
    r = np.zeros_like(u)
    lap = ((u[1:-1, 2:] - 2.0 * u[1:-1, 1:-1] + u[1:-1, :-2]) / dx ** 2
           + (u[2:, 1:-1] - 2.0 * u[1:-1, 1:-1] + u[:-2, 1:-1]) / dy ** 2)
    r[1:-1, 1:-1] = f[1:-1, 1:-1] - lap
    return r


def bottom_solve(f: np.ndarray, dx: float, dy: float) -> np.ndarray:
    ny, nx = f.shape[0] - 1, f.shape[1] - 1
    u = np.zeros_like(f)
    u[1:-1, 1:-1] = np.linalg.solve(laplacian_matrix(nx, ny, dx, dy),
                                    f[1:-1, 1:-1].reshape(-1)).reshape(ny - 1, nx - 1)
    return u


def vcycle(u: np.ndarray, f: np.ndarray, dx: float, dy: float) -> None:
    """One V-cycle on u (in place)."""
    ny, nx = u.shape[0] - 1, u.shape[1] - 1
    if coarsest(nx, ny):
        u[...] = bottom_solve(f, dx, dy)
        return
    for _ in range(NU1):
        rb_sweep(u, f, dx, dy, 0)
        rb_sweep(u, f, dx, dy, 1)
    fc = transfer.restrict_fw(residual(u, f, dx, dy))
    uc = np.zeros_like(fc)
    vcycle(uc, fc, 2.0 * dx, 2.0 * dy)
    u += transfer.prolong_bilinear(uc)
    for _ in range(NU2):
        rb_sweep(u, f, dx, dy, 1)
        rb_sweep(u, f, dx, dy, 0)


def poisson_mg(r: np.ndarray, dx: float, dy: float, cycles: int) -> np.ndarray:
    """`cycles` V-cycles from zero for Lap_h psi = r (node arrays, zero ring)."""
    u = np.zeros_like(np.asarray(r, dtype=np.float64))
    f = np.asarray(r, dtype=np.float64)
    for _ in range(cycles):
        vcycle(u, f, dx, dy)
    return u
