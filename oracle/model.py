"""CGPRK3 time step of the one- and two-layer QG models (oracle; test infrastructure only).

Vorticity form (dividing the nondimensional equations of Sec. 2.1/2.2 by Ro,
with q = Ro*omega + y, omega = Laplacian(psi), u = -psi_y, v = psi_x):

  one layer   d omega/dt = G = -J(psi, omega) - (1/Ro) J(psi, y)
                              + (1/Re) Lap(omega) + F
  two layers  d Q_i/dt = -J(psi_i, Q_i) - (1/Ro) J(psi_i, y) + (1/Re) Lap(zeta_i)
                         + [i=1] F - [i=2] (sigma/Ro) zeta_2,
              zeta_i = Q_i - F_i (psi_j - psi_i),  1/Re = A/Ro

J is the Arakawa Jacobian (Sec. 4.1).  The eddy-viscosity term nu Lap^2 psi is
applied as the 5-point Laplacian of the fine prognostic relative vorticity
(omega, or zeta_i), which is zero on the free-slip walls (Sec. 2.1, 2.2).

CGP (Sec. 3, steps (i)-(iv)): psi = P^l L_c^-1 R^l omega, with R full weighting
and P bilinear prolongation applied l times (Sec. 3.1), L_c^-1 the exact coarse
Dirichlet solve (Sec. 4.3).  l = 0 is the plain full-grid solver.

Time stepping (Sec. 3.2 listing and Sec. 4.2): TVD-RK3
  w1 = wn + dt G(wn);  w2 = 3/4 wn + 1/4 w1 + 1/4 dt G(w1);
  w_{n+1} = 1/3 wn + 2/3 w2 + 2/3 dt G(w2),
with a fresh coarse solve before each of the three right-hand sides.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import elliptic, operators as ops, transfer
from .grid import Grid


@dataclasses.dataclass(frozen=True)
class Physics:
    inv_re: float
    inv_ro: float
    f1: float = 0.0
    f2: float = 0.0
    drag: float = 0.0


RK3_A = (0.0, 0.75, 1.0 / 3.0)
RK3_B = (1.0, 0.25, 2.0 / 3.0)


def zero_ring(f):
    f = np.array(f, dtype=np.float64, copy=True)
    f[..., 0, :] = 0.0
    f[..., -1, :] = 0.0
    f[..., :, 0] = 0.0
    f[..., :, -1] = 0.0
    return f


# ---------------------------------------------------------------------------
# Elliptic map A_l (steps (ii)-(iv) of the CGP procedure).
# ---------------------------------------------------------------------------
def cgp_psi(omega, grid: Grid, level: int, route: str = "dst"):
    """psi = P^l L_c^-1 R^l omega (one layer)."""
    r = transfer.restrict(omega, level)
    cg = grid.coarse(level)
    psi_c = elliptic.poisson(r, cg.dx, cg.dy, route)
    return transfer.prolong(psi_c, level)


def cgp_psi_two_layer(Q, grid: Grid, level: int, phys: Physics, route: str = "dst"):
    """(psi1, psi2) from (Q1, Q2): restrict each layer, coupled coarse solve, prolong."""
    r1 = transfer.restrict(Q[0], level)
    r2 = transfer.restrict(Q[1], level)
    cg = grid.coarse(level)
    p1, p2 = elliptic.two_layer(r1, r2, cg.dx, cg.dy, phys.f1, phys.f2, route)
    return np.stack([transfer.prolong(p1, level), transfer.prolong(p2, level)])


# ---------------------------------------------------------------------------
# Right-hand sides.
# ---------------------------------------------------------------------------
def rhs(omega, psi, forcing, grid: Grid, phys: Physics):
    """G(omega, psi; F) at interior nodes (one layer), zero on the ring."""
    dx, dy = grid.dx, grid.dy
    g = (-ops.arakawa(psi, omega, dx, dy)
         - phys.inv_ro * ops.beta_term(psi, grid)
         + phys.inv_re * ops.laplacian(omega, dx, dy)
         + forcing)
    return zero_ring(g)


def relative_vorticity_two_layer(Q, psi, phys: Physics):
    """zeta_1 = Q_1 - F1 (psi_2 - psi_1), zeta_2 = Q_2 - F2 (psi_1 - psi_2), zero ring."""
    z1 = Q[0] - phys.f1 * (psi[1] - psi[0])
    z2 = Q[1] - phys.f2 * (psi[0] - psi[1])
    return zero_ring(np.stack([z1, z2]))


def rhs_two_layer(Q, psi, forcing, grid: Grid, phys: Physics):
    dx, dy = grid.dx, grid.dy
    zeta = relative_vorticity_two_layer(Q, psi, phys)
    out = np.zeros_like(Q, dtype=np.float64)
    for i in range(2):
        g = (-ops.arakawa(psi[i], Q[i], dx, dy)
             - phys.inv_ro * ops.beta_term(psi[i], grid)
             + phys.inv_re * ops.laplacian(zeta[i], dx, dy))
        if i == 0:
            g = g + forcing
        else:
            g = g - phys.drag * zeta[1]
        out[i] = zero_ring(g)
    return out


# ---------------------------------------------------------------------------
# CGPRK3 steps.
# ---------------------------------------------------------------------------
def step(omega, forcing, grid: Grid, level: int, phys: Physics, dt: float,
         route: str = "dst", return_stages: bool = False):
    """One CGPRK3 step of the one-layer model."""
    wn = zero_ring(omega)
    F = np.asarray(forcing, dtype=np.float64)
    stages = []
    w = wn
    for s in range(3):
        psi = cgp_psi(w, grid, level, route)
        stages.append((w, psi))
        g = rhs(w, psi, F, grid, phys)
        w = RK3_A[s] * wn + RK3_B[s] * (w + dt * g)
        w = zero_ring(w)
    if return_stages:
        return w, stages
    return w


def step_two_layer(Q, forcing, grid: Grid, level: int, phys: Physics, dt: float,
                   route: str = "dst", return_stages: bool = False):
    """One CGPRK3 step of the two-layer model."""
    Qn = zero_ring(Q)
    F = np.asarray(forcing, dtype=np.float64)
    w = Qn
    stages = []
    for s in range(3):
        psi = cgp_psi_two_layer(w, grid, level, phys, route)
        stages.append((w, psi))
        g = rhs_two_layer(w, psi, F, grid, phys)
        w = zero_ring(RK3_A[s] * Qn + RK3_B[s] * (w + dt * g))
    if return_stages:
        return w, stages
    return w


def step_qform(q, forcing_q, grid: Grid, level: int, ro: float, re: float, dt: float,
               route: str = "dst"):
    """The paper's own potential-vorticity form of one CGPRK3 step (Sec. 3.2).

    q = Ro Lap(psi) + y is stepped with G = -J(psi, q) + (Ro/Re) Lap(Lap psi)
    + forcing, where the elliptic right-hand side is (q_bar - y)/Ro on the coarse
    grid and the dissipation is applied as (Ro/Re) Lap((q - y)/Ro) (the same
    discrete viscous operator as the vorticity form).  Used to pin the
    equivalence of the two forms; it loses digits to the y offset in FP64.
    """
    y = grid.y_field()
    qn = np.array(q, dtype=np.float64)
    w = qn
    cg = grid.coarse(level)
    yc = cg.y_field()
    for s in range(3):
        rel = zero_ring((w - y) / ro)
        qbar = transfer.restrict(w, level)          # q => q_bar
        rbar = zero_ring((qbar - yc) / ro)          # (delta_I/L)^-2 (q_bar - y)
        psi = transfer.prolong(elliptic.poisson(rbar, cg.dx, cg.dy, route), level)
        g = (-ops.arakawa(psi, w, grid.dx, grid.dy)
             + (ro / re) * ops.laplacian(rel, grid.dx, grid.dy)
             + forcing_q)
        g = zero_ring(g)
        w = RK3_A[s] * qn + RK3_B[s] * (w + dt * g)
        # walls keep q = y (omega = 0 there)
        w[0, :], w[-1, :], w[:, 0], w[:, -1] = y[0, :], y[-1, :], y[:, 0], y[:, -1]
    return w


def run(omega0, forcing, grid: Grid, level: int, phys: Physics, dt: float, nsteps: int,
        nlayers: int = 1, route: str = "dst", callback=None):
    """Advance nsteps; callback(n, state) after every step if given."""
    w = np.array(omega0, dtype=np.float64)
    for n in range(nsteps):
        if nlayers == 1:
            w = step(w, forcing, grid, level, phys, dt, route)
        else:
            w = step_two_layer(w, forcing, grid, level, phys, dt, route)
        if callback is not None:
            callback(n + 1, w)
    return w
