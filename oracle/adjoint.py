"""Tangent-linear and adjoint of the one-layer CGPRK3 step (oracle; test infrastructure only).

The forward step is the one in ``model`` (Sec. 3.2 listing, Sec. 4.1 Jacobian,
Sec. 3.1 transfers, Sec. 4.3 solve).  Linearising one right-hand side about a
stage state (omega_s, psi_s):

    dG = -J(dpsi, omega_s) - J(psi_s, domega) - (1/Ro) J(dpsi, y)
         + (1/Re) Lap(domega) + dF,        dpsi = A_l domega,

with A_l = P^l L_c^-1 R^l.  The adjoint below is the literal transpose of
these maps: each 9-point operator is transposed by ``operators.transpose_apply``
(which probes the operator, no identity assumed), R and P by their scatter
transposes, and L_c^-1 by itself (the 5-point Dirichlet Laplacian is a
symmetric matrix).  The RK3 stages are reversed in the usual way for
w_{s+1} = a_s w_n + b_s (w_s + dt G_s).

Loss (final-time misfit at observation nodes):  L = (1/K) sum_p (omega_p - o_p)^2.
"""
from __future__ import annotations

import numpy as np

from . import elliptic, operators as ops, transfer
from .grid import Grid
from .model import Physics, RK3_A, RK3_B, cgp_psi, rhs, step, zero_ring


def cgp_psi_T(lam, grid: Grid, level: int, route: str = "dst"):
    """A_l^T lam = (R^l)^T L_c^-1 (P^l)^T lam (fine interior -> fine interior)."""
    g = transfer.prolong_T(zero_ring(lam), level)
    g = zero_ring(g)
    cg = grid.coarse(level)
    psi_c = elliptic.poisson(g, cg.dx, cg.dy, route)
    return zero_ring(transfer.restrict_T(psi_c, level))


def rhs_tlm(omega, psi, domega, dpsi, dforcing, grid: Grid, phys: Physics):
    dx, dy = grid.dx, grid.dy
    d = (-ops.arakawa(dpsi, omega, dx, dy) - ops.arakawa(psi, domega, dx, dy)
         - phys.inv_ro * ops.beta_term(dpsi, grid)
         + phys.inv_re * ops.laplacian(domega, dx, dy) + dforcing)
    return zero_ring(d)


def step_tlm(omega, domega, forcing, dforcing, grid: Grid, level: int, phys: Physics,
             dt: float, route: str = "dst"):
    """(omega_{n+1}, d omega_{n+1}) for one step and a perturbation (domega, dforcing)."""
    wn, dwn = zero_ring(omega), zero_ring(domega)
    F = np.asarray(forcing, dtype=np.float64)
    dF = np.asarray(dforcing, dtype=np.float64)
    w, dw = wn, dwn
    for s in range(3):
        psi = cgp_psi(w, grid, level, route)
        dpsi = cgp_psi(dw, grid, level, route)
        g = rhs(w, psi, F, grid, phys)
        dg = rhs_tlm(w, psi, dw, dpsi, dF, grid, phys)
        w = zero_ring(RK3_A[s] * wn + RK3_B[s] * (w + dt * g))
        dw = zero_ring(RK3_A[s] * dwn + RK3_B[s] * (dw + dt * dg))
    return w, dw


def rhs_adjoint(omega, psi, mu, grid: Grid, level: int, phys: Physics, route: str = "dst"):
    """(dG/domega)^T mu, including the path through psi = A_l omega."""
    dx, dy = grid.dx, grid.dy
    direct = ops.transpose_apply(
        lambda f: -ops.arakawa(psi, f, dx, dy) + phys.inv_re * ops.laplacian(f, dx, dy), mu)
    via_psi = ops.transpose_apply(
        lambda f: -ops.arakawa(f, omega, dx, dy) - phys.inv_ro * ops.beta_term(f, grid), mu)
    return zero_ring(direct + cgp_psi_T(via_psi, grid, level, route))


def step_adjoint(omega, forcing, lam, grid: Grid, level: int, phys: Physics, dt: float,
                 route: str = "dst"):
    """Given the adjoint lam of omega_{n+1}, return (adjoint of omega_n, adjoint of F)."""
    _, stages = step(omega, forcing, grid, level, phys, dt, route, return_stages=True)
    lam_next = zero_ring(lam)
    acc_n = np.zeros_like(lam_next)
    gF = np.zeros_like(lam_next)
    for s in (2, 1, 0):
        w_s, psi_s = stages[s]
        mu = RK3_B[s] * dt * lam_next
        gF += mu
        acc_n += RK3_A[s] * lam_next
        lam_next = RK3_B[s] * lam_next + rhs_adjoint(w_s, psi_s, mu, grid, level, phys, route)
    return zero_ring(lam_next + acc_n), zero_ring(gF)


def misfit_loss(omega, obs_index, obs_value):
    v = omega.ravel()[obs_index]
    return float(np.mean((v - obs_value) ** 2))


def misfit_grad(omega, obs_index, obs_value):
    g = np.zeros(omega.size)
    v = omega.ravel()[obs_index]
    g[obs_index] = 2.0 * (v - obs_value) / obs_index.size
    return g.reshape(omega.shape)


def trajectory(omega0, forcing, grid: Grid, level: int, phys: Physics, dt: float,
               nsteps: int, route: str = "dst"):
    states = [zero_ring(omega0)]
    for _ in range(nsteps):
        states.append(step(states[-1], forcing, grid, level, phys, dt, route))
    return states


def loss(omega0, forcing, obs_index, obs_value, grid, level, phys, dt, nsteps, route="dst"):
    w = trajectory(omega0, forcing, grid, level, phys, dt, nsteps, route)[-1]
    return misfit_loss(w, obs_index, obs_value)


def loss_and_gradient(omega0, forcing, obs_index, obs_value, grid: Grid, level: int,
                      phys: Physics, dt: float, nsteps: int, route: str = "dst"):
    """(L, dL/domega0, dL/dF) by a full reverse sweep over stored states."""
    states = trajectory(omega0, forcing, grid, level, phys, dt, nsteps, route)
    L = misfit_loss(states[-1], obs_index, obs_value)
    lam = zero_ring(misfit_grad(states[-1], obs_index, obs_value))
    gF = np.zeros_like(lam)
    for n in range(nsteps - 1, -1, -1):
        lam, g = step_adjoint(states[n], forcing, lam, grid, level, phys, dt, route)
        gF += g
    return L, lam, gF
