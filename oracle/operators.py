"""Spatial operators at interior nodes (oracle; test infrastructure only).

Arakawa Jacobian (Sec. 4.1): J = (J1 + J2 + J3)/3 with J1, J2, J3 the three
second-order forms written out in that section, each carrying 1/(4 dx dy).
Laplacian: standard 5-point form.  Beta term: J(psi, y), the Jacobian of psi
with the coordinate y (the beta*y part of q = omega + beta*y in eq. 2; the
vorticity form keeps it apart from J(psi, omega)).

All outputs are full node arrays with a zero ring.  The transpose helpers
compute exact transposes of any 9-point linear interior operator by probing it
with the nine mod-3 indicator fields and scattering the extracted stencil
coefficients; they rely on no identity of the operator.
"""
from __future__ import annotations

import numpy as np


def _s(f: np.ndarray, di: int, dj: int) -> np.ndarray:
    """f[j + dj, i + di] over the interior nodes (1..ny-1, 1..nx-1)."""
    ny1, nx1 = f.shape
    return f[1 + dj: ny1 - 1 + dj, 1 + di: nx1 - 1 + di]


def _full(inner: np.ndarray) -> np.ndarray:
    out = np.zeros((inner.shape[0] + 2, inner.shape[1] + 2))
    out[1:-1, 1:-1] = inner
    return out


def jacobian_j1(p, q, dx, dy):
    """J1: central second-order form (Sec. 4.1)."""
    b = (-(_s(q, 1, 0) - _s(q, -1, 0)) * (_s(p, 0, 1) - _s(p, 0, -1))
         + (_s(q, 0, 1) - _s(q, 0, -1)) * (_s(p, 1, 0) - _s(p, -1, 0)))
    return _full(b / (4.0 * dx * dy))


def jacobian_j2(p, q, dx, dy):
    """J2: the form with q at the four edge neighbours (Sec. 4.1)."""
    b = (-_s(q, 1, 0) * (_s(p, 1, 1) - _s(p, 1, -1))
         + _s(q, -1, 0) * (_s(p, -1, 1) - _s(p, -1, -1))
         + _s(q, 0, 1) * (_s(p, 1, 1) - _s(p, -1, 1))
         - _s(q, 0, -1) * (_s(p, 1, -1) - _s(p, -1, -1)))
    return _full(b / (4.0 * dx * dy))


def jacobian_j3(p, q, dx, dy):
    """J3: the form with q at the four corners (Sec. 4.1)."""
    b = (-_s(q, 1, 1) * (_s(p, 0, 1) - _s(p, 1, 0))
         + _s(q, -1, -1) * (_s(p, -1, 0) - _s(p, 0, -1))
         + _s(q, -1, 1) * (_s(p, 0, 1) - _s(p, -1, 0))
         - _s(q, 1, -1) * (_s(p, 1, 0) - _s(p, 0, -1)))
    return _full(b / (4.0 * dx * dy))


def arakawa(p, q, dx, dy):
    """J_A(p, q) = (J1 + J2 + J3) / 3 (Sec. 4.1), zero on the ring."""
    return (jacobian_j1(p, q, dx, dy) + jacobian_j2(p, q, dx, dy)
            + jacobian_j3(p, q, dx, dy)) / 3.0


def laplacian(f, dx, dy):
    """5-point discrete Laplacian at interior nodes, zero on the ring."""
    b = ((_s(f, 1, 0) - 2.0 * _s(f, 0, 0) + _s(f, -1, 0)) / (dx * dx)
         + (_s(f, 0, 1) - 2.0 * _s(f, 0, 0) + _s(f, 0, -1)) / (dy * dy))
    return _full(b)


def beta_term(psi, grid):
    """J_A(psi, y): the planetary-vorticity advection in vorticity form."""
    return arakawa(psi, grid.y_field(), grid.dx, grid.dy)


def continuous_jacobian_fd(p, q, dx, dy):
    """Plain central-difference evaluation of p_x q_y - p_y q_x (eq. 6), for tests."""
    px = (_s(p, 1, 0) - _s(p, -1, 0)) / (2 * dx)
    py = (_s(p, 0, 1) - _s(p, 0, -1)) / (2 * dy)
    qx = (_s(q, 1, 0) - _s(q, -1, 0)) / (2 * dx)
    qy = (_s(q, 0, 1) - _s(q, 0, -1)) / (2 * dy)
    return _full(px * qy - py * qx)


# ---------------------------------------------------------------------------
# Exact transposes of 9-point interior operators.
# ---------------------------------------------------------------------------
_OFFSETS = [(di, dj) for dj in (-1, 0, 1) for di in (-1, 0, 1)]


def stencil_coefficients(apply, shape):
    """Coefficients c[(di,dj)][j,i] with apply(f)[j,i] = sum c * f[j+dj, i+di].

    ``apply`` must be linear, act on full node arrays and read only the 3x3
    neighbourhood.  Probing with the indicator of nodes with (i mod 3, j mod 3)
    = (a, b) isolates, at each output node, the single neighbour in that class.
    """
    ny1, nx1 = shape
    J, I = np.meshgrid(np.arange(ny1), np.arange(nx1), indexing="ij")
    coef = {o: np.zeros((ny1 - 2, nx1 - 2)) for o in _OFFSETS}
    Jin, Iin = J[1:-1, 1:-1], I[1:-1, 1:-1]
    for a in range(3):
        for b in range(3):
            probe = ((I % 3 == a) & (J % 3 == b)).astype(np.float64)
            val = apply(probe)[1:-1, 1:-1]
            for (di, dj) in _OFFSETS:
                hit = ((Iin + di) % 3 == a) & ((Jin + dj) % 3 == b)
                coef[(di, dj)][hit] = val[hit]
    return coef


def transpose_apply(apply, mu, shape=None):
    """(apply)^T mu restricted to the interior (ring of the result is 0)."""
    shape = mu.shape if shape is None else shape
    coef = stencil_coefficients(apply, shape)
    ny1, nx1 = shape
    out = np.zeros(shape)
    m = mu[1:-1, 1:-1]
    for (di, dj), c in coef.items():
        out[1 + dj: ny1 - 1 + dj, 1 + di: nx1 - 1 + di] += c * m
    out[0, :] = 0.0
    out[-1, :] = 0.0
    out[:, 0] = 0.0
    out[:, -1] = 0.0
    return out
