"""Elliptic sub-problem solvers (oracle; test infrastructure only).

Sec. 4.3: with psi = 0 on the walls, transform the right-hand side with the
normalised double sine sum (2/Nx)(2/Ny) sum_i sum_j r_ij sin(pi k i/Nx)
sin(pi l j/Ny), divide by the eigenvalue of the 5-point Laplacian
alpha_kl / Ro = (2cos(pi k/Nx) - 2)/dx^2 + (2cos(pi l/Ny) - 2)/dy^2, and
synthesise psi_ij = sum_k sum_l psi_hat_kl sin(pi k i/Nx) sin(pi l j/Ny).
The two-layer coupled problem is solved per mode with the 2x2 closed form of
that section (Cramer's rule).

Vorticity form: the right-hand side is omega itself (the (delta_I/L)^-2 (q - y)
of the CGPRK3 listing), so the Ro factor of alpha is absent here and the
two-layer stretching terms enter as F1 = Fr/(Ro delta), F2 = Fr/(Ro (1-delta)).

Three independent routes reach the same unique discrete solution:
  'dense'  the sums written out as dense sine matrices (O(n^2) per line)
  'dst'    scipy.fft.dst type I (a library sine transform; dst1 = 2 * S)
  'sparse' scipy.sparse LU of the assembled 5-point matrix (no transform)
and, as an iterative black box for CGP, 'mg<N>': N multigrid V-cycles
(multigrid.py; one layer).
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse
import scipy.sparse.linalg


def sine_matrix(n: int) -> np.ndarray:
    """S[k-1, i-1] = sin(pi k i / n), k, i = 1..n-1."""
    k = np.arange(1, n)
    return np.sin(np.pi * np.outer(k, k) / n)


def eigenvalues(nx: int, ny: int, dx: float, dy: float) -> np.ndarray:
    """lambda[l-1, k-1] = (2cos(pi k/nx) - 2)/dx^2 + (2cos(pi l/ny) - 2)/dy^2.

    Evaluated as -4 sin^2(pi k/(2 nx))/dx^2 - 4 sin^2(pi l/(2 ny))/dy^2, the same
    number without the cancellation of 2cos - 2 (which costs ~2e-11 relative
    accuracy in the lowest mode at n = 1024)."""
    k = np.arange(1, nx)
    l = np.arange(1, ny)
    lx = -4.0 * np.sin(np.pi * k / (2.0 * nx)) ** 2 / (dx * dx)
    ly = -4.0 * np.sin(np.pi * l / (2.0 * ny)) ** 2 / (dy * dy)
    return ly[:, None] + lx[None, :]


def forward_transform(r: np.ndarray, route: str = "dst") -> np.ndarray:
    """hat r_kl = (2/nx)(2/ny) sum_i sum_j r_ij sin(pi k i/nx) sin(pi l j/ny).

    r is a node array (ny+1, nx+1); the result is indexed [l-1, k-1]."""
    ny, nx = r.shape[0] - 1, r.shape[1] - 1
    ri = r[1:-1, 1:-1]
    if route == "dense":
        Sx, Sy = sine_matrix(nx), sine_matrix(ny)
        return (2.0 / nx) * (2.0 / ny) * (Sy @ ri @ Sx.T)
    if route == "dst":
        return (2.0 / nx) * (2.0 / ny) * 0.25 * scipy.fft.dstn(ri, type=1)
    raise ValueError(route)


def inverse_transform(h: np.ndarray, route: str = "dst") -> np.ndarray:
    """psi_ij = sum_k sum_l h_kl sin(pi k i/nx) sin(pi l j/ny), as a node array."""
    ny, nx = h.shape[0] + 1, h.shape[1] + 1
    out = np.zeros((ny + 1, nx + 1))
    if route == "dense":
        Sx, Sy = sine_matrix(nx), sine_matrix(ny)
        out[1:-1, 1:-1] = Sy.T @ h @ Sx
    elif route == "dst":
        out[1:-1, 1:-1] = 0.25 * scipy.fft.dstn(h, type=1)
    else:
        raise ValueError(route)
    return out


def laplacian_matrix(nx: int, ny: int, dx: float, dy: float):
    """Sparse 5-point Dirichlet Laplacian on the (ny-1)(nx-1) interior unknowns (C order)."""
    ex = np.ones(nx - 1)
    ey = np.ones(ny - 1)
    Tx = scipy.sparse.diags([ex[:-1], -2 * ex, ex[:-1]], [-1, 0, 1]) / (dx * dx)
    Ty = scipy.sparse.diags([ey[:-1], -2 * ey, ey[:-1]], [-1, 0, 1]) / (dy * dy)
    return (scipy.sparse.kron(scipy.sparse.eye(ny - 1), Tx)
            + scipy.sparse.kron(Ty, scipy.sparse.eye(nx - 1))).tocsc()


def poisson(r: np.ndarray, dx: float, dy: float, route: str = "dst") -> np.ndarray:
    """psi with Delta_h psi = r at interior nodes, psi = 0 on the ring."""
    ny, nx = r.shape[0] - 1, r.shape[1] - 1
    if route.startswith("mg"):  # "mg<N>": N multigrid V-cycles (multigrid.py)
        from . import multigrid
        return multigrid.poisson_mg(r, dx, dy, int(route[2:]))
    if route == "sparse":
        A = laplacian_matrix(nx, ny, dx, dy)
        sol = scipy.sparse.linalg.splu(A).solve(r[1:-1, 1:-1].ravel())
        out = np.zeros_like(r, dtype=np.float64)
        out[1:-1, 1:-1] = sol.reshape(ny - 1, nx - 1)
        return out
    rh = forward_transform(r, route)
    lam = eigenvalues(nx, ny, dx, dy)
    return inverse_transform(rh / lam, route)


def two_layer(Q1, Q2, dx, dy, F1, F2, route: str = "dst"):
    """Solve Q1 = D psi1 + F1 (psi2 - psi1), Q2 = D psi2 + F2 (psi1 - psi2) per mode.

    Per mode (lambda the 5-point eigenvalue):
        psi1 = [(lambda - F2) Q1 - F1 Q2] / [lambda (lambda - F1 - F2)]
        psi2 = [(lambda - F1) Q2 - F2 Q1] / [lambda (lambda - F1 - F2)]
    (Sec. 4.3 closed form with alpha -> Ro*lambda, Fr/delta -> Ro*F1,
    Fr/(1-delta) -> Ro*F2; the Ro factors cancel.)"""
    ny, nx = Q1.shape[0] - 1, Q1.shape[1] - 1
    if route == "sparse":
        A = laplacian_matrix(nx, ny, dx, dy)
        n = A.shape[0]
        I = scipy.sparse.eye(n)
        M = scipy.sparse.bmat([[A - F1 * I, F1 * I], [F2 * I, A - F2 * I]]).tocsc()
        rhs = np.concatenate([Q1[1:-1, 1:-1].ravel(), Q2[1:-1, 1:-1].ravel()])
        sol = scipy.sparse.linalg.splu(M).solve(rhs)
        p1 = np.zeros_like(Q1, dtype=np.float64)
        p2 = np.zeros_like(Q2, dtype=np.float64)
        p1[1:-1, 1:-1] = sol[:n].reshape(ny - 1, nx - 1)
        p2[1:-1, 1:-1] = sol[n:].reshape(ny - 1, nx - 1)
        return p1, p2
    q1 = forward_transform(Q1, route)
    q2 = forward_transform(Q2, route)
    lam = eigenvalues(nx, ny, dx, dy)
    det = lam * (lam - F1 - F2)
    h1 = ((lam - F2) * q1 - F1 * q2) / det
    h2 = ((lam - F1) * q2 - F2 * q1) / det
    return inverse_transform(h1, route), inverse_transform(h2, route)
