"""Grid-transfer operators (oracle; test infrastructure only).

Sec. 3.1: full-weighting restriction (the 1/16 [4 centre, 2 edges, 1 corners]
nine-point average evaluated at coarse nodes (2I, 2J)) and bilinear
prolongation (the four injection/averaging formulas).  Several coarsening
levels are obtained by applying the half mappings repeatedly, as that section
states.

Restriction is evaluated at coarse INTERIOR nodes only; the coarse ring is the
homogeneous Dirichlet value 0.  Prolongation fills every fine node from the
coarse node array (whose ring is 0), so the fine ring comes out 0.

The transposes are written as the literal adjoint (scatter) of each formula.
"""
from __future__ import annotations

import numpy as np


def restrict_fw(f: np.ndarray) -> np.ndarray:
    """One full-weighting restriction of a node array (ny+1, nx+1) -> (ny/2+1, nx/2+1)."""
    ny, nx = f.shape[0] - 1, f.shape[1] - 1
    if nx % 2 or ny % 2:
        raise ValueError("restriction needs even interval counts")
    My, Mx = ny // 2, nx // 2
    out = np.zeros((My + 1, Mx + 1))
    J = np.arange(1, My)[:, None]
    I = np.arange(1, Mx)[None, :]
    c = lambda di, dj: f[2 * J + dj, 2 * I + di]  # noqa: E731
    out[1:My, 1:Mx] = (4.0 * c(0, 0)
                       + 2.0 * (c(0, -1) + c(0, 1) + c(-1, 0) + c(1, 0))
                       + c(1, 1) + c(1, -1) + c(-1, 1) + c(-1, -1)) / 16.0
    return out


def prolong_bilinear(g: np.ndarray) -> np.ndarray:
    """One bilinear prolongation of a node array (My+1, Mx+1) -> (2My+1, 2Mx+1)."""
    My, Mx = g.shape[0] - 1, g.shape[1] - 1
    out = np.zeros((2 * My + 1, 2 * Mx + 1))
    # phi_{2i,2j} = bar phi_{i,j}
    out[0::2, 0::2] = g
    # phi_{2i+1,2j} = (bar phi_{i,j} + bar phi_{i+1,j}) / 2   (i along x)
    out[0::2, 1::2] = 0.5 * (g[:, :-1] + g[:, 1:])
    # phi_{2i,2j+1} = (bar phi_{i,j} + bar phi_{i,j+1}) / 2
    out[1::2, 0::2] = 0.5 * (g[:-1, :] + g[1:, :])
    # phi_{2i+1,2j+1} = average of the four surrounding coarse values
    out[1::2, 1::2] = 0.25 * (g[:-1, :-1] + g[:-1, 1:] + g[1:, :-1] + g[1:, 1:])
    return out


def restrict(f: np.ndarray, level: int) -> np.ndarray:
    for _ in range(level):
        f = restrict_fw(f)
    return f


def prolong(g: np.ndarray, level: int) -> np.ndarray:
    for _ in range(level):
        g = prolong_bilinear(g)
    return g


# ---------------------------------------------------------------------------
# Literal transposes (adjoints in the plain sum inner product).
# ---------------------------------------------------------------------------
def restrict_fw_T(g: np.ndarray) -> np.ndarray:
    """Transpose of restrict_fw: scatter each coarse interior value back with its weights."""
    My, Mx = g.shape[0] - 1, g.shape[1] - 1
    out = np.zeros((2 * My + 1, 2 * Mx + 1))
    gi = g[1:My, 1:Mx]
    w = {(0, 0): 4.0, (0, -1): 2.0, (0, 1): 2.0, (-1, 0): 2.0, (1, 0): 2.0,
         (1, 1): 1.0, (1, -1): 1.0, (-1, 1): 1.0, (-1, -1): 1.0}
    for (di, dj), wt in w.items():
        out[2 + dj: 2 * My - 1 + dj: 2, 2 + di: 2 * Mx - 1 + di: 2] += (wt / 16.0) * gi
    return out


def prolong_bilinear_T(f: np.ndarray) -> np.ndarray:
    """Transpose of prolong_bilinear: gather each fine value back to its coarse sources."""
    ny, nx = f.shape[0] - 1, f.shape[1] - 1
    My, Mx = ny // 2, nx // 2
    out = np.zeros((My + 1, Mx + 1))
    out += f[0::2, 0::2]
    e = 0.5 * f[0::2, 1::2]
    out[:, :-1] += e
    out[:, 1:] += e
    n = 0.5 * f[1::2, 0::2]
    out[:-1, :] += n
    out[1:, :] += n
    c = 0.25 * f[1::2, 1::2]
    out[:-1, :-1] += c
    out[:-1, 1:] += c
    out[1:, :-1] += c
    out[1:, 1:] += c
    return out


def restrict_T(g: np.ndarray, level: int) -> np.ndarray:
    for _ in range(level):
        g = restrict_fw_T(g)
    return g


def prolong_T(f: np.ndarray, level: int) -> np.ndarray:
    for _ in range(level):
        f = prolong_bilinear_T(f)
    return f
