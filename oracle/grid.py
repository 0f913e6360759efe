"""Node grid of the rectangular basin (oracle; test infrastructure only).

Sec. 4.4: indices i = 0..Nx, j = 0..Ny, sums over the unknowns 1..N-1; so Nx, Ny
count intervals (the text's "number of grid points" is read as intervals).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    lx: float = 1.0
    ly: float = 2.0
    y0: float = -1.0

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    @property
    def shape(self):
        return (self.ny + 1, self.nx + 1)

    def x(self) -> np.ndarray:
        return np.arange(self.nx + 1) * self.dx

    def y(self) -> np.ndarray:
        return self.y0 + np.arange(self.ny + 1) * self.dy

    def y_field(self) -> np.ndarray:
        """The coordinate y on every node (used by the beta term J(psi, y))."""
        return np.broadcast_to(self.y()[:, None], self.shape).copy()

    def coarse(self, level: int) -> "Grid":
        c = 2 ** level
        if self.nx % c or self.ny % c:
            raise ValueError("grid not divisible by 2**level")
        return Grid(self.nx // c, self.ny // c, self.lx, self.ly, self.y0)


def interior(f: np.ndarray) -> np.ndarray:
    return f[..., 1:-1, 1:-1]


def with_zero_ring(inner: np.ndarray) -> np.ndarray:
    """Embed interior values into a full node array whose ring is zero."""
    out = np.zeros(inner.shape[:-2] + (inner.shape[-2] + 2, inner.shape[-1] + 2))
    out[..., 1:-1, 1:-1] = inner
    return out
