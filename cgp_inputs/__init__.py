"""Seeded synthetic workloads for the coarse-grid-projection (CGP) QG time step.

This module is shared by the FP64 oracle (``oracle/``) and the HIP path
(``paper_1308_3290_amd``) so that both see byte-identical inputs.  It holds the
problem set-up only -- grids, physical coefficients, initial states, forcing
fields, observation sets -- and none of the method's arithmetic (no Jacobian,
no transfer operator, no elliptic solve, no time stepping).

Conventions (paper Sec. 2 and Sec. 4.4):
  * ``nx``, ``ny`` count grid INTERVALS; nodes are i = 0..nx, j = 0..ny.
  * Arrays are y-major with x contiguous: shape ``(ny + 1, nx + 1)`` and, for
    two layers, ``(2, ny + 1, nx + 1)``.  The boundary ring is zero.
  * The domain is x in [0, lx], y in [y0, y0 + ly]; the workloads use the
    one-layer basin [0, 1] x [-1, 1] of the paper's 1:2 grids.
  * Prognostic variable: relative vorticity omega = (q - y) / Ro (one layer),
    Q_i = (q_i - y) / Ro (two layers); the coefficients below are those of the
    vorticity form obtained by dividing the nondimensional equations of
    Sec. 2.1 / 2.2 by Ro.

Input recipe (numpy PCG64 ``default_rng(seed)``):
  * initial field: 1e-3 * N(0, 1) drawn over the interior, C order, zero ring;
  * forcing: amp * sin(pi * y_j) on every node (the ring is ignored by the
    step), amp = 1/Ro unless the ensemble perturbs it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Case", "make_case", "case_c0", "case_c1", "case_c2", "ensemble_c3", "experiment_case",
    "adjoint_c4", "node_y", "forcing_field", "initial_field", "AdjointProblem",
    "EnsembleMember",
]

# Single-layer physics shared by the one-layer workloads: Re = 450, Ro = 0.0036
# (Munk scale 0.02, Rhines scale 0.06, Re_B = 27; Sec. 2.1 relations).
RE_1L = 450.0
RO_1L = 0.0036


@dataclasses.dataclass
class Case:
    """One basin: grid, coarsening level and vorticity-form coefficients."""
    nx: int
    ny: int
    level: int = 0
    nlayers: int = 1
    lx: float = 1.0
    ly: float = 2.0
    y0: float = -1.0
    inv_re: float = 1.0 / RE_1L
    inv_ro: float = 1.0 / RO_1L
    f1: float = 0.0
    f2: float = 0.0
    drag: float = 0.0
    dt: float = 1e-4
    cfl: float = 0.0      # CFL number of the adaptive step (Sec. 4.2); 0: fixed dt
    solver: int = 0       # coarse solver: 0 sine transform, 1 multigrid V-cycles
    mg_cycles: int = 0    # V-cycles per solve (0: the library default)
    nsteps: int = 1
    seed: int = 0
    dtype: str = "f64"
    name: str = ""

    @property
    def shape(self):
        if self.nlayers == 1:
            return (self.ny + 1, self.nx + 1)
        return (self.nlayers, self.ny + 1, self.nx + 1)

    @property
    def points(self) -> int:
        """Resolution-label point count nx * ny * layers (metric unit)."""
        return self.nx * self.ny * self.nlayers

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    def np_dtype(self):
        return np.float64 if self.dtype == "f64" else np.float32


def make_case(nx, ny, **kw) -> Case:
    return Case(nx=nx, ny=ny, **kw)


def node_y(case: Case) -> np.ndarray:
    """y coordinate of node rows j = 0..ny."""
    return case.y0 + np.arange(case.ny + 1, dtype=np.float64) * (case.ly / case.ny)


def forcing_field(case: Case, amplitude: Optional[float] = None) -> np.ndarray:
    """Double-gyre wind forcing amp * sin(pi * y) on every node (Sec. 2.1)."""
    amp = case.inv_ro if amplitude is None else amplitude
    col = amp * np.sin(np.pi * node_y(case))
    return np.ascontiguousarray(np.broadcast_to(col[:, None], (case.ny + 1, case.nx + 1)),
                                dtype=np.float64)


def initial_field(case: Case, rng: np.random.Generator, scale: float = 1e-3,
                  layers: Optional[int] = None) -> np.ndarray:
    """scale * N(0,1) over the interior (C order, layer 1 first), zero ring."""
    L = case.nlayers if layers is None else layers
    out = np.zeros((L, case.ny + 1, case.nx + 1), dtype=np.float64)
    for l in range(L):
        out[l, 1:-1, 1:-1] = scale * rng.standard_normal((case.ny - 1, case.nx - 1))
    return out[0] if (layers is None and case.nlayers == 1) else out


# --------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------
def case_c0() -> Case:
    """Single layer, 64 x 128, full grid (level 0), FP64, dt 1e-4, 100 steps."""
    return Case(nx=64, ny=128, level=0, dt=1e-4, nsteps=100, seed=0, name="c0")


def case_c1(level: int = 1) -> Case:
    """Single layer, 512 x 1024, CGP factor 2**level, FP64, dt 2.5e-5, 1000 steps."""
    return Case(nx=512, ny=1024, level=level, dt=2.5e-5, nsteps=1000, seed=0,
                name=f"c1_l{level}")


# Two-layer stratification: deformation radius 0.02 (F1 + F2 = 1 / Rd^2), depth
# ratio H1/H2 = 0.2 read literally (delta = H1/H = 1/6, F1 = (F1+F2)(1-delta),
# F2 = (F1+F2) delta), bottom drag sigma = 1e-2 entering the vorticity form as
# sigma / Ro.
RD_2L = 0.02
H1_OVER_H2 = 0.2
SIGMA_2L = 1e-2


def two_layer_coefficients(ro=RO_1L, rd=RD_2L, h1_over_h2=H1_OVER_H2, sigma=SIGMA_2L):
    delta = h1_over_h2 / (1.0 + h1_over_h2)
    fsum = 1.0 / (rd * rd)
    return dict(f1=fsum * (1.0 - delta), f2=fsum * delta, drag=sigma / ro, delta=delta)


def case_c2(level: int = 1) -> Case:
    """Two layers, 512 x 1024 per layer, CGP factor 2**level, FP64, 500 steps."""
    c = two_layer_coefficients()
    return Case(nx=512, ny=1024, level=level, nlayers=2, f1=c["f1"], f2=c["f2"],
                drag=c["drag"], dt=2.5e-5, nsteps=500, seed=2, name=f"c2_l{level}")


@dataclasses.dataclass
class EnsembleMember:
    case: Case
    amplitude: float
    omega0: np.ndarray
    forcing: np.ndarray


ENSEMBLE_SIZES = [(128, 256), (256, 512), (384, 768), (512, 1024)]


def ensemble_c3(count: int = 64, dtype: str = "f64", nsteps: int = 200,
                sizes=None, seed: int = 3) -> List[EnsembleMember]:
    """Heterogeneous ensemble: sizes ~ U{sizes}, amplitude (1/Ro)(1 + 0.1 N(0,1)),
    Re ~ U[200, 800], level 1.  Draw order: sizes, amplitudes, Re, then omega0."""
    sizes = ENSEMBLE_SIZES if sizes is None else sizes
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(sizes), size=count)
    amps = (1.0 / RO_1L) * (1.0 + 0.1 * rng.standard_normal(count))
    res = rng.uniform(200.0, 800.0, size=count)
    out = []
    for m in range(count):
        nx, ny = sizes[int(pick[m])]
        c = Case(nx=nx, ny=ny, level=1, inv_re=1.0 / res[m], dt=2.5e-5, nsteps=nsteps,
                 seed=seed, dtype=dtype, name=f"c3_m{m}")
        w0 = initial_field(c, rng)
        out.append(EnsembleMember(case=c, amplitude=float(amps[m]), omega0=w0,
                                  forcing=forcing_field(c, float(amps[m]))))
    return out


# The one-layer experiments of Sec. 5.1 (Table 1): Exp. I Re = 200,
# Ro = 0.0016; Exp. II Re = 312.5, Ro = 0.0025; forcing sin(pi y)/Ro on the
# [0, 1] x [-1, 1] basin, started from 1e-3 N(0,1) noise, adaptive steps.
EXPERIMENTS_1L = {"I": dict(ro=0.0016, re=200.0), "II": dict(ro=0.0025, re=312.5)}


def experiment_case(exp: str, nx: int, ny: int, level: int, seed: int = 1, cfl: float = 0.5,
                    dt_max: float = 5e-4, dtype: str = "f64"):
    """(Case, omega0, forcing) of one long run of experiment `exp` on an
    nx x ny grid with CGP level `level`."""
    p = EXPERIMENTS_1L[exp]
    c = Case(nx=nx, ny=ny, level=level, inv_re=1.0 / p["re"], inv_ro=1.0 / p["ro"], dt=dt_max,
             cfl=cfl, seed=seed, dtype=dtype, name=f"exp{exp}_{nx}x{ny}_l{level}")
    w0 = initial_field(c, np.random.default_rng(seed))
    return c, w0, forcing_field(c)


@dataclasses.dataclass
class AdjointProblem:
    case: Case
    omega0: np.ndarray
    forcing: np.ndarray
    obs_index: np.ndarray      # flat node indices (j * (nx + 1) + i), interior, distinct
    obs_value: np.ndarray
    dir_forcing: np.ndarray    # (ndir, ny+1, nx+1), zero ring, unit norm jointly with dir_omega
    dir_omega: np.ndarray
    ckpt_every: int


def adjoint_c4(nx: int = 256, ny: int = 512, nsteps: int = 200, ckpt_every: int = 20,
               ndir: int = 20, level: int = 1, obs_fraction: float = 0.01,
               seed: int = 4) -> AdjointProblem:
    """Adjoint workload: final-step misfit of omega at 1% of interior points."""
    c = Case(nx=nx, ny=ny, level=level, dt=2.5e-5, nsteps=nsteps, seed=seed, name="c4")
    rng = np.random.default_rng(seed)
    w0 = initial_field(c, rng)
    F = forcing_field(c)
    n_int = (nx - 1) * (ny - 1)
    K = int(round(obs_fraction * n_int))
    flat_int = rng.choice(n_int, size=K, replace=False)
    jj = 1 + flat_int // (nx - 1)
    ii = 1 + flat_int % (nx - 1)
    obs_index = (jj * (nx + 1) + ii).astype(np.int64)
    obs_value = rng.standard_normal(K)
    dF = np.zeros((ndir, ny + 1, nx + 1))
    dW = np.zeros((ndir, ny + 1, nx + 1))
    for d in range(ndir):
        dF[d, 1:-1, 1:-1] = rng.standard_normal((ny - 1, nx - 1))
        dW[d, 1:-1, 1:-1] = rng.standard_normal((ny - 1, nx - 1))
        nrm = math.sqrt(float(np.sum(dF[d] ** 2) + np.sum(dW[d] ** 2)))
        dF[d] /= nrm
        dW[d] /= nrm
    return AdjointProblem(case=c, omega0=w0, forcing=F, obs_index=obs_index,
                          obs_value=obs_value, dir_forcing=dF, dir_omega=dW,
                          ckpt_every=ckpt_every)
