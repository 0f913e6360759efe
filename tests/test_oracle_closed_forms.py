"""Closed-form pins of the oracle's diagnostics, two-layer coupling and parameters.

Each test fixes a result by exact mathematics or by the paper's physical
inputs, on grids with dx != dy and with F1 != F2, so that a swapped spacing, a
dropped area, Q_i in place of zeta_i, or F1 and F2 exchanged fails here:

- enstrophy of a discrete sine mode (interior sum of sin^2 sin^2 = (N/2)(M/2));
- energy (eq. 26) of a discrete sine mode, and its summation-by-parts identity;
- one CGPRK3 step of the two-layer model (Sec. 2.2) on a single sine mode,
  where every Jacobian vanishes and the step is the RK3 polynomial of a 2x2
  per-mode matrix built from zeta_i = lambda psi_i and the Sec. 4.3 2x2 solve;
- the stretching coefficients of Table 2's experiments from their dimensional
  inputs: F_i = f0^2 L^2 / (g' H_i), layer 1 on top (Sec. 2.2).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import diagnostics, model, operators as ops, params
from oracle.grid import Grid
from oracle.model import Physics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# dx = 1/16, dy = 3/24 = 1/8 (and lx = 2, ly = 3 for the energy/enstrophy grids)
SKEW_GRIDS = [Grid(16, 24, lx=1.0, ly=3.0, y0=-1.5), Grid(24, 20, lx=2.0, ly=3.0, y0=0.0)]


def _mode(g, k, l):
    I, J = np.meshgrid(np.arange(g.nx + 1), np.arange(g.ny + 1))
    return np.sin(np.pi * k * I / g.nx) * np.sin(np.pi * l * J / g.ny)


def _eig(g, k, l):
    """Eigenvalue of the 5-point Laplacian on sin(pi k i/nx) sin(pi l j/ny), from the
    second difference of a sine: -4 sin^2(pi k/(2nx))/dx^2 - 4 sin^2(pi l/(2ny))/dy^2."""
    return (-4.0 * math.sin(math.pi * k / (2 * g.nx)) ** 2 / g.dx ** 2
            - 4.0 * math.sin(math.pi * l / (2 * g.ny)) ** 2 / g.dy ** 2)


# ------------------------------------------------------------------ enstrophy
@pytest.mark.parametrize("g", SKEW_GRIDS)
@pytest.mark.parametrize("k,l,amp", [(1, 1, 1.0), (3, 5, 2.5), (7, 2, -0.3)])
def test_enstrophy_of_a_sine_mode(g, k, l, amp):
    """Z = 1/(2A) sum omega^2 dx dy with omega = amp sin sin: the interior sum of
    sin^2(pi k i/N) sin^2(pi l j/M) is (N/2)(M/2) for 0 < k < N, 0 < l < M, and
    dx dy N M = A, so Z = amp^2 / 8 on every grid."""
    Z = diagnostics.enstrophy(amp * _mode(g, k, l), g)
    assert abs(Z - amp * amp / 8.0) < 1e-14 * amp * amp


def test_enstrophy_is_quadratic_and_interior_only():
    g = SKEW_GRIDS[0]
    rng = np.random.default_rng(7)
    w = rng.standard_normal(g.shape)
    inner = w.copy()
    inner[0, :] = inner[-1, :] = inner[:, 0] = inner[:, -1] = 0.0
    assert diagnostics.enstrophy(w, g) == diagnostics.enstrophy(inner, g)
    assert abs(diagnostics.enstrophy(3.0 * inner, g) - 9.0 * diagnostics.enstrophy(inner, g)) \
        < 1e-13 * diagnostics.enstrophy(inner, g)


# ------------------------------------------------------------------ energy (eq. 26)
@pytest.mark.parametrize("g", SKEW_GRIDS)
@pytest.mark.parametrize("k,l", [(1, 1), (2, 5), (5, 3)])
def test_energy_of_a_sine_mode(g, k, l):
    """Summation by parts turns the link sum of squared forward differences into
    -sum psi Lap_h psi; on a sine mode that is -lambda (N/2)(M/2), so
    E = -lambda / 8 with lambda = -(2 sin(pi k/2N)/dx)^2 - (2 sin(pi l/2M)/dy)^2.
    With dx != dy the x and y spacings enter with different weights."""
    amp = 1.7
    E = diagnostics.energy(amp * _mode(g, k, l), g)
    ref = -amp * amp * _eig(g, k, l) / 8.0
    assert abs(E - ref) < 1e-13 * ref


@pytest.mark.parametrize("g", SKEW_GRIDS)
def test_energy_identity_on_a_skew_grid(g):
    rng = np.random.default_rng(31)
    psi = np.zeros(g.shape)
    psi[1:-1, 1:-1] = rng.standard_normal((g.ny - 1, g.nx - 1))
    E = diagnostics.energy(psi, g)
    ref = -g.dx * g.dy / (2 * g.lx * g.ly) * np.sum(psi * ops.laplacian(psi, g.dx, g.dy))
    assert abs(E - ref) < 1e-12 * abs(ref)


# ------------------------------------------------------------------ two layers, zeta_i
def _two_layer_mode_matrix(g, k, l, phys):
    lam = _eig(g, k, l)
    M = np.array([[lam - phys.f1, phys.f1], [phys.f2, lam - phys.f2]])
    D = np.diag([phys.inv_re * lam, phys.inv_re * lam - phys.drag])
    return lam * D @ np.linalg.inv(M)


def _two_layer_mode_step(g, k, l, phys, dt, c1, c2):
    """Exact one-step result for Q_i = c_i * phi (phi the (k, l) sine mode), no beta,
    no forcing, l = 0.

    The coupled solve of Sec. 4.3 is exact per mode: psi = M^-1 Q with
    M = [[lam - F1, F1], [F2, lam - F2]] (Q_1 = lam psi_1 + F1 (psi_2 - psi_1), ...).
    Every psi_i and Q_i is a multiple of phi, so J(psi_i, Q_i) = 0, and
    zeta_i = Q_i - F_i (psi_j - psi_i) = lam psi_i.  The right-hand side is then
    dQ_i/dt = inv_re Lap(zeta_i) - [i=2] drag zeta_2 = D_i lam psi_i with
    D = diag(inv_re lam, inv_re lam - drag), i.e. dQ/dt = K Q, K = lam D M^-1,
    and TVD-RK3 (Sec. 4.2) applies I + z + z^2/2 + z^3/6 with z = dt K."""
    z = dt * _two_layer_mode_matrix(g, k, l, phys)
    P = np.eye(2) + z + z @ z / 2.0 + z @ z @ z / 6.0
    return P @ np.array([c1, c2])


@pytest.mark.parametrize("k,l", [(1, 1), (3, 2)])
def test_two_layer_step_on_a_sine_mode(k, l):
    """Pins zeta_i (not Q_i) in the viscous and the drag terms, and which layer
    carries F1 and which F2: F1 != F2, drag != 0, coupling comparable to lam."""
    g = Grid(16, 24, lx=1.0, ly=3.0, y0=-1.5)
    lam = _eig(g, k, l)
    phys = Physics(inv_re=0.02, inv_ro=0.0, f1=3.0 * abs(lam), f2=0.4 * abs(lam), drag=5.0)
    c1, c2 = 1.3, -0.6
    phi = _mode(g, k, l)
    Q = np.stack([c1 * phi, c2 * phi])
    # scale dt so that |z| ~ 0.4: every term of the RK3 polynomial matters
    dt = 0.4 / np.linalg.norm(_two_layer_mode_matrix(g, k, l, phys), 2)
    out = model.step_two_layer(Q, np.zeros(g.shape), g, 0, phys, dt)
    a = _two_layer_mode_step(g, k, l, phys, dt, c1, c2)
    scale = max(abs(c1), abs(c2))
    assert np.max(np.abs(out[0] - a[0] * phi)) < 1e-12 * scale
    assert np.max(np.abs(out[1] - a[1] * phi)) < 1e-12 * scale
    # the result moved well away from the Q-based and the swapped-F alternatives
    assert np.max(np.abs(a - np.array([c1, c2]))) > 0.05 * scale


def test_two_layer_mode_step_alternatives_differ():
    """The closed form above separates the readings it rules out: Q_i in the
    viscous term, Q_2 in the drag term, F1 and F2 exchanged."""
    g = Grid(16, 24, lx=1.0, ly=3.0, y0=-1.5)
    k, l = 1, 1
    lam = _eig(g, k, l)
    phys = Physics(inv_re=0.02, inv_ro=0.0, f1=3.0 * abs(lam), f2=0.4 * abs(lam), drag=5.0)
    dt = 0.4 / np.linalg.norm(_two_layer_mode_matrix(g, k, l, phys), 2)
    good = _two_layer_mode_step(g, k, l, phys, dt, 1.3, -0.6)
    swapped = _two_layer_mode_step(g, k, l, Physics(phys.inv_re, 0.0, phys.f2, phys.f1, phys.drag),
                                   dt, 1.3, -0.6)
    assert np.max(np.abs(good - swapped)) > 1e-2
    # Q-based viscosity and drag: dQ/dt = diag(inv_re lam, inv_re lam - drag) Q
    zq = dt * np.diag([phys.inv_re * lam, phys.inv_re * lam - phys.drag])
    qform = (np.eye(2) + zq + zq @ zq / 2 + zq @ zq @ zq / 6) @ np.array([1.3, -0.6])
    assert np.max(np.abs(good - qform)) > 1e-2


# ------------------------------------------------------------------ F1 : F2 (Table 2)
def test_stretching_coefficients_from_layer_depths():
    """F_i = f0^2 L^2 / (g' H_i): each layer's stretching coefficient follows from
    its own depth (the two-layer QG potential vorticity, Sec. 2.2, with lengths
    scaled by L); layer 1 is the top layer of depth H1.  So F1 / F2 = H2 / H1 =
    (1 - delta) / delta, computed here from the dimensional inputs of Table 2."""
    t = json.load(open(os.path.join(GOLDEN, "table2_two_layer.json")))
    for name, e in t["inputs"].items():
        L, H1, H2 = e["L_km"] * 1e3, e["H1_km"] * 1e3, e["H2_km"] * 1e3
        p = params.two_layer(L, H1, H2, e["f0"], e["beta"], e["rho1"], e["gprime"],
                             e["tau0"], e["gamma"], e["nu"])
        F1 = e["f0"] ** 2 * L ** 2 / (e["gprime"] * H1)
        F2 = e["f0"] ** 2 * L ** 2 / (e["gprime"] * H2)
        assert math.isclose(p["f1"], F1, rel_tol=1e-12)
        assert math.isclose(p["f2"], F2, rel_tol=1e-12)
        assert math.isclose(p["f1"] / p["f2"], H2 / H1, rel_tol=1e-12)
        assert H1 != H2  # the experiments distinguish the layers
