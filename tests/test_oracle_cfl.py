"""Pins of the oracle's adaptive CFL step size (Sec. 4.2)."""
import math

import numpy as np
import pytest

import cgp_inputs as ci
from oracle import cfl, model
from oracle.grid import Grid
from oracle.model import Physics


def test_linear_field_gives_its_slopes():
    # centred differences are exact on affine fields; dx != dy
    g = Grid(16, 8, lx=1.0, ly=2.0, y0=-1.0)
    X, Y = np.meshgrid(g.x(), g.y())
    for a, b in ((3.0, -5.0), (7.0, 2.0), (-0.5, 0.25)):
        psi = a * X + b * Y
        assert cfl.max_velocity(psi, g) == pytest.approx(max(abs(a), abs(b)), rel=1e-13)
        assert cfl.cfl_dt(psi, g, 0.5, 1.0) == pytest.approx(
            0.5 * min(g.dx, g.dy) / max(abs(a), abs(b)), rel=1e-13)


def test_quadratic_fields_and_interior_nodes_only():
    # centred differences are exact on quadratics: psi = x^2 -> 2x, largest at
    # the last interior column; psi = y^2 -> 2y, largest in magnitude at an
    # interior row next to a wall
    g = Grid(20, 12, lx=1.0, ly=2.0, y0=-1.0)
    X, Y = np.meshgrid(g.x(), g.y())
    assert cfl.max_velocity(X ** 2, g) == pytest.approx(2 * (1 - g.dx), rel=1e-13)
    y = g.y()[1:-1]
    assert cfl.max_velocity(Y ** 2, g) == pytest.approx(np.abs(2 * y).max(), rel=1e-13)


def test_sine_field_closed_form():
    # (sin(k(x+h)) - sin(k(x-h))) / 2h = cos(kx) sin(kh)/h; with k = pi on
    # [0, 1] the largest |cos| at an interior node is cos(pi dx)
    g = Grid(32, 16, lx=1.0, ly=2.0, y0=-1.0)
    X, _ = np.meshgrid(g.x(), g.y())
    psi = np.sin(np.pi * X)
    h = g.dx
    expect = math.cos(math.pi * h) * math.sin(math.pi * h) / h
    assert cfl.max_velocity(psi, g) == pytest.approx(expect, rel=1e-13)
    # a forward difference would give a different number
    assert abs(expect - (math.sin(math.pi * h) / h)) > 1e-3


def test_brute_force_on_a_tiny_grid_and_two_layers():
    g = Grid(6, 5, lx=1.5, ly=1.0, y0=0.0)
    rng = np.random.default_rng(7)
    psi = rng.standard_normal((2, 6, 7))
    best = 0.0
    for l in range(2):
        for j in range(1, 5):
            for i in range(1, 6):
                best = max(best, abs(psi[l, j, i + 1] - psi[l, j, i - 1]) / (2 * g.dx),
                           abs(psi[l, j + 1, i] - psi[l, j - 1, i]) / (2 * g.dy))
    assert cfl.max_velocity(psi, g) == best
    # the larger layer decides
    assert cfl.max_velocity(psi[0], g) <= best and cfl.max_velocity(psi[1], g) <= best
    assert max(cfl.max_velocity(psi[0], g), cfl.max_velocity(psi[1], g)) == best


def test_cap_and_zero_state():
    g = Grid(8, 8)
    assert cfl.cfl_dt(np.zeros((9, 9)), g, 0.8, 2e-4) == 2e-4
    X, _ = np.meshgrid(g.x(), g.y())
    assert cfl.cfl_dt(1e-9 * X, g, 0.8, 2e-4) == 2e-4      # CFL bound far above the cap
    assert cfl.cfl_dt(1e9 * X, g, 0.8, 2e-4) == pytest.approx(0.8 * g.dx / 1e9, rel=1e-13)


def _small(nx=32, ny=64, level=1):
    case = ci.make_case(nx, ny, dt=1e-4)
    g = Grid(nx, ny)
    phys = Physics(inv_re=case.inv_re, inv_ro=case.inv_ro)
    w0 = ci.initial_field(case, np.random.default_rng(0))
    F = ci.forcing_field(case)
    return g, phys, w0, F, level


def test_huge_cfl_reduces_to_the_fixed_step():
    g, phys, w0, F, level = _small()
    wa, dts = cfl.run_adaptive(w0, F, g, level, phys, cfl=1e30, dt_max=1e-4, nsteps=5)
    wf = model.run(w0, F, g, level, phys, 1e-4, 5)
    assert dts == [1e-4] * 5
    assert np.array_equal(wa, wf)


def test_adaptive_steps_follow_the_third_stage_psi():
    # first step at dt_max; every later step at c min(dx, dy) / max|grad psi|
    # of the previous step's third-stage psi (capped at dt_max)
    g, phys, w0, F, level = _small()
    c, dt_max = 0.002, 1e-3
    states = []
    wa, dts = cfl.run_adaptive(w0, F, g, level, phys, cfl=c, dt_max=dt_max, nsteps=6,
                               callback=lambda n, w, dt: states.append(w))
    assert dts[0] == dt_max
    w = np.array(w0, dtype=np.float64)
    for n in range(6):
        w_next, stages = model.step(w, F, g, level, phys, dts[n], return_stages=True)
        assert np.array_equal(w_next, states[n])
        if n + 1 < 6:
            m = cfl.max_velocity(stages[2][1], g)
            assert dts[n + 1] == min(dt_max, c * min(g.dx, g.dy) / m)
        w = w_next
    # the steps really adapt (the cap binds only at the start of the spin-up)
    assert len(set(dts[1:])) > 3 and min(dts) < 0.5 * dt_max


# ------------------------------------------------------------------ time means (Sec. 5.1)
def test_time_mean_of_psi_is_the_mean_of_the_per_step_psi():
    # brute force: average A(omega_n) step by step; the oracle maps the mean
    # of omega once (A is linear)
    from oracle import statistics
    g, phys, w0, F, level = _small()
    c, dt_max = 0.002, 1e-3
    mean_w, mean_psi, tsum, _ = statistics.time_mean(w0, F, g, level, phys, c, dt_max, 3, 5)
    acc_w = np.zeros_like(w0)
    acc_p = np.zeros_like(w0)
    t = 0.0

    def cb(n, w, dt):
        nonlocal t
        if n > 3:
            acc_w[...] += dt * w
            acc_p[...] += dt * model.cgp_psi(w, g, level)
            t += dt

    cfl.run_adaptive(w0, F, g, level, phys, c, dt_max, 8, callback=cb)
    assert tsum == pytest.approx(t, rel=1e-15)
    np.testing.assert_allclose(mean_w, acc_w / t, rtol=0, atol=1e-13 * np.abs(acc_w / t).max())
    np.testing.assert_allclose(mean_psi, acc_p / t, rtol=0, atol=1e-12 * np.abs(acc_p / t).max())


def test_time_mean_with_fixed_steps_is_the_plain_average():
    from oracle import statistics
    g, phys, w0, F, level = _small()
    states = []
    mean_w, _, tsum, _ = statistics.time_mean(w0, F, g, level, phys, 0.0, 1e-4, 2, 4)
    w = np.array(w0, dtype=np.float64)
    for n in range(6):
        w = model.step(w, F, g, level, phys, 1e-4)
        if n >= 2:
            states.append(w)
    assert tsum == pytest.approx(4e-4, rel=1e-14)
    np.testing.assert_allclose(mean_w, np.mean(states, axis=0), rtol=0,
                               atol=1e-13 * np.abs(mean_w).max())
