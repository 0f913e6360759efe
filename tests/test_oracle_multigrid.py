"""Pins of the oracle's multigrid V-cycles (the iterative black-box solver under CGP)."""
import numpy as np
import pytest

import cgp_inputs as ci
from oracle import elliptic, model, multigrid as mg
from oracle.grid import Grid
from oracle.model import Physics


def _rhs(nx, ny, seed=0):
    rng = np.random.default_rng(seed)
    r = np.zeros((ny + 1, nx + 1))
    r[1:-1, 1:-1] = rng.standard_normal((ny - 1, nx - 1))
    return r


@pytest.mark.parametrize("nx,ny,lx,ly", [(64, 128, 1.0, 2.0), (48, 96, 1.0, 2.0),
                                         (32, 64, 1.0, 1.0), (96, 48, 2.0, 1.0)])
def test_cycles_converge_to_the_direct_solve(nx, ny, lx, ly):
    dx, dy = lx / nx, ly / ny
    r = _rhs(nx, ny)
    exact = elliptic.poisson(r, dx, dy, "dst")
    got = mg.poisson_mg(r, dx, dy, 40)
    assert np.abs(got - exact).max() < 1e-12 * np.abs(exact).max()


def test_residual_falls_by_a_textbook_factor_per_cycle():
    nx, ny = 128, 256
    dx, dy = 1.0 / nx, 2.0 / ny
    f = _rhs(nx, ny, 3)
    u = np.zeros_like(f)
    norms = [np.linalg.norm(mg.residual(u, f, dx, dy))]
    for _ in range(4):
        mg.vcycle(u, f, dx, dy)
        norms.append(np.linalg.norm(mg.residual(u, f, dx, dy)))
    rates = np.array(norms[1:]) / np.array(norms[:-1])
    assert rates.max() < 0.2, rates


def test_coarsest_grid_is_solved_exactly_and_solutions_are_fixed_points():
    dx, dy = 1.0 / 4, 2.0 / 8
    f = _rhs(4, 8, 5)
    assert mg.coarsest(4, 8) and not mg.coarsest(8, 16)
    u = mg.poisson_mg(f, dx, dy, 1)
    assert np.abs(mg.residual(u, f, dx, dy)).max() < 1e-12 * np.abs(f).max()
    # a half sweep leaves the exact solution of a finer grid unchanged
    nx, ny = 16, 32
    f = _rhs(nx, ny, 6)
    x = elliptic.poisson(f, 1.0 / nx, 2.0 / ny, "sparse")
    y = x.copy()
    mg.rb_sweep(y, f, 1.0 / nx, 2.0 / ny, 0)
    mg.rb_sweep(y, f, 1.0 / nx, 2.0 / ny, 1)
    assert np.abs(y - x).max() < 1e-12 * np.abs(x).max()


def test_dense_matrix_matches_the_sparse_one():
    A = mg.laplacian_matrix(6, 5, 0.3, 0.7)
    B = elliptic.laplacian_matrix(6, 5, 0.3, 0.7).toarray()
    assert np.array_equal(A, B)


def test_cgp_step_with_converged_multigrid_equals_the_sine_transform_step():
    case = ci.make_case(64, 128, dt=1e-4)
    g = Grid(64, 128)
    phys = Physics(inv_re=case.inv_re, inv_ro=case.inv_ro)
    w = ci.initial_field(case, np.random.default_rng(2), scale=1.0)
    F = ci.forcing_field(case)
    a = model.step(w, F, g, 1, phys, case.dt, route="dst")
    b = model.step(w, F, g, 1, phys, case.dt, route="mg30")
    assert np.linalg.norm(a - b) < 1e-12 * np.linalg.norm(a)
