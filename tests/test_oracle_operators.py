"""Pins of the oracle's spatial operators (Arakawa Jacobian, Laplacian, beta term).

Sec. 4.1 states the properties that the J1/J2/J3 combination is built for:
discrete conservation of energy and enstrophy and skew-symmetry, which J1 alone
lacks.  Each test below is chosen so that a dropped term, a wrong sign or a
swapped index in any of the twelve bracket products fails it.
"""
import numpy as np
import pytest

from oracle import operators as ops
from oracle.grid import Grid


def _rand_zero_ring(rng, ny, nx):
    f = np.zeros((ny + 1, nx + 1))
    f[1:-1, 1:-1] = rng.standard_normal((ny - 1, nx - 1))
    return f


@pytest.fixture
def g():
    return Grid(32, 64)


def test_arakawa_conserves_energy_and_enstrophy(g):
    rng = np.random.default_rng(11)
    psi = _rand_zero_ring(rng, g.ny, g.nx)
    w = _rand_zero_ring(rng, g.ny, g.nx)
    J = ops.arakawa(psi, w, g.dx, g.dy)
    scale = np.abs(psi * J).sum() + np.abs(w * J).sum()
    assert abs((psi * J).sum()) < 1e-13 * scale
    assert abs((w * J).sum()) < 1e-13 * scale


def test_j1_alone_does_not_conserve(g):
    """Sec. 4.1: the central form J1 is not enough (guards the test above)."""
    rng = np.random.default_rng(12)
    psi = _rand_zero_ring(rng, g.ny, g.nx)
    w = _rand_zero_ring(rng, g.ny, g.nx)
    J1 = ops.jacobian_j1(psi, w, g.dx, g.dy)
    scale = np.abs(w * J1).sum()
    assert abs((w * J1).sum()) > 1e-6 * scale


def test_arakawa_antisymmetric(g):
    rng = np.random.default_rng(13)
    a = rng.standard_normal(g.shape)
    b = rng.standard_normal(g.shape)
    Jab = ops.arakawa(a, b, g.dx, g.dy)
    Jba = ops.arakawa(b, a, g.dx, g.dy)
    assert np.max(np.abs(Jab + Jba)) < 1e-12 * np.max(np.abs(Jab))
    assert np.max(np.abs(ops.arakawa(a, a, g.dx, g.dy))) < 1e-12 * np.max(np.abs(Jab))


def test_arakawa_skew_adjoint_in_second_argument(g):
    """sum a J(psi, w) = - sum w J(psi, a) for zero-ring fields (enstrophy conservation, polarised)."""
    rng = np.random.default_rng(14)
    psi, w, a = (_rand_zero_ring(rng, g.ny, g.nx) for _ in range(3))
    lhs = (a * ops.arakawa(psi, w, g.dx, g.dy)).sum()
    rhs = -(w * ops.arakawa(psi, a, g.dx, g.dy)).sum()
    assert abs(lhs - rhs) < 1e-12 * np.abs(a * ops.arakawa(psi, w, g.dx, g.dy)).sum()


def _smooth(grid, kind):
    x = grid.x()[None, :]
    y = grid.y()[:, None]
    if kind == "p":
        return np.sin(1.3 * x + 0.4) * np.cos(0.7 * y - 0.2) + 0.3 * x * y * y
    return np.exp(0.5 * x) * np.sin(1.1 * y + 0.3) + 0.2 * x * x


def _exact_jacobian(grid):
    x = grid.x()[None, :] + 0 * grid.y()[:, None]
    y = grid.y()[:, None] + 0 * grid.x()[None, :]
    px = 1.3 * np.cos(1.3 * x + 0.4) * np.cos(0.7 * y - 0.2) + 0.3 * y * y
    py = -0.7 * np.sin(1.3 * x + 0.4) * np.sin(0.7 * y - 0.2) + 0.6 * x * y
    qx = 0.5 * np.exp(0.5 * x) * np.sin(1.1 * y + 0.3) + 0.4 * x
    qy = 1.1 * np.exp(0.5 * x) * np.cos(1.1 * y + 0.3)
    return px * qy - py * qx


@pytest.mark.parametrize("fn", ["arakawa", "jacobian_j1", "jacobian_j2", "jacobian_j3"])
def test_each_jacobian_form_is_second_order(fn):
    """Every one of J1, J2, J3 (and their mean) approximates p_x q_y - p_y q_x at O(h^2)."""
    errs = []
    for n in (16, 32, 64):
        gr = Grid(n, 2 * n)
        J = getattr(ops, fn)(_smooth(gr, "p"), _smooth(gr, "q"), gr.dx, gr.dy)
        errs.append(np.max(np.abs((J - _exact_jacobian(gr))[1:-1, 1:-1])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs


def test_beta_term_closed_forms(g):
    """J(psi, y) is a centred x-derivative: exact for psi quadratic in x, zero for psi(y)."""
    x = g.x()[None, :] + 0 * g.y()[:, None]
    y = g.y()[:, None] + 0 * g.x()[None, :]
    b = ops.beta_term(x * x + 3 * x, g)
    assert np.allclose(b[1:-1, 1:-1], (2 * x + 3)[1:-1, 1:-1], rtol=0, atol=1e-11)
    b0 = ops.beta_term(np.sin(3 * y) + y * y, g)
    assert np.max(np.abs(b0)) < 1e-11


def test_beta_term_matches_arakawa_psi_x_limit():
    errs = []
    for n in (16, 32, 64):
        gr = Grid(n, 2 * n)
        x = gr.x()[None, :] + 0 * gr.y()[:, None]
        y = gr.y()[:, None] + 0 * gr.x()[None, :]
        psi = np.sin(2 * x) * np.cos(1.5 * y)
        errs.append(np.max(np.abs((ops.beta_term(psi, gr) - 2 * np.cos(2 * x) * np.cos(1.5 * y))[1:-1, 1:-1])))
    assert 3.7 < errs[0] / errs[1] < 4.3 and 3.8 < errs[1] / errs[2] < 4.2


def test_laplacian_eigenfunction(g):
    m, n = 3, 5
    x = g.x()[None, :]
    y = g.y()[:, None]
    f = np.sin(m * np.pi * x / g.lx) * np.sin(n * np.pi * (y - g.y0) / g.ly)
    mu = ((2 * np.cos(m * np.pi * g.dx / g.lx) - 2) / g.dx ** 2
          + (2 * np.cos(n * np.pi * g.dy / g.ly) - 2) / g.dy ** 2)
    L = ops.laplacian(f, g.dx, g.dy)
    assert np.max(np.abs(L[1:-1, 1:-1] - mu * f[1:-1, 1:-1])) < 1e-10 * abs(mu)


def _dense_matrix(apply, shape):
    n = shape[0] * shape[1]
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = apply(e.reshape(shape)).ravel()
    return M


def test_transpose_apply_matches_dense_transpose():
    gr = Grid(5, 7)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(gr.shape)
    op = lambda f: ops.arakawa(psi, f, gr.dx, gr.dy) + 0.3 * ops.laplacian(f, gr.dx, gr.dy)  # noqa: E731
    M = _dense_matrix(op, gr.shape)
    inner = np.zeros(gr.shape, bool)
    inner[1:-1, 1:-1] = True
    idx = np.flatnonzero(inner.ravel())
    Mi = M[np.ix_(idx, idx)]
    mu = np.zeros(gr.shape)
    mu[1:-1, 1:-1] = rng.standard_normal((gr.ny - 1, gr.nx - 1))
    ref = np.zeros(gr.shape)
    ref.ravel()[idx] = Mi.T @ mu.ravel()[idx]
    got = ops.transpose_apply(op, mu)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
