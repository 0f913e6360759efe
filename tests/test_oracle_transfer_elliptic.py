"""Pins of the oracle's grid transfers (Sec. 3.1) and elliptic solvers (Sec. 4.3)."""
import numpy as np
import pytest
import scipy.signal

from oracle import elliptic, operators as ops, transfer
from oracle.grid import Grid


def _rand_zero_ring(rng, ny, nx):
    f = np.zeros((ny + 1, nx + 1))
    f[1:-1, 1:-1] = rng.standard_normal((ny - 1, nx - 1))
    return f


# ---------------------------------------------------------------- transfers
def test_full_weighting_exact_on_affine_and_quadratic():
    g = Grid(16, 32)
    x = g.x()[None, :] + 0 * g.y()[:, None]
    y = g.y()[:, None] + 0 * g.x()[None, :]
    c = g.coarse(1)
    xc = c.x()[None, :] + 0 * c.y()[:, None]
    yc = c.y()[:, None] + 0 * c.x()[None, :]
    r = transfer.restrict_fw(2.0 + 3 * x - 5 * y)
    assert np.max(np.abs(r[1:-1, 1:-1] - (2.0 + 3 * xc - 5 * yc)[1:-1, 1:-1])) < 1e-13
    # [1,2,1]/4 of x^2 is x^2 + h^2/2 (closed form of the weights)
    r2 = transfer.restrict_fw(x * x)
    assert np.max(np.abs(r2[1:-1, 1:-1] - (xc * xc + g.dx ** 2 / 2)[1:-1, 1:-1])) < 1e-14
    assert np.all(r[0] == 0) and np.all(r[-1] == 0) and np.all(r[:, 0] == 0) and np.all(r[:, -1] == 0)


def test_bilinear_prolongation_exact_on_bilinear_fields():
    c = Grid(8, 16)
    g = Grid(16, 32)
    f = lambda X, Y: 1.5 - 2 * X + 0.5 * Y + 3 * X * Y  # noqa: E731
    Xc, Yc = np.meshgrid(c.x(), c.y())
    Xf, Yf = np.meshgrid(g.x(), g.y())
    p = transfer.prolong_bilinear(f(Xc, Yc))
    assert np.max(np.abs(p - f(Xf, Yf))) < 1e-13


@pytest.mark.parametrize("level", [1, 2])
def test_prolongation_is_four_times_restriction_transpose(level):
    """4^l <R f, g> = <f, P g> in plain sums (zero rings)."""
    rng = np.random.default_rng(5)
    g = Grid(32, 64)
    c = g.coarse(level)
    f = _rand_zero_ring(rng, g.ny, g.nx)
    h = _rand_zero_ring(rng, c.ny, c.nx)
    lhs = 4 ** level * np.sum(transfer.restrict(f, level) * h)
    rhs = np.sum(f * transfer.prolong(h, level))
    assert abs(lhs - rhs) < 1e-12 * np.sum(np.abs(f))


def test_two_level_restriction_is_separable_seven_point():
    rng = np.random.default_rng(6)
    g = Grid(32, 64)
    f = _rand_zero_ring(rng, g.ny, g.nx)
    w1 = np.array([1, 2, 3, 4, 3, 2, 1]) / 16.0
    conv = scipy.signal.correlate2d(f, np.outer(w1, w1), mode="same")
    ref = conv[4:-4:4, 4:-4:4]
    got = transfer.restrict(f, 2)[1:-1, 1:-1]
    assert np.max(np.abs(got - ref)) < 1e-14


def test_two_level_prolongation_is_direct_bilinear():
    rng = np.random.default_rng(7)
    c = Grid(8, 16)
    h = _rand_zero_ring(rng, c.ny, c.nx)
    got = transfer.prolong(h, 2)
    # direct bilinear interpolation from the 4h grid
    fy = np.arange(4 * c.ny + 1) / 4.0
    fx = np.arange(4 * c.nx + 1) / 4.0
    J0 = np.minimum(fy.astype(int), c.ny - 1)
    I0 = np.minimum(fx.astype(int), c.nx - 1)
    ty = (fy - J0)[:, None]
    tx = (fx - I0)[None, :]
    ref = ((1 - ty) * (1 - tx) * h[J0][:, I0] + (1 - ty) * tx * h[J0][:, I0 + 1]
           + ty * (1 - tx) * h[J0 + 1][:, I0] + ty * tx * h[J0 + 1][:, I0 + 1])
    assert np.max(np.abs(got - ref)) < 1e-14


def _dense(apply, shape_in):
    n = shape_in[0] * shape_in[1]
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        cols.append(apply(e.reshape(shape_in)).ravel())
    return np.array(cols).T


def test_transfer_transposes_match_dense():
    rng = np.random.default_rng(8)
    fshape, cshape = (9, 7), (5, 4)
    R = _dense(transfer.restrict_fw, fshape)
    P = _dense(transfer.prolong_bilinear, cshape)
    g = rng.standard_normal(cshape)
    f = rng.standard_normal(fshape)
    assert np.allclose(transfer.restrict_fw_T(g).ravel(), R.T @ g.ravel(), atol=1e-14)
    assert np.allclose(transfer.prolong_bilinear_T(f).ravel(), P.T @ f.ravel(), atol=1e-14)


# ---------------------------------------------------------------- elliptic
def test_sine_matrix_orthogonality():
    for n in (8, 12, 64):
        S = elliptic.sine_matrix(n)
        assert np.max(np.abs((2.0 / n) * S @ S - np.eye(n - 1))) < 1e-13


@pytest.mark.parametrize("nx,ny", [(16, 32), (24, 48), (32, 64)])
def test_three_routes_agree_and_residual(nx, ny):
    rng = np.random.default_rng(9)
    g = Grid(nx, ny)
    r = _rand_zero_ring(rng, ny, nx)
    sols = {rt: elliptic.poisson(r, g.dx, g.dy, rt) for rt in ("dense", "dst", "sparse")}
    ref = sols["sparse"]
    for rt in ("dense", "dst"):
        assert np.max(np.abs(sols[rt] - ref)) < 1e-12 * np.max(np.abs(ref))
    res = ops.laplacian(sols["dst"], g.dx, g.dy) - r
    assert np.max(np.abs(res[1:-1, 1:-1])) < 1e-10 * np.max(np.abs(r))
    assert np.all(sols["dst"][0] == 0) and np.all(sols["dst"][:, -1] == 0)


@pytest.mark.parametrize("m,n", [(1, 1), (3, 2)])
def test_manufactured_solution(m, n):
    """psi = sin(m pi x) sin(n pi (y+1)/2): exact from the discrete RHS, O(h^2) from the continuous one."""
    errs = []
    for N in (32, 64, 128):
        g = Grid(N, 2 * N)
        X, Y = np.meshgrid(g.x(), g.y())
        ky = n * np.pi / g.ly
        psi = np.sin(m * np.pi * X) * np.sin(ky * (Y - g.y0))
        rd = ops.laplacian(psi, g.dx, g.dy)
        sd = elliptic.poisson(rd, g.dx, g.dy)
        assert np.max(np.abs(sd - psi)) < 1e-12
        rc = -((m * np.pi) ** 2 + ky ** 2) * psi
        errs.append(np.max(np.abs(elliptic.poisson(rc, g.dx, g.dy) - psi)))
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.9 < errs[1] / errs[2] < 4.1


def test_eigenvalues_match_laplacian_of_sine_modes():
    g = Grid(12, 18)
    lam = elliptic.eigenvalues(g.nx, g.ny, g.dx, g.dy)
    for k, l in [(1, 1), (5, 3), (11, 17)]:
        X, Y = np.meshgrid(np.arange(g.nx + 1), np.arange(g.ny + 1))
        f = np.sin(np.pi * k * X / g.nx) * np.sin(np.pi * l * Y / g.ny)
        L = ops.laplacian(f, g.dx, g.dy)
        assert np.max(np.abs(L[1:-1, 1:-1] - lam[l - 1, k - 1] * f[1:-1, 1:-1])) < 1e-9 * abs(lam[l - 1, k - 1])


def test_two_layer_cramer_matches_coupled_sparse_and_residual():
    rng = np.random.default_rng(10)
    g = Grid(16, 32)
    F1, F2 = 2000.0, 500.0
    Q1 = _rand_zero_ring(rng, g.ny, g.nx)
    Q2 = _rand_zero_ring(rng, g.ny, g.nx)
    p1, p2 = elliptic.two_layer(Q1, Q2, g.dx, g.dy, F1, F2, "dst")
    s1, s2 = elliptic.two_layer(Q1, Q2, g.dx, g.dy, F1, F2, "sparse")
    d1, d2 = elliptic.two_layer(Q1, Q2, g.dx, g.dy, F1, F2, "dense")
    sc = max(np.max(np.abs(s1)), np.max(np.abs(s2)))
    for a, b in [(p1, s1), (p2, s2), (d1, s1), (d2, s2)]:
        assert np.max(np.abs(a - b)) < 1e-12 * sc
    r1 = ops.laplacian(p1, g.dx, g.dy) + F1 * (p2 - p1) - Q1
    r2 = ops.laplacian(p2, g.dx, g.dy) + F2 * (p1 - p2) - Q2
    assert np.max(np.abs(r1[1:-1, 1:-1])) < 1e-9 and np.max(np.abs(r2[1:-1, 1:-1])) < 1e-9


def test_two_layer_mode_split_equals_cramer():
    """delta = F2/(F1+F2): delta Q1 + (1-delta) Q2 is a Poisson problem for the
    barotropic streamfunction and Q1 - Q2 a Helmholtz problem for psi1 - psi2."""
    rng = np.random.default_rng(15)
    g = Grid(16, 32)
    F1, F2 = 2083.3333, 416.6667
    Q1 = _rand_zero_ring(rng, g.ny, g.nx)
    Q2 = _rand_zero_ring(rng, g.ny, g.nx)
    p1, p2 = elliptic.two_layer(Q1, Q2, g.dx, g.dy, F1, F2, "sparse")
    d = F2 / (F1 + F2)
    bt = elliptic.poisson(d * Q1 + (1 - d) * Q2, g.dx, g.dy, "sparse")
    A = elliptic.laplacian_matrix(g.nx, g.ny, g.dx, g.dy)
    import scipy.sparse
    import scipy.sparse.linalg
    H = (A - (F1 + F2) * scipy.sparse.eye(A.shape[0])).tocsc()
    bc = np.zeros_like(Q1)
    bc[1:-1, 1:-1] = scipy.sparse.linalg.spsolve(H, (Q1 - Q2)[1:-1, 1:-1].ravel()).reshape(g.ny - 1, g.nx - 1)
    assert np.max(np.abs(bt + (1 - d) * bc - p1)) < 1e-12 * np.max(np.abs(p1))
    assert np.max(np.abs(bt - d * bc - p2)) < 1e-12 * np.max(np.abs(p2))


def test_two_layer_uncoupled_reduces_to_poisson():
    rng = np.random.default_rng(16)
    g = Grid(16, 32)
    Q1 = _rand_zero_ring(rng, g.ny, g.nx)
    Q2 = _rand_zero_ring(rng, g.ny, g.nx)
    p1, p2 = elliptic.two_layer(Q1, Q2, g.dx, g.dy, 0.0, 0.0, "dst")
    assert np.max(np.abs(p1 - elliptic.poisson(Q1, g.dx, g.dy))) < 1e-14
    assert np.max(np.abs(p2 - elliptic.poisson(Q2, g.dx, g.dy))) < 1e-14
