"""Pins of the oracle's CGPRK3 step, two-layer model, diagnostics, adjoint and parameters."""
import json
import math
import os

import numpy as np
import pytest

import cgp_inputs as ci
from oracle import adjoint, diagnostics, elliptic, model, operators as ops, params
from oracle.grid import Grid
from oracle.model import Physics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_zero_ring(rng, ny, nx, scale=1.0):
    f = np.zeros((ny + 1, nx + 1))
    f[1:-1, 1:-1] = scale * rng.standard_normal((ny - 1, nx - 1))
    return f


def _setup(nx=32, ny=64, seed=0):
    case = ci.make_case(nx, ny, dt=1e-4)
    g = Grid(nx, ny)
    phys = Physics(inv_re=case.inv_re, inv_ro=case.inv_ro)
    rng = np.random.default_rng(seed)
    w = _rand_zero_ring(rng, ny, nx, 1.0)
    F = ci.forcing_field(case)
    return case, g, phys, w, F


# ------------------------------------------------------------------ step
def test_level0_cgp_step_is_full_grid_step():
    """l = 0 means no coarsening: bitwise the plain solver."""
    case, g, phys, w, F = _setup()
    psi0 = model.cgp_psi(w, g, 0)
    assert np.array_equal(psi0, elliptic.poisson(w, g.dx, g.dy))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_step_independent_of_solver_route(level):
    case, g, phys, w, F = _setup()
    ref = model.step(w, F, g, level, phys, case.dt, "sparse")
    for rt in ("dense", "dst"):
        got = model.step(w, F, g, level, phys, case.dt, rt)
        assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("level", [0, 1])
def test_vorticity_form_equals_paper_q_form(level):
    """q = Ro omega + y stepped with J(psi, q) equals the vorticity-form step."""
    case, g, phys, w, F = _setup()
    ro = 1.0 / phys.inv_ro
    re = 1.0 / phys.inv_re
    w = 100.0 * w
    q = ro * w + g.y_field()
    qn = model.step_qform(q, ro * F, g, level, ro, re, case.dt)
    wn = model.step(w, F, g, level, phys, case.dt)
    back = (qn - g.y_field()) / ro
    assert np.linalg.norm(back - wn) < 1e-8 * np.linalg.norm(wn)


def test_rk3_stability_polynomial_on_an_eigenmode():
    """No beta, no forcing, l = 0, omega0 a discrete sine mode: psi is proportional
    to omega, J(psi, omega) vanishes and one step multiplies by 1 + z + z^2/2 + z^3/6."""
    g = Grid(16, 32)
    phys = Physics(inv_re=1.0 / 50.0, inv_ro=0.0)
    I, J = np.meshgrid(np.arange(g.nx + 1), np.arange(g.ny + 1))
    w = np.sin(np.pi * 3 * I / g.nx) * np.sin(np.pi * 4 * J / g.ny)
    mu = elliptic.eigenvalues(g.nx, g.ny, g.dx, g.dy)[3, 2]
    dt = 2e-4
    z = dt * phys.inv_re * mu
    w1 = model.step(w, np.zeros_like(w), g, 0, phys, dt)
    amp = 1 + z + z * z / 2 + z ** 3 / 6
    assert np.max(np.abs(w1 - amp * w)) < 1e-13


def test_rhs_conserves_energy_without_dissipation_and_forcing():
    """<psi, G> = 0 when 1/Re = F = 0, with the beta term on (J and beta are skew)."""
    case, g, phys, w, F = _setup()
    phys0 = Physics(inv_re=0.0, inv_ro=phys.inv_ro)
    psi = model.cgp_psi(w, g, 0)
    G = model.rhs(w, psi, np.zeros_like(w), g, phys0)
    scale = np.sum(np.abs(psi * G))
    assert abs(np.sum(psi * G)) < 1e-12 * scale
    # enstrophy: <omega, G> = 0 once beta is off too
    G2 = model.rhs(w, psi, np.zeros_like(w), g, Physics(inv_re=0.0, inv_ro=0.0))
    assert abs(np.sum(w * G2)) < 1e-12 * np.sum(np.abs(w * G2))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_cgp_map_is_symmetric(level):
    rng = np.random.default_rng(21)
    g = Grid(32, 64)
    a = _rand_zero_ring(rng, g.ny, g.nx)
    b = _rand_zero_ring(rng, g.ny, g.nx)
    lhs = np.sum(b * model.cgp_psi(a, g, level))
    rhs = np.sum(a * model.cgp_psi(b, g, level))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ------------------------------------------------------------------ two layers
@pytest.mark.parametrize("level", [0, 1])
def test_two_layer_decouples(level):
    """F1 = F2 = 0: layer 1 is the one-layer step with F; with zero drag, layer 2
    is the one-layer step with F = 0."""
    case, g, phys, w, F = _setup()
    rng = np.random.default_rng(3)
    w2 = _rand_zero_ring(rng, g.ny, g.nx)
    Q = np.stack([w, w2])
    p2 = Physics(inv_re=phys.inv_re, inv_ro=phys.inv_ro, f1=0.0, f2=0.0, drag=0.0)
    out = model.step_two_layer(Q, F, g, level, p2, case.dt)
    r1 = model.step(w, F, g, level, phys, case.dt)
    r2 = model.step(w2, np.zeros_like(F), g, level, phys, case.dt)
    assert np.linalg.norm(out[0] - r1) < 1e-14 * np.linalg.norm(r1)
    assert np.linalg.norm(out[1] - r2) < 1e-14 * np.linalg.norm(r2)


def test_two_layer_relative_vorticity_is_laplacian_of_psi():
    """At l = 0 the coupled solve is exact, so zeta_i = Q_i - F_i (psi_j - psi_i)
    must equal the 5-point Laplacian of psi_i (the definition of zeta)."""
    rng = np.random.default_rng(5)
    g = Grid(16, 32)
    p = Physics(inv_re=0.0, inv_ro=0.0, f1=2083.3, f2=416.7, drag=0.0)
    Q = np.stack([_rand_zero_ring(rng, g.ny, g.nx), _rand_zero_ring(rng, g.ny, g.nx)])
    psi = model.cgp_psi_two_layer(Q, g, 0, p)
    z = model.relative_vorticity_two_layer(Q, psi, p)
    for i in range(2):
        L = ops.laplacian(psi[i], g.dx, g.dy)
        assert np.max(np.abs(z[i] - L)) < 1e-10 * np.max(np.abs(L))


def test_two_layer_drag_damps_layer_two():
    """With only drag acting (no J, beta, viscosity, coupling), zeta_2 = Q_2 decays by
    the RK3 polynomial of z = -drag dt."""
    g = Grid(16, 32)
    rng = np.random.default_rng(4)
    Q = np.stack([np.zeros(g.shape), _rand_zero_ring(rng, g.ny, g.nx)])
    # remove the Jacobian by using a single sine mode (psi proportional to Q)
    I, J = np.meshgrid(np.arange(g.nx + 1), np.arange(g.ny + 1))
    Q[1] = np.sin(np.pi * 2 * I / g.nx) * np.sin(np.pi * 5 * J / g.ny)
    p = Physics(inv_re=0.0, inv_ro=0.0, f1=0.0, f2=0.0, drag=3.0)
    dt = 1e-2
    out = model.step_two_layer(Q, np.zeros(g.shape), g, 0, p, dt)
    z = -3.0 * dt
    assert np.max(np.abs(out[1] - (1 + z + z * z / 2 + z ** 3 / 6) * Q[1])) < 1e-14
    assert np.max(np.abs(out[0])) == 0.0


# ------------------------------------------------------------------ diagnostics
def test_energy_equals_minus_psi_laplacian_sum():
    rng = np.random.default_rng(30)
    g = Grid(32, 64)
    psi = _rand_zero_ring(rng, g.ny, g.nx)
    E = diagnostics.energy(psi, g)
    ref = -g.dx * g.dy / (2 * g.lx * g.ly) * np.sum(psi * ops.laplacian(psi, g.dx, g.dy))
    assert abs(E - ref) < 1e-12 * abs(ref)


def test_energy_converges_to_continuous_value():
    errs = []
    for N in (32, 64, 128):
        g = Grid(N, 2 * N)
        X, Y = np.meshgrid(g.x(), g.y())
        psi = np.sin(np.pi * X) * np.sin(np.pi * (Y + 1) / 2)
        exact = 0.5 * (np.pi ** 2 + (np.pi / 2) ** 2) * 0.25  # 1/2 <|grad psi|^2> over the basin
        errs.append(abs(diagnostics.energy(psi, g) - exact))
    assert 3.8 < errs[0] / errs[1] < 4.2


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("level", [0, 1])
def test_tlm_matches_central_difference(level):
    case, g, phys, w, F = _setup(16, 32)
    rng = np.random.default_rng(40)
    w = 50 * w
    dw = _rand_zero_ring(rng, g.ny, g.nx)
    dF = _rand_zero_ring(rng, g.ny, g.nx)
    eps = 1e-4
    dt = 5e-4
    plus = model.step(w + eps * dw, F + eps * dF, g, level, phys, dt)
    minus = model.step(w - eps * dw, F - eps * dF, g, level, phys, dt)
    fd = (plus - minus) / (2 * eps)
    _, tl = adjoint.step_tlm(w, dw, F, dF, g, level, phys, dt)
    assert np.linalg.norm(fd - tl) < 1e-8 * np.linalg.norm(tl)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_adjoint_dot_product(level):
    case, g, phys, w, F = _setup(16, 32)
    rng = np.random.default_rng(41)
    w = 50 * w
    dw = _rand_zero_ring(rng, g.ny, g.nx)
    dF = _rand_zero_ring(rng, g.ny, g.nx)
    lam = _rand_zero_ring(rng, g.ny, g.nx)
    dt = 5e-4
    _, tl = adjoint.step_tlm(w, dw, F, dF, g, level, phys, dt)
    aw, aF = adjoint.step_adjoint(w, F, lam, g, level, phys, dt)
    lhs = np.sum(tl * lam)
    rhs = np.sum(dw * aw) + np.sum(dF * aF)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + np.sum(np.abs(tl * lam)))


def test_adjoint_uses_identities_the_gpu_relies_on():
    """(J(psi, .))^T = -J(psi, .) and (J(., omega))^T = J(omega, .) on zero-ring fields;
    the beta stencil is skew."""
    rng = np.random.default_rng(42)
    g = Grid(12, 20)
    psi, w, mu = (_rand_zero_ring(rng, g.ny, g.nx) for _ in range(3))
    t1 = ops.transpose_apply(lambda f: ops.arakawa(psi, f, g.dx, g.dy), mu)
    assert np.max(np.abs(t1 + ops.arakawa(psi, mu, g.dx, g.dy))) < 1e-10 * np.max(np.abs(t1))
    t2 = ops.transpose_apply(lambda f: ops.arakawa(f, w, g.dx, g.dy), mu)
    assert np.max(np.abs(t2 - ops.arakawa(w, mu, g.dx, g.dy))) < 1e-10 * np.max(np.abs(t2))
    t3 = ops.transpose_apply(lambda f: ops.beta_term(f, g), mu)
    assert np.max(np.abs(t3 + ops.beta_term(mu, g))) < 1e-10 * np.max(np.abs(t3))


def test_trajectory_gradient_matches_finite_differences():
    p = ci.adjoint_c4(nx=16, ny=32, nsteps=6, ckpt_every=2, ndir=3, obs_fraction=0.1)
    c = p.case
    g = Grid(c.nx, c.ny)
    phys = Physics(inv_re=c.inv_re, inv_ro=c.inv_ro)
    w0 = 100 * p.omega0
    dt = 2e-4
    L, gw, gF = adjoint.loss_and_gradient(w0, p.forcing, p.obs_index, p.obs_value, g, c.level,
                                          phys, dt, c.nsteps)
    for d in range(3):
        eps = 1e-5
        lp = adjoint.loss(w0 + eps * p.dir_omega[d], p.forcing + eps * p.dir_forcing[d],
                          p.obs_index, p.obs_value, g, c.level, phys, dt, c.nsteps)
        lm = adjoint.loss(w0 - eps * p.dir_omega[d], p.forcing - eps * p.dir_forcing[d],
                          p.obs_index, p.obs_value, g, c.level, phys, dt, c.nsteps)
        fd = (lp - lm) / (2 * eps)
        an = np.sum(gw * p.dir_omega[d]) + np.sum(gF * p.dir_forcing[d])
        assert abs(fd - an) < 1e-6 * abs(an) + 1e-12


# ------------------------------------------------------------------ parameters
def _close(a, b, rel):
    return abs(a - b) <= rel * abs(b)


def test_table1_recomputed():
    t = json.load(open(os.path.join(GOLDEN, "table1_one_layer.json")))
    for name, e in t["experiments"].items():
        p = params.one_layer(e["L_km"] * 1e3, e["beta"], e["nu"], e["V"])
        assert _close(p["Ro"], e["Ro"], 1e-3)
        assert _close(p["Re"], e["Re"], 1e-2)
        assert _close(p["delta_M_over_L"], e["delta_M_over_L"], 1e-3)
        assert _close(p["delta_I_over_L"], e["delta_I_over_L"], 1e-3)
        assert _close(p["L_over_V_years"], e["L_over_V_year"], 2e-3)
        assert _close(p["Re_B"], t["text_values"]["Re_B"][name], 1e-2)


def test_table2_recomputed():
    t = json.load(open(os.path.join(GOLDEN, "table2_two_layer.json")))
    for name, e in t["inputs"].items():
        pr = t["printed"][name]
        p = params.two_layer(e["L_km"] * 1e3, e["H1_km"] * 1e3, e["H2_km"] * 1e3, e["f0"], e["beta"],
                             e["rho1"], e["gprime"], e["tau0"], e["gamma"], e["nu"])
        assert _close(p["delta_M"] / 1e3, pr["delta_M_km"], 2e-3)
        assert _close(p["delta_S"] / 1e3, pr["delta_S_km"], 2e-3)
        assert _close(p["delta_I"] / 1e3, pr["delta_I_km"], 2e-3)
        assert _close(p["V"], pr["V"], 5e-3)
        assert _close(p["L_over_V_years"], pr["L_over_V_year"], 3e-3)
        assert _close(p["Ro"], pr["Ro"], 5e-3)
        assert _close(p["Fr"], pr["Fr"], 1e-2)
        assert _close(p["sigma"], pr["sigma"], 5e-3)
        assert _close(p["A"], pr["A"], 5e-3)
        assert p["delta"] == pr["delta"]
        assert _close(p["Re"], pr["Re"], 1e-3)
        if name == "1":
            assert _close(p["Rd"] / 1e3, pr["Rd_km"], 1e-3)
            assert _close(p["L_over_Rd"], pr["L_over_Rd"], 1e-3)
        else:  # printed 31.16 km is a misprint: the inputs give 34.16 km
            assert _close(p["Rd"] / 1e3, 34.16, 1e-3)
            assert not _close(p["Rd"] / 1e3, pr["Rd_km"], 5e-2)
        # F1 + F2 = (L/Rd)^2 in the vorticity form
        assert _close(p["f1"] + p["f2"], p["L_over_Rd"] ** 2, 1e-12)


def test_two_layer_workload_coefficients():
    c = ci.case_c2(1)
    assert math.isclose(c.f1 + c.f2, 1.0 / 0.02 ** 2, rel_tol=1e-14)
    assert math.isclose(c.f2 / (c.f1 + c.f2), 1.0 / 6.0, rel_tol=1e-14)
    assert math.isclose(c.drag, 1e-2 / 0.0036, rel_tol=1e-14)
