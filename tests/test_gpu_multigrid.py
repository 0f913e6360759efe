"""GPU parity of the multigrid coarse solver (the iterative black box under
CGP) with the oracle's V-cycles, through the C ABI."""
import numpy as np
import pytest
import torch

import cgp_inputs as ci
from gpu_common import oracle_setup, random_state, rel_l2, say, to_dev, to_np
from oracle import cfl as ocfl, elliptic, model as om, transfer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_3290_amd import _lib
    _lib.load()
    yield
    torch.cuda.synchronize()


def _basin(case, dtype="f64"):
    from paper_1308_3290_amd.api import Basin, config_from_case
    return Basin(config_from_case(case, dtype))


def _oracle_psi(case, w, route):
    g, _ = oracle_setup(case)
    r = transfer.restrict(w, case.level)
    cg = g.coarse(case.level)
    return transfer.prolong(elliptic.poisson(r, cg.dx, cg.dy, route), case.level)


# coarse grids 32x64 (levels down to 4x8), 128x256, 48x96 (coarsest 6x12:
# 55 unknowns), 64x128
@pytest.mark.parametrize("nx,ny,level", [(64, 128, 1), (128, 256, 0), (96, 192, 1),
                                         (256, 512, 2)])
def test_multigrid_solve_matches_oracle_cycles(nx, ny, level):
    case = ci.make_case(nx, ny, level=level, solver=1, mg_cycles=6)
    say(f"multigrid solve {nx}x{ny} level {level}, 6 V-cycles")
    w = random_state(case, 50 + level, 1.0)
    ref = _oracle_psi(case, w, "mg6")
    psi = _basin(case).solve(to_dev(w))
    torch.cuda.synchronize()
    err = rel_l2(to_np(psi), ref)
    say(f"  rel L2 vs oracle = {err:.3e}")
    assert err < 1e-12


def test_multigrid_converges_to_the_sine_transform_solve():
    case = ci.make_case(128, 256, level=1, solver=1, mg_cycles=30)
    w = random_state(case, 60, 1.0)
    a = _basin(case).solve(to_dev(w))
    b = _basin(ci.make_case(128, 256, level=1)).solve(to_dev(w))
    torch.cuda.synchronize()
    assert rel_l2(to_np(a), to_np(b)) < 1e-12


def test_multigrid_fp32():
    case = ci.make_case(64, 128, level=1, solver=1, mg_cycles=6)
    w = random_state(case, 61, 1.0)
    ref = _oracle_psi(case, w, "mg6")
    psi = _basin(case, "f32").solve(to_dev(w, torch.float32))
    torch.cuda.synchronize()
    assert rel_l2(to_np(psi), ref) < 1e-5


@pytest.mark.parametrize("level", [0, 1])
def test_multigrid_trajectory_matches_oracle(level):
    case = ci.make_case(64, 128, level=level, dt=1e-4, solver=1, mg_cycles=8)
    say(f"multigrid CGP step 64x128 level {level}: 15 steps")
    g, phys = oracle_setup(case)
    w0 = random_state(case, 62, 1e-2)
    F = ci.forcing_field(case)
    b = _basin(case)
    w = to_dev(w0)
    Fd = to_dev(F)
    wo = np.array(w0)
    errs = []
    for _ in range(15):
        b.step(w, Fd, nsteps=1)
        wo = om.step(wo, F, g, level, phys, case.dt, route="mg8")
        errs.append(rel_l2(to_np(w), wo))
    say(f"  max per-step rel L2 = {max(errs):.3e}")
    assert max(errs) < 1e-11


def test_multigrid_adaptive_steps_and_graphs():
    """Adaptive steps (the step size set without a pass B launch) against the
    oracle, and captured graphs giving the same bits as direct launches."""
    case = ci.make_case(64, 128, level=1, dt=1e-3, cfl=0.01, solver=1, mg_cycles=8)
    g, phys = oracle_setup(case)
    w0 = random_state(case, 63, 1e-2)
    F = ci.forcing_field(case)
    ref = []
    _, dts = ocfl.run_adaptive(w0, F, g, 1, phys, case.cfl, case.dt, 12, route="mg8",
                               callback=lambda n, w, dt: ref.append(w))
    b = _basin(case)
    w = to_dev(w0)
    Fd = to_dev(F)
    for n in range(12):
        b.step(w, Fd, nsteps=1)
        torch.cuda.synchronize()
        assert rel_l2(to_np(w), ref[n]) < 1e-11, n
    ts = b.time_state()
    assert float(ts[1]) == pytest.approx(sum(dts), rel=1e-12)
    totals = []
    for use_graph in (False, True):
        bb = _basin(case)
        ww = to_dev(w0)
        tot = torch.zeros_like(ww)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            bb.step_mean(ww, Fd, 5, tot, use_graph=use_graph, stream=side)
        torch.cuda.synchronize()
        totals.append((ww, tot))
    assert torch.equal(totals[0][0], totals[1][0]) and torch.equal(totals[0][1], totals[1][1])
