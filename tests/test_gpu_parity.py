"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 per-step relative L2 of omega <= 1e-11, FP32 <= 1e-4 (the
targets set for this method); the elliptic map alone to 1e-12 (FP64).
Sizes span several tiles with ragged tails (64-wide stencil tiles against
nx + 1 = 65, 97, 129, ... nodes), coarse lengths 2^k and 3*2^k, the largest
workload (512 x 1024), and the degenerate coarse grid 4 x 4.
"""
import numpy as np
import pytest
import torch

import cgp_inputs as ci
from oracle import adjoint as oadj
from oracle import diagnostics as odiag
from oracle import model as om

from gpu_common import oracle_setup, random_state, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-4


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


def _tdt(dtype):
    return torch.float64 if dtype == "f64" else torch.float32


# ----------------------------------------------------------------- elliptic map
SOLVE_CASES = [
    (64, 128, 0), (64, 128, 1), (64, 128, 2), (96, 192, 1), (48, 96, 0), (128, 64, 1),
    (16, 16, 2), (192, 384, 2), (512, 1024, 1), (512, 1024, 2), (512, 1024, 0),
    (64, 128, 3), (512, 1024, 3),  # three levels of coarsening (c = 8)
    (64, 768, 0), (96, 1536, 1),  # column transforms of 1536 points (radix 3 last)
]


@pytest.mark.parametrize("nx,ny,level", SOLVE_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_solve_matches_oracle(nx, ny, level, dtype):
    say(f"solve parity nx={nx} ny={ny} level={level} {dtype}")
    case = ci.make_case(nx, ny, level=level)
    g, _ = oracle_setup(case)
    w = random_state(case, 100 + level)
    ref = om.cgp_psi(w, g, level)
    b = _basin(case, dtype)
    psi = b.solve(to_dev(w, _tdt(dtype)))
    torch.cuda.synchronize()
    err = rel_l2(to_np(psi), ref)
    say(f"  rel L2 = {err:.3e}")
    assert err < (1e-12 if dtype == "f64" else 2e-6)
    assert np.all(to_np(psi)[[0, -1], :] == 0) and np.all(to_np(psi)[:, [0, -1]] == 0)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_two_layer_solve_matches_oracle(level):
    say(f"two-layer solve parity level={level}")
    c2 = ci.case_c2(level)
    case = ci.make_case(64, 128, level=level, nlayers=2, f1=c2.f1, f2=c2.f2, drag=c2.drag)
    g, phys = oracle_setup(case)
    Q = random_state(case, 7)
    ref = om.cgp_psi_two_layer(Q, g, level, phys)
    b = _basin(case)
    psi = b.solve(to_dev(Q))
    torch.cuda.synchronize()
    err = rel_l2(to_np(psi), ref)
    say(f"  rel L2 = {err:.3e}")
    assert err < 1e-12


# ----------------------------------------------------------------- trajectories
def _trajectory_errors(case, w0, F, nsteps, dtype="f64", layers=1):
    g, phys = oracle_setup(case)
    b = _basin(case, dtype)
    w_dev = to_dev(w0, _tdt(dtype))
    F_dev = to_dev(F, _tdt(dtype))
    w_or = np.array(w0, dtype=np.float64)
    errs = []
    for n in range(nsteps):
        b.step(w_dev, F_dev, nsteps=1)
        if layers == 1:
            w_or = om.step(w_or, F, g, case.level, phys, case.dt)
        else:
            w_or = om.step_two_layer(w_or, F, g, case.level, phys, case.dt)
        errs.append(rel_l2(to_np(w_dev), w_or))
    return np.array(errs), to_np(w_dev), w_or


def test_c0_full_grid_100_steps_fp64():
    case = ci.case_c0()
    say("c0: 64x128 full grid, 100 steps, FP64")
    rng = np.random.default_rng(case.seed)
    w0 = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    errs, w, _ = _trajectory_errors(case, w0, F, case.nsteps)
    say(f"  max per-step rel L2 = {errs.max():.3e} (final {errs[-1]:.3e})")
    assert errs.max() < TOL64
    assert np.all(w[[0, -1], :] == 0) and np.all(w[:, [0, -1]] == 0)


@pytest.mark.parametrize("level", [1, 2, 3])
def test_c0_physics_cgp_100_steps_fp64(level):
    case = ci.case_c0()
    case.level = level
    say(f"64x128 CGP level {level}, 100 steps, FP64")
    rng = np.random.default_rng(case.seed)
    w0 = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    errs, _, _ = _trajectory_errors(case, w0, F, case.nsteps)
    say(f"  max per-step rel L2 = {errs.max():.3e}")
    assert errs.max() < TOL64


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_c0_physics_100_steps_fp32(level):
    case = ci.case_c0()
    case.level = level
    say(f"64x128 level {level}, 100 steps, FP32")
    rng = np.random.default_rng(case.seed)
    w0 = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    errs, _, _ = _trajectory_errors(case, w0, F, case.nsteps, dtype="f32")
    say(f"  max per-step rel L2 = {errs.max():.3e}")
    assert errs.max() < TOL32


def test_fused_c8_fp32():
    """The FP32 fused stage kernel at c = 8 with its compile-time 128-point
    transform (512 x 256, a 64 x 32 solve), 30 steps against the FP64 oracle."""
    case = ci.make_case(512, 256, level=3, dt=1e-4, dtype="f32")
    say("512x256 level 3, 30 steps FP32")
    w0 = random_state(case, 7, 1e-3)
    F = ci.forcing_field(case)
    errs, _, _ = _trajectory_errors(case, w0, F, 30, dtype="f32")
    say(f"  max per-step rel L2 = {errs.max():.3e}")
    assert errs.max() < TOL32


# (512, 32, 0): the fused transform + stencil pass at its widest rows (512
# intervals, transforms of 1024 complex values); (1024, 64, 1), (1024, 48, 0):
# rows too wide for it, the unfused one-layer step.  (8, 6, 0): 6 coarse rows,
# not a multiple of the 4 a fused block owns at c = 1 (unfused); (24, 12, 0)
# and (16, 12, 1): the smallest fused grids (3 blocks).  c = 8: (256, 512, 3)
# the fused pass with a runtime transform length (64 points), (512, 256, 3)
# with the compile-time 128-point one, (1024, 64, 3) the unfused passes;
# (256, 512, 4): c = 16 (16 x 32 coarse grid), the unfused passes.
@pytest.mark.parametrize("nx,ny,level", [(96, 192, 1), (48, 96, 0), (192, 96, 2),
                                         (512, 32, 0), (1024, 64, 1), (1024, 48, 0),
                                         (8, 6, 0), (24, 12, 0), (16, 12, 1), (256, 512, 3),
                                         (512, 256, 3), (1024, 64, 3), (256, 512, 4),
                                         (64, 768, 0)])
def test_ragged_and_radix3_trajectories(nx, ny, level):
    case = ci.make_case(nx, ny, level=level, dt=1e-4)
    say(f"{nx}x{ny} level {level}, 30 steps FP64")
    w0 = random_state(case, 5, 1e-3)
    F = ci.forcing_field(case)
    errs, _, _ = _trajectory_errors(case, w0, F, 30)
    say(f"  max per-step rel L2 = {errs.max():.3e}")
    assert errs.max() < TOL64


# Every compile-time row length of the one-layer fused pass at c = 1 (rows of
# 256, 384, 512 and 768 points: nx = 128, 192, 256, 384 at l = 0) and at c = 4
# with 128 points (256x512 at l = 2), whose transforms' last stages write the
# coarse psi rows and the next spectra directly; FP64 and FP32.
@pytest.mark.parametrize("nx,ny,level", [(128, 256, 0), (192, 384, 0), (256, 512, 0),
                                         (384, 768, 0), (256, 512, 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_row_lengths_follow_the_oracle(nx, ny, level, dtype):
    case = ci.make_case(nx, ny, level=level, dt=1e-4)
    say(f"{nx}x{ny} level {level} {dtype}, 10 steps")
    w0 = random_state(case, 6, 1e-3)
    F = ci.forcing_field(case)
    errs, _, _ = _trajectory_errors(case, w0, F, 10, dtype=dtype)
    say(f"  max per-step rel L2 = {errs.max():.3e}")
    assert errs.max() < (TOL64 if dtype == "f64" else TOL32)


# 64x128 at l = 1, 2 (transforms of 64 and 32 points): the unfused two-layer
# passes; 128x256 / 256x128 / 384x192 at l >= 1 (transforms of 128 and 384)
# and 64x128 / 192x96 / 384x192 at l = 0 (c = 1: transforms of 128, 384 and
# 768): the fused two-layer stage kernel
@pytest.mark.parametrize("nx,ny,level", [(64, 128, 0), (64, 128, 1), (64, 128, 2),
                                         (128, 256, 1), (256, 128, 2), (384, 192, 1),
                                         (128, 256, 3), (128, 1536, 1),
                                         (192, 96, 0), (384, 192, 0)])
def test_two_layer_trajectory_fp64(nx, ny, level):
    c2 = ci.case_c2(level)
    case = ci.make_case(nx, ny, level=level, nlayers=2, f1=c2.f1, f2=c2.f2, drag=c2.drag,
                        dt=2.5e-5)
    say(f"two-layer {nx}x{ny} level {level}, 50 steps FP64")
    rng = np.random.default_rng(c2.seed)
    Q0 = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    errs, w, _ = _trajectory_errors(case, Q0, F, 50, layers=2)
    say(f"  max per-step rel L2 = {errs.max():.3e}")
    assert errs.max() < TOL64


def test_two_layer_trajectory_fp32():
    c2 = ci.case_c2(1)
    case = ci.make_case(64, 128, level=1, nlayers=2, f1=c2.f1, f2=c2.f2, drag=c2.drag, dt=2.5e-5)
    rng = np.random.default_rng(c2.seed)
    Q0 = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    errs, _, _ = _trajectory_errors(case, Q0, F, 50, dtype="f32", layers=2)
    say(f"two-layer FP32 max per-step rel L2 = {errs.max():.3e}")
    assert errs.max() < TOL32


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_c1_full_size_steps(level):
    """The 512 x 1024 workload itself, in the bench's launch configuration."""
    case = ci.case_c1(level)
    say(f"c1 512x1024 level {level}: 3 steps FP64 + diagnostics")
    rng = np.random.default_rng(case.seed)
    w0 = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    errs, w, w_or = _trajectory_errors(case, w0, F, 3)
    say(f"  per-step rel L2 = {errs}")
    assert errs.max() < TOL64
    g, _ = oracle_setup(case)
    from paper_1308_3290_amd.api import Basin, config_from_case
    b = Basin(config_from_case(case))
    wd = to_dev(w)
    psi = b.solve(wd)
    diag = to_np(b.diagnostics(wd, psi))
    psi_or = om.cgp_psi(w, g, level)
    E, Z = odiag.energy(psi_or, g), odiag.enstrophy(w, g)
    say(f"  E gpu {diag[0]:.12e} oracle {E:.12e}; Z gpu {diag[1]:.12e} oracle {Z:.12e}")
    assert abs(diag[0] - E) < 1e-11 * abs(E)
    assert abs(diag[1] - Z) < 1e-12 * abs(Z)
    # the reduction order is fixed: the same bits on every call
    assert np.array_equal(to_np(b.diagnostics(wd, psi)), diag)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_c2_full_size_two_layer_steps(level):
    case = ci.case_c2(level)
    say(f"c2 512x1024 two-layer level {level}: 2 steps FP64")
    rng = np.random.default_rng(case.seed)
    Q0 = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    errs, _, _ = _trajectory_errors(case, Q0, F, 2, layers=2)
    say(f"  per-step rel L2 = {errs}")
    assert errs.max() < TOL64


def test_psi_out_and_input_ring_ignored():
    case = ci.make_case(64, 128, level=1)
    g, phys = oracle_setup(case)
    w0 = random_state(case, 9, 1e-2)
    F = ci.forcing_field(case)
    dirty = w0.copy()
    dirty[0, :] = 5.0
    dirty[:, -1] = -3.0
    b = _basin(case)
    wd = to_dev(dirty)
    psi = torch.empty_like(wd)
    b.step(wd, to_dev(F), nsteps=2, psi_out=psi)
    ref = om.step(om.step(w0, F, g, 1, phys, case.dt), F, g, 1, phys, case.dt)
    assert rel_l2(to_np(wd), ref) < TOL64
    assert rel_l2(to_np(psi), om.cgp_psi(ref, g, 1)) < 1e-12
    out = to_np(wd)
    assert np.all(out[[0, -1], :] == 0) and np.all(out[:, [0, -1]] == 0)


def test_zero_steps_is_identity():
    case = ci.make_case(32, 64, level=1)
    b = _basin(case)
    w0 = random_state(case, 1)
    wd = to_dev(w0)
    b.step(wd, to_dev(ci.forcing_field(case)), nsteps=0)
    assert np.array_equal(to_np(wd), w0)


def test_diagnostics_two_layer():
    c2 = ci.case_c2(1)
    case = ci.make_case(64, 128, level=1, nlayers=2, f1=c2.f1, f2=c2.f2, drag=c2.drag)
    g, phys = oracle_setup(case)
    Q = random_state(case, 3)
    psi = om.cgp_psi_two_layer(Q, g, 1, phys)
    b = _basin(case)
    d = to_np(b.diagnostics(to_dev(Q), to_dev(psi)))
    for l in range(2):
        assert abs(d[2 * l] - odiag.energy(psi[l], g)) < 1e-12 * odiag.energy(psi[l], g)
        assert abs(d[2 * l + 1] - odiag.enstrophy(Q[l], g)) < 1e-12 * odiag.enstrophy(Q[l], g)


def test_check_finite_flags_nan_and_inf():
    case = ci.make_case(32, 64)
    b = _basin(case)
    w = to_dev(random_state(case, 2))
    assert int(b.check_finite(w).item()) == 0
    w[5, 7] = float("nan")
    assert int(b.check_finite(w).item()) == 1
    w[5, 7] = float("inf")
    assert int(b.check_finite(w).item()) == 1


def test_assert_finite_returns_the_nonfinite_status():
    from paper_1308_3290_amd._lib import CGP_ERR_NONFINITE, CGPError
    case = ci.make_case(32, 64)
    b = _basin(case)
    w = to_dev(random_state(case, 2))
    b.assert_finite(w)
    w[3, 4] = float("-inf")
    with pytest.raises(CGPError) as ei:
        b.assert_finite(w)
    assert ei.value.status == CGP_ERR_NONFINITE


def test_blow_up_is_detected():
    """A far too large dt drives the state non-finite; the finite check reports it."""
    case = ci.make_case(64, 128, level=0, dt=0.1)
    b = _basin(case)
    w = to_dev(random_state(case, 4))
    F = to_dev(ci.forcing_field(case))
    b.step(w, F, nsteps=300)
    assert int(b.check_finite(w).item()) == 1


def test_steps_are_deterministic():
    case = ci.make_case(96, 192, level=1)
    b = _basin(case)
    w0 = random_state(case, 8, 1e-2)
    F = to_dev(ci.forcing_field(case))
    a = to_dev(w0)
    c = to_dev(w0)
    b.step(a, F, nsteps=5)
    b.step(c, F, nsteps=5)
    assert torch.equal(a, c)


@pytest.mark.parametrize("nx,ny,level,layers", [
    (96, 192, 0, 1), (96, 192, 1, 1), (96, 192, 2, 1), (256, 512, 0, 1), (256, 512, 1, 1),
    (256, 512, 2, 1), (512, 256, 3, 1), (256, 512, 1, 2), (256, 512, 2, 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_steps_split_over_calls_give_the_same_bits(nx, ny, level, layers, dtype):
    """Six steps in one call, in calls of 1, 2 and 3 steps, and through the
    captured-graph path agree bit for bit: the spectra a fused step leaves for
    the next one equal those the first step of a call computes itself, and the
    rotation of the state through the stage buffers does not matter."""
    from paper_1308_3290_amd.api import Ensemble, config_from_case
    if layers == 2:
        c2 = ci.case_c2(level)
        case = ci.make_case(nx, ny, level=level, nlayers=2, f1=c2.f1, f2=c2.f2, drag=c2.drag,
                            dt=2.5e-5)
    else:
        case = ci.make_case(nx, ny, level=level, dt=1e-4)
    say(f"{nx}x{ny} level {level} layers {layers} {dtype}: 6 steps in one call vs 1+2+3 vs graph")
    tdt = _tdt(dtype)
    w0 = random_state(case, 21, 1e-2)
    F = to_dev(ci.forcing_field(case), tdt)
    b = _basin(case, dtype)
    one = to_dev(w0, tdt)
    b.step(one, F, nsteps=6)
    split = to_dev(w0, tdt)
    for n in (1, 2, 3):
        b.step(split, F, nsteps=n)
    ens = Ensemble([config_from_case(case, dtype)])
    g = to_dev(w0, tdt).reshape(-1).contiguous()
    Fg = F.reshape(-1).contiguous()
    if layers == 2:  # packed ensemble fields hold both layers (layer 2 forcing unused)
        Fg = torch.cat([Fg, torch.zeros_like(Fg)])
    side = torch.cuda.Stream()  # graphs are captured on a non-default stream
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ens.step(g, Fg, nsteps=2, use_graph=True)
        ens.step(g, Fg, nsteps=4, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(one, split)
    assert torch.equal(one.reshape(-1), g)


# ----------------------------------------------------------------- ensemble
def _members(dtype):
    sizes = [(64, 128, 1), (96, 192, 1), (32, 64, 1), (128, 256, 1), (48, 96, 1)]
    res = [200.0, 350.0, 800.0, 500.0, 650.0]
    out = []
    for (nx, ny, lv), re in zip(sizes, res):
        out.append(ci.make_case(nx, ny, level=lv, inv_re=1.0 / re, dt=2.5e-5, dtype=dtype))
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_ensemble_matches_single_basins_and_oracle(dtype, use_graph):
    from paper_1308_3290_amd.api import Ensemble, config_from_case
    say(f"ensemble dtype={dtype} graph={use_graph}")
    cases = _members(dtype)
    rng = np.random.default_rng(33)
    w0s = [ci.initial_field(c, rng, 1e-2) for c in cases]
    amps = [277.0 * (1 + 0.1 * k) for k in range(len(cases))]
    Fs = [ci.forcing_field(c, a) for c, a in zip(cases, amps)]
    ens = Ensemble([config_from_case(c) for c in cases])
    W = ens.pack(w0s)
    Fp = ens.pack(Fs)
    nsteps = 6
    # two calls: the graph is captured on the first and replayed on both
    # (graphs need a non-default stream)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ens.step(W, Fp, nsteps=nsteps // 2, use_graph=use_graph)
        ens.step(W, Fp, nsteps=nsteps - nsteps // 2, use_graph=use_graph)
    torch.cuda.synchronize()
    tdt = _tdt(dtype)
    for m, c in enumerate(cases):
        b = _basin(c, dtype)
        ws = to_dev(w0s[m], tdt)
        b.step(ws, to_dev(Fs[m], tdt), nsteps=nsteps)
        got = ens.member_view(W, m)
        assert torch.equal(got, ws), f"member {m} differs from its single-basin run"
        g, phys = oracle_setup(c)
        w_or = w0s[m]
        for _ in range(nsteps):
            w_or = om.step(w_or, Fs[m], g, c.level, phys, c.dt)
        err = rel_l2(to_np(got), w_or)
        say(f"  member {m} {c.nx}x{c.ny}: rel L2 vs oracle {err:.3e}")
        assert err < (TOL64 if dtype == "f64" else TOL32)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_chained_ensemble_graph_matches_single_basins(dtype):
    """Members of three sizes with compile-time transform lengths: each size is
    one chain of pass B and fused launches, and a captured step runs the
    chains on separate streams.  Every member must equal its single-basin
    run bit for bit, over 7 steps (a rotation graph plus single steps)."""
    from paper_1308_3290_amd.api import Ensemble, config_from_case
    sizes = [(128, 256), (256, 512), (128, 256), (384, 768), (256, 512)]
    cases = [ci.make_case(nx, ny, level=1, inv_re=1.0 / (300 + 50 * k), dt=2.5e-5, dtype=dtype)
             for k, (nx, ny) in enumerate(sizes)]
    rng = np.random.default_rng(44)
    w0s = [ci.initial_field(c, rng, 1e-2) for c in cases]
    Fs = [ci.forcing_field(c) for c in cases]
    ens = Ensemble([config_from_case(c) for c in cases])
    W = ens.pack(w0s)
    Fp = ens.pack(Fs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ens.step(W, Fp, nsteps=4, use_graph=True)
        ens.step(W, Fp, nsteps=3, use_graph=True)
    torch.cuda.synchronize()
    tdt = _tdt(dtype)
    for m, c in enumerate(cases):
        b = _basin(c, dtype)
        ws = to_dev(w0s[m], tdt)
        b.step(ws, to_dev(Fs[m], tdt), nsteps=7)
        assert torch.equal(ens.member_view(W, m), ws), f"member {m} differs"


def test_ensemble_of_mixed_coarsening_factors():
    """Members at c = 1, 2, 4 and 8 (compile-time transform lengths of 128 and
    256 points and runtime ones of 64 and 96) in one ensemble: the fused pass
    runs one launch per (c, length) group; every member equals its
    single-basin run bit for bit over graph replays and follows the oracle."""
    from paper_1308_3290_amd.api import Ensemble, config_from_case
    sizes = [(128, 256, 0), (128, 256, 1), (256, 512, 2), (512, 256, 3), (256, 512, 3),
             (96, 192, 1)]
    cases = [ci.make_case(nx, ny, level=lv, inv_re=1.0 / (300 + 60 * k), dt=1e-4)
             for k, (nx, ny, lv) in enumerate(sizes)]
    say("ensemble of levels 0, 1, 2, 3: 5 steps, graph replays")
    rng = np.random.default_rng(55)
    w0s = [ci.initial_field(c, rng, 1e-2) for c in cases]
    Fs = [ci.forcing_field(c) for c in cases]
    ens = Ensemble([config_from_case(c) for c in cases])
    W = ens.pack(w0s)
    Fp = ens.pack(Fs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ens.step(W, Fp, nsteps=3, use_graph=True)
        ens.step(W, Fp, nsteps=2, use_graph=True)
    torch.cuda.synchronize()
    for m, c in enumerate(cases):
        b = _basin(c)
        ws = to_dev(w0s[m])
        b.step(ws, to_dev(Fs[m]), nsteps=5)
        got = ens.member_view(W, m)
        assert torch.equal(got, ws), f"member {m} differs from its single-basin run"
        g, phys = oracle_setup(c)
        w_or = w0s[m]
        for _ in range(5):
            w_or = om.step(w_or, Fs[m], g, c.level, phys, c.dt)
        err = rel_l2(to_np(got), w_or)
        say(f"  member {m} {c.nx}x{c.ny} level {c.level}: rel L2 vs oracle {err:.3e}")
        assert err < TOL64


# ----------------------------------------------------------------- adjoint
def test_adjoint_segment_matches_oracle():
    case = ci.make_case(32, 64, level=1, dt=2.5e-4)
    g, phys = oracle_setup(case)
    w0 = random_state(case, 12, 1.0)
    F = ci.forcing_field(case)
    lam = random_state(case, 13, 1.0)
    nsteps = 3
    states = oadj.trajectory(w0, F, g, 1, phys, case.dt, nsteps)
    l_or = lam.copy()
    gF_or = np.zeros_like(lam)
    for n in range(nsteps - 1, -1, -1):
        l_or, gg = oadj.step_adjoint(states[n], F, l_or, g, 1, phys, case.dt)
        gF_or += gg
    b = _basin(case)
    ld = to_dev(lam)
    gF = torch.zeros_like(ld)
    b.adjoint_step(to_dev(w0), to_dev(F), nsteps, ld, gF)
    torch.cuda.synchronize()
    e1, e2 = rel_l2(to_np(ld), l_or), rel_l2(to_np(gF), gF_or)
    say(f"adjoint vs oracle: lambda {e1:.3e}, grad F {e2:.3e}")
    assert e1 < 1e-11 and e2 < 1e-11


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_adjoint_dot_product_with_oracle_tlm(level):
    case = ci.make_case(64, 128, level=level, dt=1e-4)
    g, phys = oracle_setup(case)
    w0 = random_state(case, 20, 1.0)
    F = ci.forcing_field(case)
    dw = random_state(case, 21)
    dF = random_state(case, 22)
    lam = random_state(case, 23)
    _, tl = oadj.step_tlm(w0, dw, F, dF, g, level, phys, case.dt)
    b = _basin(case)
    ld = to_dev(lam)
    gF = torch.zeros_like(ld)
    b.adjoint_step(to_dev(w0), to_dev(F), 1, ld, gF)
    lhs = float(np.sum(tl * lam))
    rhs = float(np.sum(dw * to_np(ld)) + np.sum(dF * to_np(gF)))
    say(f"dot product level {level}: {lhs:.15e} vs {rhs:.15e}")
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_c4_gradient_matches_finite_differences():
    """Full adjoint workload: 256 x 512, level 1, 200 steps, checkpoints every 20,
    final-time misfit at 1% of interior nodes; 20 random unit directions."""
    from paper_1308_3290_amd.api import Basin, Trajectory, config_from_case
    p = ci.adjoint_c4()
    c = p.case
    say("c4: 256x512 adjoint, 200 steps, ckpt 20, 20 FD directions")
    b = Basin(config_from_case(c))
    idx = torch.as_tensor(p.obs_index, device="cuda")
    obs = to_dev(p.obs_value)

    def final_at_obs(w0, F):
        w = w0.clone()
        b.step(w, F, nsteps=c.nsteps)
        return w.view(-1)[idx]

    w0 = to_dev(p.omega0).requires_grad_(True)
    F = to_dev(p.forcing).requires_grad_(True)
    wT = Trajectory.apply(w0, F, b, c.nsteps, p.ckpt_every)
    L = ((wT.view(-1)[idx] - obs) ** 2).mean()
    L.backward()
    gw, gF = w0.grad.detach(), F.grad.detach()
    K = idx.numel()
    rows = []
    for d in range(p.dir_forcing.shape[0]):
        dW, dF = to_dev(p.dir_omega[d]), to_dev(p.dir_forcing[d])
        an = float((gw * dW).sum().item() + (gF * dF).sum().item())
        fds = []
        for eps in (1e-6, 1e-4):
            vp = final_at_obs(w0.detach() + eps * dW, F.detach() + eps * dF)
            vm = final_at_obs(w0.detach() - eps * dW, F.detach() - eps * dF)
            # central difference (L+ - L-)/(2 eps) with L+ - L- evaluated as
            # (1/K) sum (v+ - v-)(v+ + v- - 2 o): the same quotient without the
            # cancellation of two O(1) losses
            fds.append(float(((vp - vm) * (vp + vm - 2 * obs)).sum().item()) / K / (2 * eps))
        rows.append((an, fds[0], fds[1]))
        say(f"  dir {d:2d}: adjoint {an:+.12e}  FD(1e-6) {fds[0]:+.12e}  FD(1e-4) {fds[1]:+.12e}"
            f"  rel {abs(fds[0] - an) / abs(an):.1e} / {abs(fds[1] - an) / abs(an):.1e}")
    an = np.array([r[0] for r in rows])
    f6 = np.array([r[1] for r in rows])
    f4 = np.array([r[2] for r in rows])
    agg6 = np.linalg.norm(f6 - an) / np.linalg.norm(an)
    worst4 = np.max(np.abs(f4 - an) / np.abs(an))
    say(f"  eps 1e-6: aggregate rel {agg6:.2e}, max abs err / max |dL| "
        f"{np.max(np.abs(f6 - an)) / np.max(np.abs(an)):.2e};  eps 1e-4: worst rel {worst4:.2e}")
    # eps = 1e-6 sits at the roundoff floor of two 200-step trajectories
    # (~1e-16 |omega| / eps relative to the directional derivative): bound the
    # aggregate; eps = 1e-4 lowers that floor 100x and is checked per direction.
    assert agg6 < 2e-6
    assert np.max(np.abs(f6 - an)) < 1e-5 * np.max(np.abs(an))
    worst = worst4
    assert worst < 1e-6
