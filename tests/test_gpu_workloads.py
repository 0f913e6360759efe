"""GPU parity of the workloads themselves against the FP64 oracle.

The library's own configurations at the sizes the workloads run:
  - the c = 2 stage kernels of the ensemble members (256 x 512, 384 x 768:
    row transforms of 256 and 384 points, column transforms of 512 and 768)
    and of 512 x 1024, in FP64 and FP32, 30 steps each;
  - the 512 x 1024 one-layer workload at levels 0, 1, 2: per-step parity over
    the first 100 steps, then the energy and enstrophy every 10 steps up to
    step 1000 against the oracle's series (tests/golden/series_512x1024.json,
    written by tests/golden/make_series.py from the oracle alone);
  - the 512 x 1024 two-layer workload at levels 0, 1, 2: the same, 100 steps,
    then E and Z of both layers up to step 500;
  - the 64-member ensemble in FP64 and FP32 (graph replays), every member
    against its own oracle run at steps 1, 2, 5 and 10;
  - the adjoint workload's forward trajectory (256 x 512, 200 steps) and its
    gradient, on a shortened segment, against the oracle's reverse sweep.

Tolerances: per-step relative L2 of the state <= 1e-11 (FP64), <= 1e-4
(FP32); E and Z relative <= 1e-9 beyond the per-step horizon.
"""
import json
import os

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
TOL_SERIES = 1e-9
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "series_512x1024.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_3290_amd import _lib
    _lib.load()
    yield
    torch.cuda.synchronize()


def _tdt(dtype):
    return torch.float64 if dtype == "f64" else torch.float32


def _basin(case, dtype=None):
    from paper_1308_3290_amd.api import Basin, config_from_case
    return Basin(config_from_case(case, dtype))


def _series(name, level):
    doc = json.load(open(GOLDEN))
    for r in doc["runs"]:
        if r["workload"] == name and r["level"] == level:
            return r
    raise KeyError((name, level))


def _oracle_step(case, g, phys):
    if case.nlayers == 1:
        return lambda w, F: om.step(w, F, g, case.level, phys, case.dt)
    return lambda w, F: om.step_two_layer(w, F, g, case.level, phys, case.dt)


def _oracle_stats(case, g, phys, w):
    if case.nlayers == 1:
        psi = om.cgp_psi(w, g, case.level)
        return [[odiag.energy(psi, g), odiag.enstrophy(w, g)]]
    psi = om.cgp_psi_two_layer(w, g, case.level, phys)
    return [[odiag.energy(psi[l], g), odiag.enstrophy(w[l], g)] for l in range(2)]


# ------------------------------------------------------------ stage kernels at c = 2
@pytest.mark.parametrize("nx,ny,dtype", [(256, 512, "f64"), (384, 768, "f64"),
                                         (256, 512, "f32"), (384, 768, "f32"),
                                         (512, 1024, "f32")])
def test_c2_stage_kernels_of_the_workload_sizes(nx, ny, dtype):
    """30 steps at level 1 from an O(1) noise state (the Jacobian matters from
    the first step), per-step parity with the FP64 oracle."""
    case = ci.make_case(nx, ny, level=1, dt=2.5e-5, dtype=dtype)
    say(f"{nx}x{ny} level 1 {dtype}: 30 steps vs oracle")
    g, phys = oracle_setup(case)
    w0 = random_state(case, 61, 1.0)
    F = ci.forcing_field(case)
    b = _basin(case, dtype)
    tdt = _tdt(dtype)
    wd, Fd = to_dev(w0, tdt), to_dev(F, tdt)
    w = w0
    errs = []
    for n in range(30):
        b.step(wd, Fd, nsteps=1)
        w = om.step(w, F, g, 1, phys, case.dt)
        errs.append(rel_l2(to_np(wd), w))
    say(f"  max per-step rel L2 = {max(errs):.3e}")
    assert max(errs) < (TOL64 if dtype == "f64" else TOL32)


# ------------------------------------------------------------ 512 x 1024 horizons
def _horizon(case, nsteps_total, name):
    """Per-step parity over the first 100 steps, then E and Z every 10 steps
    against the oracle's stored series up to nsteps_total."""
    g, phys = oracle_setup(case)
    rng = np.random.default_rng(case.seed)
    w0 = ci.initial_field(case, rng)
    F = ci.forcing_field(case)
    ostep = _oracle_step(case, g, phys)
    ser = _series(name, case.level)
    assert ser["nsteps"] == nsteps_total and ser["dt"] == case.dt
    ref = dict(zip(ser["steps"], ser["E_Z"]))
    b = _basin(case)
    wd, Fd = to_dev(w0), to_dev(F)
    w = w0
    errs = []
    for n in range(1, 101):
        b.step(wd, Fd, nsteps=1)
        w = ostep(w, F)
        errs.append(rel_l2(to_np(wd), w))
    say(f"  steps 1-100: max per-step rel L2 = {max(errs):.3e}")
    assert max(errs) < TOL64
    # the stored series is the oracle's: its step-100 entry equals the
    # oracle state computed here
    here = _oracle_stats(case, g, phys, w)
    assert np.allclose(here, ref[100], rtol=1e-12, atol=0)
    worst = 0.0
    n = 100
    while n < nsteps_total:
        b.step(wd, Fd, nsteps=10)
        n += 10
        psi = b.solve(wd)
        d = to_np(b.diagnostics(wd, psi)).reshape(-1, 2)
        e = np.abs(d - np.array(ref[n])) / np.abs(np.array(ref[n]))
        worst = max(worst, float(e.max()))
        assert e.max() < TOL_SERIES, (n, d, ref[n])
    say(f"  steps 110-{nsteps_total}: max rel error of E, Z = {worst:.3e}")
    assert np.all(np.isfinite(to_np(wd)))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_c1_horizon_100_steps_then_series_to_1000(level):
    case = ci.case_c1(level)
    say(f"512x1024 one layer level {level}: 100 steps per-step, E/Z to 1000")
    _horizon(case, 1000, "c1")


@pytest.mark.parametrize("level", [0, 1, 2])
def test_c2_horizon_100_steps_then_series_to_500(level):
    case = ci.case_c2(level)
    say(f"512x1024 two layers level {level}: 100 steps per-step, E/Z to 500")
    _horizon(case, 500, "c2")


# ------------------------------------------------------------ the 64-member ensemble
def test_c3_ensemble_members_follow_the_oracle():
    """Both dtypes of the 64-member workload, graph replays on a side stream
    (the launch mode of the benchmark); snapshots at steps 1, 2, 5, 10, each
    member compared with its own oracle run."""
    from paper_1308_3290_amd.api import Ensemble, config_from_case
    marks = (1, 2, 5, 10)
    snaps = {}
    members = None
    for dtype in ("f64", "f32"):
        members = ci.ensemble_c3(64, dtype=dtype)
        ens = Ensemble([config_from_case(m.case) for m in members])
        W = ens.pack([m.omega0 for m in members])
        Fp = ens.pack([m.forcing for m in members])
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        done = 0
        snaps[dtype] = {}
        with torch.cuda.stream(side):
            for k in marks:
                ens.step(W, Fp, nsteps=k - done, use_graph=True)
                done = k
                snaps[dtype][k] = W.clone()
        torch.cuda.synchronize()
        snaps[dtype]["ens"] = ens
        say(f"ensemble {dtype}: {len(members)} members, {ens.total} packed elements, 10 steps")
    worst = {"f64": 0.0, "f32": 0.0}
    for m, mem in enumerate(members):
        c = mem.case
        g, phys = oracle_setup(c)
        w = mem.omega0
        n = 0
        for k in marks:
            while n < k:
                w = om.step(w, mem.forcing, g, c.level, phys, c.dt)
                n += 1
            for dtype in ("f64", "f32"):
                got = to_np(snaps[dtype]["ens"].member_view(snaps[dtype][k], m))
                err = rel_l2(got, w)
                worst[dtype] = max(worst[dtype], err)
                assert err < (TOL64 if dtype == "f64" else TOL32), (m, c.nx, c.ny, k, dtype, err)
    say(f"  worst member rel L2: FP64 {worst['f64']:.3e}, FP32 {worst['f32']:.3e}")


# ------------------------------------------------------------ the adjoint workload
def test_c4_forward_trajectory_matches_oracle():
    p = ci.adjoint_c4()
    c = p.case
    say("c4 forward: 256x512 level 1, 200 steps, per-step parity")
    g, phys = oracle_setup(c)
    b = _basin(c)
    wd, Fd = to_dev(p.omega0), to_dev(p.forcing)
    w = p.omega0
    errs = []
    for n in range(c.nsteps):
        b.step(wd, Fd, nsteps=1)
        w = om.step(w, p.forcing, g, c.level, phys, c.dt)
        errs.append(rel_l2(to_np(wd), w))
    say(f"  max per-step rel L2 = {max(errs):.3e}")
    assert max(errs) < TOL64


def test_c4_gradient_matches_oracle_gradient():
    """The autograd trajectory (checkpoints, recomputed segments, the library's
    adjoint) against the oracle's full reverse sweep: 256 x 512, level 1,
    10 steps, checkpoint every 5, the c4 loss."""
    from paper_1308_3290_amd.api import Trajectory
    p = ci.adjoint_c4(nsteps=10, ckpt_every=5, ndir=1)
    c = p.case
    say("c4 gradient: 256x512, 10 steps, ckpt 5, vs oracle reverse sweep")
    g, phys = oracle_setup(c)
    L_or, gw_or, gF_or = oadj.loss_and_gradient(p.omega0, p.forcing, p.obs_index, p.obs_value,
                                                g, c.level, phys, c.dt, c.nsteps)
    b = _basin(c)
    idx = torch.as_tensor(p.obs_index, device="cuda")
    obs = to_dev(p.obs_value)
    w0 = to_dev(p.omega0).requires_grad_(True)
    F = to_dev(p.forcing).requires_grad_(True)
    wT = Trajectory.apply(w0, F, b, c.nsteps, p.ckpt_every)
    L = ((wT.view(-1)[idx] - obs) ** 2).mean()
    L.backward()
    e_L = abs(float(L.item()) - L_or) / abs(L_or)
    e_w = rel_l2(to_np(w0.grad), gw_or)
    e_F = rel_l2(to_np(F.grad), gF_or)
    say(f"  loss {e_L:.2e}, dL/domega0 {e_w:.2e}, dL/dF {e_F:.2e}")
    assert e_L < 1e-12 and e_w < 1e-11 and e_F < 1e-11


# ------------------------------------------------------------ handles of several sizes
def test_large_handle_keeps_working_after_a_small_one_is_created():
    """Kernel attributes are process-wide: creating a small handle after a
    512 x 1024 one must not restrict the launches of the large one."""
    big = ci.case_c1(1)
    g, phys = oracle_setup(big)
    rng = np.random.default_rng(big.seed)
    w0 = ci.initial_field(big, rng)
    F = ci.forcing_field(big)
    b_big = _basin(big)
    b_small = _basin(ci.make_case(64, 128, level=1))
    b_small2 = _basin(ci.make_case(64, 128, level=0, nlayers=2, f1=10.0, f2=5.0))
    wd = to_dev(w0)
    b_big.step(wd, to_dev(F), nsteps=2)
    ref = om.step(om.step(w0, F, g, 1, phys, big.dt), F, g, 1, phys, big.dt)
    err = rel_l2(to_np(wd), ref)
    say(f"512x1024 after two small handles: rel L2 {err:.3e}")
    assert err < TOL64
    del b_small, b_small2
