"""GPU parity of the adaptive CFL step (Sec. 4.2) with the oracle, through the
C ABI, and its bit-for-bit reproducibility over call splits, graphs and
ensembles."""
import numpy as np
import pytest
import torch

import cgp_inputs as ci
from gpu_common import oracle_setup, random_state, rel_l2, say, to_dev, to_np
from oracle import cfl as ocfl

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


def _case(nx, ny, level, layers, c, dt_max=1e-3, dtype="f64"):
    if layers == 2:
        c2 = ci.case_c2(level)
        return ci.make_case(nx, ny, level=level, nlayers=2, f1=c2.f1, f2=c2.f2, drag=c2.drag,
                            dt=dt_max, cfl=c, dtype=dtype)
    return ci.make_case(nx, ny, level=level, dt=dt_max, cfl=c, dtype=dtype)


def _run(case, nsteps, dtype="f64"):
    """Per-step rel L2 errors vs the oracle, GPU and oracle dt sequences, GPU time."""
    from paper_1308_3290_amd.api import Basin, config_from_case
    tdt = torch.float64 if dtype == "f64" else torch.float32
    g, phys = oracle_setup(case)
    w0 = random_state(case, 5, 1e-2)
    F = ci.forcing_field(case)
    ref = []
    _, dts = ocfl.run_adaptive(w0, F, g, case.level, phys, case.cfl, case.dt, nsteps,
                               nlayers=case.nlayers, callback=lambda n, w, dt: ref.append(w))
    b = Basin(config_from_case(case, dtype))
    w = to_dev(w0, tdt)
    Fd = to_dev(F, tdt)
    errs, gdts = [], []
    for n in range(nsteps):
        b.step(w, Fd, nsteps=1)
        ts = b.time_state()
        torch.cuda.synchronize()
        gdts.append(float(ts[0]))
        errs.append(rel_l2(to_np(w), ref[n]))
    t = float(b.time_state()[1])
    return np.array(errs), np.array(gdts), np.array(dts), t


# fused one-layer step at c = 2, 1, 4, 8; (1024, 64, 1): rows too wide for the
# fused kernel (unfused passes); two layers: (64, 128, 1) unfused, (128, 256, 1)
# and (64, 128, 0) the fused two-layer kernel at c = 2 and 1
@pytest.mark.parametrize("nx,ny,level,layers,c", [
    (64, 128, 1, 1, 0.01), (64, 128, 0, 1, 0.01), (64, 128, 2, 1, 0.01),
    (512, 256, 3, 1, 0.01), (1024, 64, 1, 1, 0.01), (64, 128, 1, 2, 0.003), (128, 256, 1, 2, 0.003),
    (64, 128, 0, 2, 0.003)])
def test_adaptive_trajectory_matches_oracle(nx, ny, level, layers, c):
    case = _case(nx, ny, level, layers, c)
    say(f"adaptive {nx}x{ny} level {level} layers {layers} cfl {c}: 30 steps FP64")
    errs, gdts, dts, t = _run(case, 30)
    say(f"  max per-step rel L2 = {errs.max():.3e}; dt {dts[0]:.3g} .. {dts[-1]:.3g}")
    assert errs.max() < TOL64
    assert gdts[0] == case.dt                       # the first step takes dt itself
    assert np.abs(gdts / dts - 1).max() < 1e-12     # the same step sizes
    assert t == pytest.approx(dts.sum(), rel=1e-12)
    assert len(set(dts.tolist())) > 5 and dts.min() < 0.8 * case.dt  # the steps adapt


def test_adaptive_trajectory_fp32():
    case = _case(64, 128, 1, 1, 0.01, dtype="f32")
    errs, gdts, dts, _ = _run(case, 30, dtype="f32")
    say(f"adaptive FP32 max per-step rel L2 = {errs.max():.3e}")
    assert errs.max() < TOL32
    assert np.abs(gdts / dts - 1).max() < TOL32


@pytest.mark.parametrize("nx,ny,level,layers", [(96, 192, 1, 1), (96, 192, 0, 1),
                                                (1024, 64, 1, 1), (128, 256, 1, 2)])
def test_adaptive_steps_split_over_calls_give_the_same_bits(nx, ny, level, layers):
    """Six adaptive steps in one call, in calls of 1, 2 and 3 steps, and through
    the captured-graph path give the same state and step state bit for bit."""
    from paper_1308_3290_amd.api import Basin, Ensemble, config_from_case
    case = _case(nx, ny, level, layers, 0.005)
    say(f"adaptive {nx}x{ny} level {level} layers {layers}: 6 steps, 1+2+3, graph")
    w0 = random_state(case, 21, 3e-2)
    F = to_dev(ci.forcing_field(case))
    b1 = Basin(config_from_case(case))
    one = to_dev(w0)
    b1.step(one, F, nsteps=6)
    b2 = Basin(config_from_case(case))
    split = to_dev(w0)
    for n in (1, 2, 3):
        b2.step(split, F, nsteps=n)
    ens = Ensemble([config_from_case(case)])
    g = to_dev(w0).reshape(-1).contiguous()
    Fg = F.reshape(-1).contiguous()
    if layers == 2:
        Fg = torch.cat([Fg, torch.zeros_like(Fg)])
    side = torch.cuda.Stream()  # graphs are captured on a non-default stream
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ens.step(g, Fg, nsteps=2, use_graph=True)
        ens.step(g, Fg, nsteps=4, use_graph=True)
    torch.cuda.synchronize()
    s1, s2, s3 = b1.time_state(), b2.time_state(), ens.time_state()[0]
    torch.cuda.synchronize()
    assert torch.equal(one, split) and torch.equal(one.reshape(-1), g)
    assert torch.equal(s1, s2) and torch.equal(s1, s3)
    assert float(s1[0]) < case.dt  # the last steps adapted


def test_ensemble_mixes_adaptive_and_fixed_members():
    """Members with and without adaptive steps in one ensemble take the steps
    they take alone, bit for bit."""
    from paper_1308_3290_amd.api import Basin, Ensemble, config_from_case
    cases = [_case(64, 128, 1, 1, 0.01), _case(96, 192, 1, 1, 0.0, dt_max=1e-4),
             _case(32, 64, 1, 1, 0.004)]
    ens = Ensemble([config_from_case(c) for c in cases])
    w0 = [random_state(c, 30 + i, 1e-2) for i, c in enumerate(cases)]
    F = [ci.forcing_field(c) for c in cases]
    Wp = ens.pack(w0).to(torch.float64)
    Fp = ens.pack(F).to(torch.float64)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ens.step(Wp, Fp, nsteps=10, use_graph=True)
    torch.cuda.synchronize()
    st = ens.time_state()
    for m, c in enumerate(cases):
        b = Basin(config_from_case(c))
        w = to_dev(w0[m])
        b.step(w, to_dev(F[m]), nsteps=10)
        ts = b.time_state()
        torch.cuda.synchronize()
        assert torch.equal(ens.member_view(Wp, m), w), m
        assert torch.equal(st[m], ts), m
    assert float(st[1][0]) == 1e-4 and float(st[1][1]) == pytest.approx(1e-3, rel=1e-14)
    assert float(st[0][0]) < 1e-3


# ----------------------------------------------------------------- time means (Sec. 5.1)
def test_accumulate_matches_numpy():
    from paper_1308_3290_amd.api import Basin, config_from_case
    case = _case(64, 128, 1, 1, 0.01)
    b = Basin(config_from_case(case))
    rng = np.random.default_rng(3)
    f = rng.standard_normal(case.shape)
    s0 = rng.standard_normal(case.shape)
    total = to_dev(s0)
    b.accumulate(to_dev(f), total, weight=0.3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(to_np(total), s0 + 0.3 * f, rtol=1e-15, atol=1e-15)
    # times_dt: the weight times the dt of the latest step (the configured dt
    # before any step)
    b.accumulate(to_dev(f), total, weight=2.0, times_dt=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(to_np(total), s0 + 0.3 * f + 2.0 * case.dt * f, rtol=1e-14,
                               atol=1e-14)


@pytest.mark.parametrize("nx,ny,level,layers", [(64, 128, 1, 1), (64, 128, 0, 1),
                                                (128, 256, 1, 2)])
def test_step_mean_matches_oracle_time_mean(nx, ny, level, layers):
    from oracle import statistics as ost
    from paper_1308_3290_amd.api import Basin, config_from_case
    case = _case(nx, ny, level, layers, 0.01 if layers == 1 else 0.003)
    say(f"time mean {nx}x{ny} level {level} layers {layers}: 5 + 12 adaptive steps")
    g, phys = oracle_setup(case)
    w0 = random_state(case, 11, 1e-2)
    F = ci.forcing_field(case)
    mw_ref, mp_ref, tsum_ref, _ = ost.time_mean(w0, F, g, level, phys, case.cfl, case.dt, 5, 12,
                                                nlayers=layers)
    means = []
    for use_graph in (False, True):
        b = Basin(config_from_case(case))
        w = to_dev(w0)
        Fd = to_dev(F)
        total = torch.zeros_like(w)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            b.step(w, Fd, nsteps=5, stream=side)
            t0 = b.time_state(side)[1].clone()
            b.step_mean(w, Fd, 12, total, use_graph=use_graph, stream=side)
            t1 = b.time_state(side)[1].clone()
        torch.cuda.synchronize()
        tsum = float(t1 - t0)
        mw = to_np(total) / tsum
        mp = to_np(b.solve(to_dev(mw)))
        means.append(total)
        assert tsum == pytest.approx(tsum_ref, rel=1e-12)
        assert rel_l2(mw, mw_ref) < TOL64 and rel_l2(mp, mp_ref) < TOL64
    assert torch.equal(means[0], means[1])  # graphs and direct launches agree


def test_long_run_driver_matches_oracle():
    """The statistics driver (spin-up, averaging window, energy history) on a
    short horizon, against the oracle's time mean over the same steps."""
    from oracle import statistics as ost
    from paper_1308_3290_amd.api import Basin, config_from_case
    from paper_1308_3290_amd.statistics import long_run
    case = _case(64, 128, 1, 1, 0.01)
    g, phys = oracle_setup(case)
    w0 = random_state(case, 12, 1e-2)
    F = ci.forcing_field(case)
    b = Basin(config_from_case(case))
    w = to_dev(w0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r = long_run(b, w, to_dev(F), t_spin=0.004, t_end=0.012, chunk=5, stream=side)
    say(f"long run: {r['steps_spin']} + {r['steps_avg']} steps, window {r['t0']:.4g}..{r['t1']:.4g}")
    assert r["steps_spin"] > 0 and r["steps_avg"] > 0 and r["t1"] >= 0.012
    mw_ref, mp_ref, tsum_ref, w_ref = ost.time_mean(w0, F, g, 1, phys, case.cfl, case.dt,
                                                    r["steps_spin"], r["steps_avg"])
    assert (r["t1"] - r["t0"]) == pytest.approx(tsum_ref, rel=1e-12)
    assert rel_l2(r["mean_omega"], mw_ref) < TOL64 and rel_l2(r["mean_psi"], mp_ref) < TOL64
    assert rel_l2(to_np(w), w_ref) < TOL64
    n = (r["steps_spin"] + r["steps_avg"]) // 5 + 1
    assert r["energy"].shape == (n, 1) and np.all(np.diff(r["times"]) > 0)


@pytest.mark.parametrize("nx,ny,level", [(16, 32, 0), (32, 64, 1), (64, 128, 2)])
def test_long_run_driver_at_the_fixed_16x32_elliptic_grid(nx, ny, level):
    """The driver on the shapes of the paper's fixed 16 x 32 elliptic grid
    comparison (Sec. 5.1: fine grids 16x32, 32x64 and 64x128 over one 16x32
    solve), Exp. I physics and inputs, a short window against the oracle."""
    from oracle import statistics as ost
    from paper_1308_3290_amd.api import Basin, config_from_case
    from paper_1308_3290_amd.statistics import long_run
    case, w0, F = ci.experiment_case("I", nx, ny, level, seed=1, cfl=0.5, dt_max=5e-4)
    g, phys = oracle_setup(case)
    b = Basin(config_from_case(case))
    w = to_dev(w0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r = long_run(b, w, to_dev(F), t_spin=0.02, t_end=0.06, chunk=10, stream=side)
    say(f"{nx}x{ny}:{level} long run: {r['steps_spin']} + {r['steps_avg']} steps")
    mw_ref, mp_ref, tsum_ref, w_ref = ost.time_mean(w0, F, g, level, phys, case.cfl, case.dt,
                                                    r["steps_spin"], r["steps_avg"])
    assert (r["t1"] - r["t0"]) == pytest.approx(tsum_ref, rel=1e-12)
    e = (rel_l2(r["mean_omega"], mw_ref), rel_l2(r["mean_psi"], mp_ref), rel_l2(to_np(w), w_ref))
    say(f"  rel L2 mean omega {e[0]:.2e}, mean psi {e[1]:.2e}, final state {e[2]:.2e}")
    assert max(e) < TOL64
