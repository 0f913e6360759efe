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


# fused one-layer step at c = 2, 1, 4; (1024, 64, 1): rows too wide for the
# fused kernel (unfused passes); two layers: (64, 128, 1) unfused, (128, 256, 1)
# the fused two-layer kernel
@pytest.mark.parametrize("nx,ny,level,layers,c", [
    (64, 128, 1, 1, 0.01), (64, 128, 0, 1, 0.01), (64, 128, 2, 1, 0.01),
    (1024, 64, 1, 1, 0.01), (64, 128, 1, 2, 0.003), (128, 256, 1, 2, 0.003)])
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
