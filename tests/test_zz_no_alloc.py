"""cgp_step_noalloc (workspace in the library's static device scratch) against
cgp_step on a caller workspace: two calls in a row on one GPU, the second with
a smaller basin, each compared with a fresh handle's cgp_step on the same
inputs (FP64: relative L2 <= 1e-11; the same kernels and tables, so the bits
are expected to agree as well), plus the psi output and an FP32 call."""
import numpy as np
import pytest
import torch

import cgp_inputs as ci

from gpu_common import random_state, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_3290_amd import _lib
    _lib.load()
    yield
    torch.cuda.synchronize()


def _reference(case, w0, F, nsteps, dtype, psi=False):
    from paper_1308_3290_amd.api import Basin, config_from_case
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = Basin(config_from_case(case, dtype))
    w = to_dev(w0, tdt)
    p = torch.empty_like(w) if psi else None
    b.step(w, to_dev(F, tdt), nsteps=nsteps, psi_out=p)
    torch.cuda.synchronize()
    b.close()
    return w, p


def _noalloc(case, w0, F, nsteps, dtype, psi=False):
    from paper_1308_3290_amd.api import cgp_step_noalloc, config_from_case
    tdt = torch.float64 if dtype == "f64" else torch.float32
    w = to_dev(w0, tdt)
    p = torch.empty_like(w) if psi else None
    cgp_step_noalloc(config_from_case(case, dtype), w, to_dev(F, tdt), p, nsteps)
    torch.cuda.synchronize()
    return w, p


def test_noalloc_matches_cgp_step_on_two_calls_second_smaller():
    big = ci.case_c1(1)
    small = ci.make_case(64, 128, level=1, dt=1e-4)
    for case, nsteps, seed in ((big, 7, 1), (small, 5, 2)):
        say(f"noalloc {case.nx}x{case.ny} level {case.level}: {nsteps} steps")
        w0 = random_state(case, seed, 1.0)
        F = ci.forcing_field(case)
        got, gp = _noalloc(case, w0, F, nsteps, "f64", psi=True)
        ref, rp = _reference(case, w0, F, nsteps, "f64", psi=True)
        e, ep = rel_l2(to_np(got), to_np(ref)), rel_l2(to_np(gp), to_np(rp))
        say(f"  rel L2 omega {e:.3e}, psi {ep:.3e}, bitwise {torch.equal(got, ref)}")
        assert e <= 1e-11 and ep <= 1e-11
        assert torch.equal(got, ref) and torch.equal(gp, rp)


def test_noalloc_other_configurations():
    """Two layers at 512 x 1024 (the largest workspace that fits), then an FP32
    basin, then a one-layer basin again: each call sets up its own tables."""
    c2 = ci.case_c2(0)
    cases = [(c2, 2, "f64"), (ci.make_case(96, 192, level=2, dt=1e-4), 4, "f32"),
             (ci.make_case(128, 256, level=0, dt=1e-4), 3, "f64")]
    for case, nsteps, dtype in cases:
        say(f"noalloc {case.nx}x{case.ny} layers {case.nlayers} level {case.level} {dtype}")
        w0 = random_state(case, 3, 1e-2)
        F = ci.forcing_field(case)
        got, _ = _noalloc(case, w0, F, nsteps, dtype)
        ref, _ = _reference(case, w0, F, nsteps, dtype)
        e = rel_l2(to_np(got), to_np(ref))
        say(f"  rel L2 {e:.3e}")
        assert e <= (1e-11 if dtype == "f64" else 1e-4)
        assert torch.equal(got, ref)


def test_noalloc_rejects_a_workspace_above_the_scratch():
    from paper_1308_3290_amd._lib import CGPError
    from paper_1308_3290_amd.api import cgp_step_noalloc, make_config
    cfg = make_config(1024, 1024, level=0, nlayers=2, f1=10.0, f2=5.0, inv_re=1e-3, dt=1e-5)
    w = torch.zeros(2 * 1025 * 1025, dtype=torch.float64, device="cuda")
    with pytest.raises(CGPError, match="static scratch"):
        cgp_step_noalloc(cfg, w, w[: 1025 * 1025], None, 1)
