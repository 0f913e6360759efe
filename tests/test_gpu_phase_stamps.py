"""The measurement build (libcgp_stamps.so): its phase stamps are consistent
and it computes the same bits as libcgp.so.

The stamps tool runs in a child process (a process loads one of the two
libraries); this process steps the same seeded 512x1024 level-1 workload
through libcgp.so with the same calls and compares omega bit for bit."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import cgp_inputs as ci
from gpu_common import dev, say
from paper_1308_3290_amd import _lib
from paper_1308_3290_amd.api import Basin, config_from_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU"),
    pytest.mark.skipif(not os.path.exists(_lib.STAMPS_LIB_PATH),
                       reason="libcgp_stamps.so not built"),
]


def test_stamps_build_matches_libcgp_and_its_phases_add_up(tmp_path):
    steps, repeats = 3, 2
    final = tmp_path / "omega.npy"
    say(f"phase stamps: child run, 512x1024 level 1, {repeats} calls of {steps} steps")
    r = subprocess.run([sys.executable, "-u", "-m", "paper_1308_3290_amd.phase_stamps",
                        "--level", "1", "--steps", str(steps), "--repeats", str(repeats),
                        "--warmup", "2", "--save-final", str(final)],
                       cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    out = json.loads([ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1])
    say(json.dumps(out))
    # launch shapes of the 512x1024 level-1 basin: 255 spectral columns in
    # pairs, 511 coarse rows two per fused block
    assert out["pass_b"]["blocks"] == 128
    assert out["fused"]["blocks"] == 256
    for part, phases in (("pass_b", 3), ("fused", 6)):
        ph = out[part]["phase_us"]
        assert len(ph) == phases
        assert all(v >= 0 for v in ph.values()), ph
        # thread 0's phase medians fit inside the launch's span
        assert sum(ph.values()) <= out[part]["span_us"] * 1.05 + 0.1, (part, out[part])
    assert out["gap_b_to_fused_us"] > 0
    assert 0 < out["pass_b"]["span_us"] + out["fused"]["span_us"] < out["us_per_stage"]

    case = ci.case_c1(1)
    w0 = ci.initial_field(case, np.random.default_rng(case.seed))
    b = Basin(config_from_case(case), device=dev())
    w = torch.as_tensor(w0, device=dev()).contiguous()
    F = torch.as_tensor(ci.forcing_field(case), device=dev()).contiguous()
    for _ in range(repeats):
        b.step(w, F, nsteps=steps)
    torch.cuda.synchronize()
    got = np.load(final)
    ref = w.cpu().numpy()
    b.close()
    assert np.isfinite(ref).all()
    assert np.array_equal(got, ref), float(np.abs(got - ref).max())
