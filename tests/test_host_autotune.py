"""Host-side checks of the autotuner's candidate set and cache file (no GPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1308_3290_amd import autotune  # noqa: E402


def test_candidates_start_with_the_reference_and_cover_the_tile_shapes():
    plain = autotune.candidates(False)
    full = autotune.candidates(True)
    assert plain[0] == autotune.REFERENCE and full[0] == autotune.REFERENCE
    assert len(plain) == 2 and all(c["launch"]["mode"] == 0 for c in plain)
    pers = [c["launch"] for c in full if c["launch"]["mode"] == 1]
    assert {p["b_tile"] for p in pers} == {1, 2, 4, 8}
    assert {p["f_tile"] for p in pers} == {1, 2, 4}
    assert {p["wg_per_cu"] for p in pers} == {0, 1}


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune._load(path) == {}
    autotune._store(path, {"k": {"setting": autotune.REFERENCE}})
    assert json.load(open(path))["k"]["setting"] == autotune.REFERENCE
    os.environ["CGP_TUNE_CACHE"] = path
    try:
        assert autotune.cache_path() == path
    finally:
        del os.environ["CGP_TUNE_CACHE"]


class _Probe:
    def __init__(self, cfgs, device=None):
        pass

    def launch(self):
        return None, True  # the persistent mode is available

    def close(self):
        pass


def test_tune_rejects_differing_or_faulted_candidates_and_caches_the_fastest(tmp_path,
                                                                             monkeypatch):
    import torch
    from paper_1308_3290_amd import api
    cfgs = [api.cgp_config(nx=256, ny=512, level=1, nlayers=1)]
    cands = autotune.candidates(True, autotune.has_rows_choice(cfgs))
    ref = torch.arange(6.0)
    # the reference is slowest; a faster candidate with other bits and a faster
    # one whose persistent waits faulted must both lose to the fastest accepted
    plan = {0: (3.0, ref, 0), 1: (1.0, ref + 1e-12, 0), 2: (1.5, ref, 5), 3: (2.0, ref, 0)}
    calls = []

    def fake_run(cfgs_, omega, forcing, cand, steps, warmup, repeats, device):
        i = cands.index(cand)
        calls.append(i)
        ms, state, fault = plan.get(i, (2.5, ref, 0))
        return ms, state.clone(), fault

    monkeypatch.setattr(autotune, "_run", fake_run)
    monkeypatch.setattr(autotune.api, "Ensemble", _Probe)
    monkeypatch.setattr(autotune, "workload_key", lambda c, d=None: "gfx950|f64|L1|256x512l1*1")
    path = str(tmp_path / "tune.json")
    report = []
    omega = torch.zeros(6)
    setting = autotune.tune(cfgs, omega, omega, cache=path, report=report)
    assert calls == list(range(len(cands)))  # the reference first, every candidate once
    assert setting == cands[3]
    assert [r["accepted"] for r in report[:4]] == [True, False, False, True]
    assert all(r["accepted"] for r in report[4:])
    doc = json.load(open(path))
    assert doc["gfx950|f64|L1|256x512l1*1"]["setting"] == cands[3]
    assert doc["gfx950|f64|L1|256x512l1*1"]["ms_per_step"] == 2.0
    # a cached key is returned without timing; retune times again
    calls.clear()
    assert autotune.tune(cfgs, omega, omega, cache=path) == cands[3] and calls == []
    assert autotune.tune(cfgs, omega, omega, cache=path, retune=True) == cands[3]
    assert len(calls) == len(cands)
