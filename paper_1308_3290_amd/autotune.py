"""Autotuner of how a handle's time steps are launched.

    setting = tune(cfgs, omega_packed, forcing_packed)   # cached per device and workload
    ens.set_launch(**setting["launch"]); ens.step(..., use_graph=setting["use_graph"])

Candidates (``cgp_launch`` and ``cgp_config.fused_rows`` in include/cgp.h):
  - launch mode 0 (one launch per pass and group of members), as replays of
    captured graphs (member chains forked onto streams) or as direct
    launches, each with 2 and (where a member has one layer at coarsening
    factor 2) 4 coarse rows per fused-pass block;
  - launch mode 1 (one persistent launch per RK3 stage over every member),
    where the handle has it, over the work-tile shapes b_tile (pass-B column
    pairs per tile), f_tile (fused-pass row blocks per tile) and the grid's
    workgroups per compute unit.

Each candidate runs on a fresh handle from the same state: ``warmup`` steps,
then ``repeats`` timed runs of ``steps`` steps (HIP events on a side stream;
the median is its time).  Its final state must equal, bit for bit, that of
the reference candidate (mode 0, graph replays, the launch form the GPU
parity tests check against the FP64 oracle); a candidate that differs, or
whose persistent waits reported a fault, is rejected and never cached.  The
fastest accepted candidate is stored in a JSON cache keyed by the device's
architecture name, the dtype, the layer count and the members' grid sizes
and levels, and later calls with the same key return it without timing.
The cache file is $CGP_TUNE_CACHE if set, else ~/.cache/cgp/autotune.json.
A setting is applied as ``configs(cfgs, setting)`` (the handle's configs),
``ens.set_launch(**setting["launch"])`` and ``use_graph``.
"""
from __future__ import annotations

import json
import os
import statistics
from typing import Dict, List, Optional, Sequence

import torch

from . import api

REFERENCE = {"launch": dict(mode=0, b_tile=1, f_tile=1, wg_per_cu=0), "use_graph": True,
             "fused_rows": 2}


def configs(cfgs: Sequence[api.cgp_config], setting: dict) -> List[api.cgp_config]:
    """The members' configs with the setting's fused-pass rows per block."""
    return api.with_fused_rows(cfgs, setting.get("fused_rows", 2))


def has_rows_choice(cfgs: Sequence[api.cgp_config]) -> bool:
    """Whether fused_rows changes anything: a one-layer member at factor 2."""
    return any(c.nlayers == 1 and c.level == 1 for c in cfgs)


def cache_path() -> str:
    return os.environ.get("CGP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cgp", "autotune.json"))


def workload_key(cfgs: Sequence[api.cgp_config], device=None) -> str:
    """Device architecture, dtype, layers and the sorted (nx, ny, level) of
    the members."""
    props = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    dt = "f64" if cfgs[0].dtype == api.CGP_F64 else "f32"
    sizes = sorted((c.nx, c.ny, c.level) for c in cfgs)
    runs: Dict[str, int] = {}
    for s in sizes:
        k = f"{s[0]}x{s[1]}l{s[2]}"
        runs[k] = runs.get(k, 0) + 1
    body = ",".join(f"{k}*{n}" for k, n in sorted(runs.items()))
    return f"{arch}|{dt}|L{cfgs[0].nlayers}|{body}"


def candidates(persistent: bool, rows: bool = False) -> List[dict]:
    base = dict(REFERENCE["launch"])
    out = [dict(REFERENCE), {"launch": dict(base), "use_graph": False, "fused_rows": 2}]
    if rows:
        out += [{"launch": dict(base), "use_graph": g, "fused_rows": 4} for g in (True, False)]
    if persistent:
        for b_tile in (1, 2, 4, 8):
            for f_tile in (1, 2, 4):
                for wg in (0, 1):
                    out.append({"launch": dict(mode=1, b_tile=b_tile, f_tile=f_tile, wg_per_cu=wg),
                                "use_graph": True, "fused_rows": 2})
    return out


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, doc: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _run(cfgs, omega, forcing, cand, steps, warmup, repeats, device):
    ens = api.Ensemble(configs(cfgs, cand), device=device)
    ens.set_launch(**cand["launch"])
    w = omega.clone()
    side = torch.cuda.Stream(device=device)
    side.wait_stream(torch.cuda.current_stream(device))
    with torch.cuda.stream(side):
        ens.step(w, forcing, nsteps=warmup, use_graph=cand["use_graph"], stream=side)
    times = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(side):
            e0.record(side)
            ens.step(w, forcing, nsteps=steps, use_graph=cand["use_graph"], stream=side)
            e1.record(side)
        torch.cuda.synchronize(device)
        times.append(e0.elapsed_time(e1) / steps)
    fault = ens.persistent_fault() if cand["launch"]["mode"] == 1 else 0
    ens.close()
    return statistics.median(times), w, fault


def tune(cfgs: Sequence[api.cgp_config], omega_packed: torch.Tensor,
         forcing_packed: torch.Tensor, steps: int = 30, warmup: int = 6, repeats: int = 3,
         cache: Optional[str] = None, retune: bool = False, report: Optional[list] = None) -> dict:
    """The fastest accepted launch setting for this workload (see the module
    docstring).  omega_packed, forcing_packed: the members' packed fields (as
    Ensemble.pack gives them); they are only read.  report, if given,
    receives one dict per candidate timed (ms per step, accepted)."""
    cfgs = list(cfgs)
    device = omega_packed.device
    path = cache or cache_path()
    key = workload_key(cfgs, device)
    doc = _load(path)
    if not retune and key in doc:
        return doc[key]["setting"]
    probe = api.Ensemble(cfgs, device=device)
    persistent = probe.launch()[1]
    probe.close()
    rows = has_rows_choice(cfgs)
    best = None
    ref_state = None
    for cand in candidates(persistent, rows):
        ms, state, fault = _run(cfgs, omega_packed, forcing_packed, cand, steps, warmup, repeats,
                                device)
        if ref_state is None:
            ref_state = state  # the reference candidate comes first
        accepted = fault == 0 and torch.equal(state, ref_state)
        if report is not None:
            report.append(dict(cand, ms_per_step=ms, accepted=accepted))
        if accepted and (best is None or ms < best[0]):
            best = (ms, cand)
        del state
    setting = best[1]
    doc = _load(path)  # another process may have written meanwhile
    doc[key] = {"setting": setting, "ms_per_step": best[0],
                "steps": steps, "repeats": repeats,
                "candidates": len(candidates(persistent, rows))}
    _store(path, doc)
    return setting
