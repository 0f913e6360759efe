"""Phase times of a single basin's time step, from the measurement build.

    python -m paper_1308_3290_amd.phase_stamps [--level 1] [--steps 20] [--repeats 20]

Loads libcgp_stamps.so: the kernels of libcgp.so with the same arithmetic,
where thread 0 of every block of pass B and of the fused one-layer stage pass
writes the device's steady clock at each phase boundary (`cgp_phase_stamps`
in include/cgp.h names the slots).  The 512x1024 FP64 one-layer workload at
the given level is advanced by `steps` steps per call (direct launches, as
`cgp_step` runs them); after each call the stamps of that call's last
launches are read, pass B and the fused pass of the last RK3 stage of the
last step, which ran behind a full queue of earlier launches.  Per call:

- pass B: span from its first block's start to its last block's end, and
  per-block phase times (medians over the blocks);
- the gap from pass B's last block end to the fused pass's first block start;
- the fused pass: span and per-block phase times (medians over the blocks);

and the step time of the same build (events around `steps` x `repeats`
steps).  One JSON line holds the medians over the calls.  `--save-final`
writes omega after the repeats (before the timed run) to a .npy file, which
lets a test compare the build's bits with libcgp.so's.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import statistics
import sys

import numpy as np

from . import _lib

B_PHASES = ["columns loaded", "forward transform + divide", "inverse transform + stores"]
F_PHASES = ["spectra in LDS", "inverse x transform", "vorticity tile in LDS",
            "stencil + RK3 combine", "restriction", "forward x transform + stores"]


def read_stamps(kind: int, nmax: int = 4096):
    """(stamps [n, 8] of the last launch's n blocks, clock rate in kHz)."""
    buf = (ctypes.c_uint64 * (nmax * 8))()
    khz = ctypes.c_int32(0)
    _lib.check(_lib.load().cgp_phase_stamps(kind, buf, nmax, ctypes.byref(khz)))
    a = np.frombuffer(buf, dtype=np.uint64).reshape(nmax, 8).astype(np.int64)
    written = np.nonzero(a[:, 0])[0]
    n = int(written[-1]) + 1 if written.size else 0
    if n == 0 or written.size != n:
        raise RuntimeError(f"stamps of kind {kind}: blocks written {written.size}, "
                           f"highest index {n - 1}")
    return a[:n], khz.value


def launch_summary(b: np.ndarray, f: np.ndarray, us_per_tick: float) -> dict:
    """Spans, gap and per-block phase medians (us) of one pass-B launch b and
    the fused launch f that followed it."""
    def phases(a, nslots):
        d = np.diff(a[:, :nslots], axis=1) * us_per_tick
        return [float(np.median(d[:, i])) for i in range(nslots - 1)]
    return dict(
        b_span=float(b[:, 3].max() - b[:, 0].min()) * us_per_tick,
        b_start_spread=float(b[:, 0].max() - b[:, 0].min()) * us_per_tick,
        b_phases=phases(b, 4),
        gap_b_to_f=float(f[:, 0].min() - b[:, 3].max()) * us_per_tick,
        f_span=float(f[:, 6].max() - f[:, 0].min()) * us_per_tick,
        f_start_spread=float(f[:, 0].max() - f[:, 0].min()) * us_per_tick,
        f_phases=phases(f, 7),
        b_blocks=int(b.shape[0]), f_blocks=int(f.shape[0]))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--level", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="steps per call")
    ap.add_argument("--repeats", type=int, default=20, help="calls (stamps read after each)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--save-final", default=None)
    args = ap.parse_args(argv)

    _lib.LIB_PATH = _lib.STAMPS_LIB_PATH
    import torch

    import cgp_inputs as ci
    from .api import Basin, config_from_case

    assert torch.cuda.is_available(), "phase stamps need a GPU"
    lib = _lib.load()
    if not hasattr(lib, "cgp_phase_stamps"):
        raise RuntimeError(f"{_lib.LIB_PATH} has no cgp_phase_stamps (not the measurement build)")
    case = ci.case_c1(args.level)
    w0 = ci.initial_field(case, np.random.default_rng(case.seed))
    F = ci.forcing_field(case)
    dev = torch.device("cuda:0")
    basin = Basin(config_from_case(case), device=dev)
    w = torch.as_tensor(w0, device=dev).contiguous()
    Fd = torch.as_tensor(F, device=dev).contiguous()
    per_call = []
    khz = 0
    for _ in range(args.repeats):
        basin.step(w, Fd, nsteps=args.steps)
        b, khz = read_stamps(0)
        f, _ = read_stamps(1)
        per_call.append(launch_summary(b, f, 1e3 / khz))
    if args.save_final:
        torch.cuda.synchronize()
        np.save(args.save_final, w.cpu().numpy())
    # step time of this build
    wt = torch.as_tensor(w0, device=dev).contiguous()
    basin.step(wt, Fd, nsteps=args.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nt = args.steps * args.repeats
    torch.cuda.synchronize()
    e0.record()
    basin.step(wt, Fd, nsteps=nt)
    e1.record()
    torch.cuda.synchronize()
    us_step = e0.elapsed_time(e1) * 1e3 / nt

    def med(key, i=None):
        vals = [c[key] if i is None else c[key][i] for c in per_call]
        return round(statistics.median(vals), 3)

    s = dict(b_span=med("b_span"), gap_b_to_f=med("gap_b_to_f"), f_span=med("f_span"))
    stage = us_step / 3
    out = dict(
        workload=f"512x1024 FP64 one layer, CGP level {args.level}", library="libcgp_stamps.so",
        clock_khz=khz, calls=args.repeats, steps_per_call=args.steps,
        us_per_step=round(us_step, 3), us_per_stage=round(stage, 3),
        pass_b=dict(blocks=per_call[-1]["b_blocks"], span_us=s["b_span"],
                    start_spread_us=med("b_start_spread"),
                    phase_us={n: med("b_phases", i) for i, n in enumerate(B_PHASES)}),
        gap_b_to_fused_us=s["gap_b_to_f"],
        fused=dict(blocks=per_call[-1]["f_blocks"], span_us=s["f_span"],
                   start_spread_us=med("f_start_spread"),
                   phase_us={n: med("f_phases", i) for i, n in enumerate(F_PHASES)}),
        # what a stage's time leaves after the two spans and the gap between
        # them: the gap from the fused pass's end to the next pass B's start
        gap_fused_to_next_b_us=round(stage - s["b_span"] - s["gap_b_to_f"] - s["f_span"], 3),
    )
    print(json.dumps(out), flush=True)
    basin.close()
    return out


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
