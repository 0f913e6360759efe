"""Long runs and their statistics on the GPU (the paper's Sec. 5.1 experiments).

A run spins up from the initial state to t_spin, then averages omega over
[t_spin, t_end] in time (every step adds dt * omega to an FP64 running sum in
the library, `cgp_step_mean`), and records the basin energy and enstrophy
(eq. 26, `cgp_diagnostics`) every chunk of steps.  The mean of psi is the
elliptic map of the mean of omega (the map is linear, `cgp_solve`); the mean
potential vorticity is q = Ro <omega> + y (vorticity form).  The division of
the running sum by the window length and q = Ro <omega> + y are applied once
per run to the final fields, in NumPy: post-processing of the statistics,
outside the time step, whose per-step work all runs in the library.

    python -m paper_1308_3290_amd.statistics --exp I --runs 256x512:0 256x512:1 256x512:2

runs the one-layer four-gyre experiments of Sec. 5.1 (Table 1: Exp. I
Re = 200, Ro = 0.0016; Exp. II Re = 312.5, Ro = 0.0025; forcing
sin(pi y) / Ro on [0, 1] x [-1, 1], inputs from cgp_inputs.experiment_case)
with adaptive steps (Sec. 4.2) and prints one JSON line per run with the
differences of its mean fields from the first run (the reference, the
full-grid run the paper calls DNS).  Runs on coarser fine grids than the
reference (the fixed 16 x 32 elliptic grid of the paper's last comparison:
16x32:0, 32x64:1, 64x128:2) are compared at their own nodes, where the
grids nest (the reference sampled every nx_ref / nx nodes).
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Optional

import numpy as np
import torch

import cgp_inputs as ci

from .api import Basin, config_from_case


def _now(basin: Basin, stream=None) -> float:
    return float(basin.time_state(stream)[1].item())


def long_run(basin: Basin, omega: torch.Tensor, forcing: torch.Tensor, t_spin: float,
             t_end: float, chunk: int = 250, use_graph: bool = True, stream=None,
             max_steps: Optional[int] = None, progress=None) -> dict:
    """Advance omega (in place) to t_spin, then to t_end while averaging.

    Returns host arrays mean_omega, mean_psi, the window [t0, t1] actually
    averaged (chunk boundaries at or after t_spin and t_end), the energy and
    enstrophy history (times, E, Z per layer) over the whole run, step
    counts and the wall time of the stepping (seconds).  progress(t, steps),
    if given, is called after every chunk."""
    dev = omega.device
    nl = basin.cfg.nlayers
    total = torch.zeros(omega.shape, dtype=torch.float64, device=dev)
    spin = torch.zeros(omega.shape, dtype=torch.float64, device=dev)  # discarded
    psi = torch.empty_like(omega)
    hist_t, hist_ez = [], []
    steps_spin = steps_avg = 0
    limit = max_steps if max_steps is not None else 1 << 62

    def record():
        basin.solve(omega, psi, stream)
        ez = basin.diagnostics(omega, psi, stream=stream)
        ts = basin.time_state(stream)
        hist_t.append(ts[1].clone())
        hist_ez.append(ez.clone())

    torch.cuda.synchronize()
    w0 = time.perf_counter()
    record()
    while _now(basin, stream) < t_spin and steps_spin < limit:
        basin.step_mean(omega, forcing, chunk, spin, use_graph=use_graph, stream=stream)
        steps_spin += chunk
        record()
        if progress:
            progress(_now(basin, stream), steps_spin)
    t0 = _now(basin, stream)
    while _now(basin, stream) < t_end and steps_spin + steps_avg < limit:
        basin.step_mean(omega, forcing, chunk, total, use_graph=use_graph, stream=stream)
        steps_avg += chunk
        record()
        if progress:
            progress(_now(basin, stream), steps_spin + steps_avg)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    t1 = _now(basin, stream)
    mean_w = total.cpu().numpy() / (t1 - t0) if t1 > t0 else total.cpu().numpy() * 0.0
    mw_dev = torch.as_tensor(mean_w, dtype=omega.dtype, device=dev).contiguous()
    mean_psi = basin.solve(mw_dev, stream=stream).cpu().to(torch.float64).numpy()
    hist = torch.stack(hist_ez).cpu().numpy().reshape(len(hist_ez), nl, 2)
    return dict(mean_omega=mean_w, mean_psi=mean_psi, t0=t0, t1=t1,
                times=torch.stack(hist_t).cpu().numpy(), energy=hist[:, :, 0],
                enstrophy=hist[:, :, 1], steps_spin=steps_spin, steps_avg=steps_avg,
                wall_s=wall)


def gyre_count(mean_psi: np.ndarray, frac: float = 0.01) -> int:
    """Sign-alternating regions of the zonally averaged mean psi along y
    (ignoring values below frac of its largest magnitude): 4 for the four-gyre
    time mean."""
    prof = np.asarray(mean_psi)[..., 1:-1, 1:-1].mean(axis=-1)
    if prof.ndim > 1:
        prof = prof[0]
    thr = frac * np.abs(prof).max()
    signs = [np.sign(v) for v in prof if abs(v) > thr]
    return int(1 + sum(1 for a, b in zip(signs, signs[1:]) if a != b)) if signs else 0


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def on_grid(field: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """field (a node array of a finer nested grid) at the nodes of an nx x ny
    grid over the same basin."""
    fy, fx = field.shape[-2] - 1, field.shape[-1] - 1
    if fx % nx or fy % ny or fx // nx != fy // ny:
        raise ValueError(f"{fx}x{fy} does not nest {nx}x{ny}")
    k = fx // nx
    return field[..., ::k, ::k]


def parse_run(spec: str):
    """'NXxNY:LEVEL' -> (nx, ny, level)."""
    g, lv = spec.split(":")
    nx, ny = g.lower().split("x")
    return int(nx), int(ny), int(lv)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--exp", default="I", choices=sorted(ci.EXPERIMENTS_1L))
    ap.add_argument("--runs", nargs="+", default=["256x512:0", "256x512:1", "256x512:2"],
                    help="NXxNY:LEVEL per run; the first is the reference")
    ap.add_argument("--t-spin", type=float, default=10.0)
    ap.add_argument("--t-end", type=float, default=50.0)
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--dt-max", type=float, default=5e-4)
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--control-seed", type=int, default=None,
                    help="also run the reference configuration from another initial state "
                         "(this seed) and report its differences from the reference: the "
                         "sampling spread of the time means")
    ap.add_argument("--save", default=None, help="write every run's mean fields to this .npz")
    args = ap.parse_args(argv)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream()  # graphs are captured on a non-default stream
    ref = None
    runs = [(parse_run(r), args.seed) for r in args.runs]
    if args.control_seed is not None:
        runs.append((runs[0][0], args.control_seed))
    saved = {}
    for (nx, ny, lv), seed in runs:
        case, w0, F = ci.experiment_case(args.exp, nx, ny, lv, seed=seed, cfl=args.cfl,
                                         dt_max=args.dt_max, dtype=args.dtype)
        ro = 1.0 / case.inv_ro
        y = ci.node_y(case)
        b = Basin(config_from_case(case), device=dev)
        w = torch.as_tensor(w0, dtype=tdt, device=dev).contiguous()
        Fd = torch.as_tensor(F, dtype=tdt, device=dev).contiguous()
        mark = [0.0]

        def progress(t, n, lv=lv, nx=nx, ny=ny):
            if t >= mark[0]:
                print(f"{nx}x{ny} level {lv}: t = {t:.3f} after {n} steps", file=sys.stderr,
                      flush=True)
                mark[0] += 5.0

        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            r = long_run(b, w, Fd, args.t_spin, args.t_end, chunk=args.chunk, stream=side,
                         progress=progress)
        q = ro * r["mean_omega"] + y[:, None]
        sel = r["times"] >= r["t0"]
        out = dict(experiment=args.exp, grid=f"{nx}x{ny}", level=lv, seed=seed,
                   elliptic_grid=f"{nx >> lv}x{ny >> lv}", cfl=args.cfl, dt_max=args.dt_max,
                   t_window=[round(r["t0"], 4), round(r["t1"], 4)],
                   steps=r["steps_spin"] + r["steps_avg"], wall_s=round(r["wall_s"], 2),
                   us_per_step=round(1e6 * r["wall_s"] / (r["steps_spin"] + r["steps_avg"]), 2),
                   mean_energy=float(r["energy"][sel, 0].mean()),
                   final_energy=float(r["energy"][-1, 0]),
                   gyres=gyre_count(r["mean_psi"]),
                   finite=bool(np.isfinite(r["mean_omega"]).all()))
        if ref is None:
            ref = dict(psi=r["mean_psi"], q=q, grid=f"{nx}x{ny}:{lv}")
        else:
            out["reference"] = ref["grid"]
            out["mean_psi_rel_diff_vs_ref"] = _rel(r["mean_psi"], on_grid(ref["psi"], nx, ny))
            out["mean_q_rel_diff_vs_ref"] = _rel(q, on_grid(ref["q"], nx, ny))
        tag = f"{nx}x{ny}_l{lv}_s{seed}"
        saved[f"psi_{tag}"] = r["mean_psi"]
        saved[f"q_{tag}"] = q
        saved[f"t_{tag}"] = r["times"]
        saved[f"E_{tag}"] = r["energy"][:, 0]
        print(json.dumps(out), flush=True)
        b.close()
    if args.save:
        np.savez_compressed(args.save, **saved)


if __name__ == "__main__":
    main()
