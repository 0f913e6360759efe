"""Long runs and their statistics on the GPU (the paper's Sec. 5.1 experiments).

A run spins up from the initial state to t_spin, then averages omega over
[t_spin, t_end] in time (every step adds dt * omega to an FP64 running sum in
the library, `cgp_step_mean`), and records the basin energy and enstrophy
(eq. 26, `cgp_diagnostics`) every chunk of steps.  The mean of psi is the
elliptic map of the mean of omega (the map is linear); the mean potential
vorticity is q = Ro <omega> + y (vorticity form).

    python -m paper_1308_3290_amd.statistics --exp I --levels 0 1 2

runs the one-layer four-gyre experiments of Sec. 5.1 (Table 1: Exp. I
Re = 200, Ro = 0.0016; Exp. II Re = 312.5, Ro = 0.0025; forcing
sin(pi y) / Ro on [0, 1] x [-1, 1]) at 256 x 512 with CGP levels 0 (the
full-grid run the paper calls DNS), 1 and 2, adaptive steps (Sec. 4.2), and
prints one JSON line per run with the differences of its mean fields from
the level-0 run.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Optional

import numpy as np
import torch

from .api import Basin, make_config

# Table 1 (one layer): Ro = (delta_I / L)^2, Re = Ro / (delta_M / L)^3
EXPERIMENTS = {"I": dict(ro=0.0016, re=200.0), "II": dict(ro=0.0025, re=312.5)}


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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--exp", default="I", choices=sorted(EXPERIMENTS))
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--levels", type=int, nargs="+", default=[0, 1, 2])
    ap.add_argument("--t-spin", type=float, default=10.0)
    ap.add_argument("--t-end", type=float, default=50.0)
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--dt-max", type=float, default=5e-4)
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--control-seed", type=int, default=None,
                    help="also run level 0 from another initial state (this seed) and report "
                         "its differences from the first level-0 run: the sampling spread of "
                         "the time means")
    args = ap.parse_args(argv)
    p = EXPERIMENTS[args.exp]
    nx, ny = args.nx, args.ny
    y = -1.0 + np.arange(ny + 1) * (2.0 / ny)
    F = np.broadcast_to((np.sin(np.pi * y) / p["ro"])[:, None], (ny + 1, nx + 1)).copy()
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream()  # graphs are captured on a non-default stream
    ref = None
    runs = [(lv, args.seed) for lv in args.levels]
    if args.control_seed is not None:
        runs.append((0, args.control_seed))
    for lv, seed in runs:
        w0 = np.zeros((ny + 1, nx + 1))
        w0[1:-1, 1:-1] = 1e-3 * np.random.default_rng(seed).standard_normal((ny - 1, nx - 1))
        cfg = make_config(nx, ny, level=lv, dtype=args.dtype, inv_re=1.0 / p["re"],
                          inv_ro=1.0 / p["ro"], dt=args.dt_max, cfl=args.cfl)
        b = Basin(cfg, device=dev)
        w = torch.as_tensor(w0, dtype=tdt, device=dev).contiguous()
        Fd = torch.as_tensor(F, dtype=tdt, device=dev).contiguous()
        mark = [0.0]

        def progress(t, n, lv=lv):
            if t >= mark[0]:
                print(f"level {lv}: t = {t:.3f} after {n} steps", file=sys.stderr, flush=True)
                mark[0] += 5.0

        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            r = long_run(b, w, Fd, args.t_spin, args.t_end, chunk=args.chunk, stream=side,
                         progress=progress)
        q = p["ro"] * r["mean_omega"] + y[:, None]
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
            ref = dict(psi=r["mean_psi"], q=q)
        else:
            out["mean_psi_rel_diff_vs_level0"] = _rel(r["mean_psi"], ref["psi"])
            out["mean_q_rel_diff_vs_level0"] = _rel(q, ref["q"])
        print(json.dumps(out), flush=True)
        b.close()


if __name__ == "__main__":
    main()
