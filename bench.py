"""Throughput of the CGP QG time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extras]

Workload (the value): single-layer barotropic QG, 512 x 1024 fine grid, FP64,
CGP factor 2 (256 x 512 coarse solve), Re 450, Ro 0.0036, dt 2.5e-5, seeded
omega0 = 1e-3 N(0,1), forcing (1/Ro) sin(pi y).  Metric: fine-grid
Mpoint-steps/s = 512 * 1024 * K / seconds over K timed steps (hipGraph replay
of one step, inputs resident in HBM).  Beside it: the same basin with the
full-grid solve (factor 1) and factor 4, the CGP/full-grid speed-up, the
adjoint/forward time ratio of the 256 x 512, 200-step checkpointed adjoint,
per-pass launch times (HIP events on the library's stream), the roofline of
the dominant kernel and the FP64 oracle timed on the host CPU.

Prints ONE JSON line.  Only one GPU is used; --gpus N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "Mpoint-steps/s at 512x1024, CGP vs full-grid on 1 GPU; adjoint/forward time ratio"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--extras", action="store_true",
                    help="also time two layers, FP32 and the 64-member ensemble")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", default="", help="comma list: l0,l1,l2,timed (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration runs)")
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV",
                    help="print per-kernel launch statistics of a rocprofv3 --kernel-trace CSV "
                         "as a markdown table and exit (no GPU needed)")
    ap.add_argument("--trace-tail", type=int, default=0, metavar="N",
                    help="with --summarize-trace: statistics over each kernel's last N launches "
                         "(the cgp_time_passes launches that end a --only timed run)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) into "
                         "profiles/traffic_c1_l1.json and exit (no GPU needed)")
    return ap.parse_args()


COPY_BYTES = 256 << 20


def summarize_pmc(fetch_csv, write_csv, out_path=None):
    """HBM bytes per dispatch of each CGP kernel from FETCH_SIZE / WRITE_SIZE (KiB),
    each scaled so that the plain copy of COPY_BYTES reads and writes exactly that;
    written to out_path (default profiles/traffic_c1_l1.json)."""
    import csv
    import statistics

    def load(path, counter):
        per = {}
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name", counter) != counter:
                continue
            name = r["Kernel_Name"]
            per.setdefault(name, {}).setdefault(r["Dispatch_Id"], 0.0)
            per[name][r["Dispatch_Id"]] += float(r["Counter_Value"])
        return {k: statistics.median(v.values()) for k, v in per.items()}

    fetch = load(fetch_csv, "FETCH_SIZE")
    write = load(write_csv, "WRITE_SIZE")

    def copy_value(d):
        cands = [v for k, v in d.items() if "MulFunctor" in k]
        return max(cands) if cands else None

    cf, cw = copy_value(fetch), copy_value(write)
    sf = COPY_BYTES / (cf * 1024.0) if cf else 1.0
    sw = COPY_BYTES / (cw * 1024.0) if cw else 1.0
    out = {"source_hash": source_hash(), "copy_bytes": COPY_BYTES,
           "scale_fetch": sf, "scale_write": sw, "kernels": {}}
    for name in fetch:
        if "cgp::" not in name:
            continue
        short = name.split("cgp::")[1].split("<")[0].split("(")[0]
        fb = fetch[name] * 1024.0 * sf
        wb = write.get(name, 0.0) * 1024.0 * sw
        out["kernels"][short] = {"fetch_bytes": fb, "write_bytes": wb,
                                 "hbm_bytes_per_launch": fb + wb}
    path = out_path or os.path.join(ROOT, "profiles", "traffic_c1_l1.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out, indent=1))


def summarize_trace(trace_csv, tail=0):
    """Launch count and duration statistics (us) per kernel of a kernel trace
    (tail > 0: over each kernel's last `tail` launches in start order)."""
    import csv
    import statistics
    per = {}
    for r in csv.DictReader(open(trace_csv)):
        name = r["Kernel_Name"]
        if "cgp::" in name:
            name = name.split("cgp::")[1].split("(")[0]
        start = int(r["Start_Timestamp"])
        per.setdefault(name, []).append((start, (int(r["End_Timestamp"]) - start) / 1000.0))
    per = {k: [d for _, d in sorted(v)][-tail if tail > 0 else 0:] for k, v in per.items()}
    print("| kernel | launches | mean us | median us | min us | max us |")
    print("|---|---|---|---|---|---|")
    for name, d in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        print(f"| {name} | {len(d)} | {statistics.mean(d):.2f} | {statistics.median(d):.2f} | "
              f"{min(d):.2f} | {max(d):.2f} |")


def pass_bytes(case, es):
    """Algorithmic bytes of one launch of each pass as timed by cgp_time_passes
    (fine node arrays with ring, coarse interior spectra); pass D in its
    stage-2 form reads four fine fields and writes one; the fused C + D pass
    reads the coarse spectra and three fine fields and writes one; with the
    next stage's pass A it also writes the spectra of its result."""
    fine = (case.nx + 1) * (case.ny + 1) * case.nlayers * es
    c = 2 ** case.level
    coarse = (case.nx // c - 1) * (case.ny // c - 1) * case.nlayers * es
    return {"A": fine + coarse, "B": 2 * coarse, "C": coarse + fine, "D": 5.0 * fine,
            "CD": coarse + 4.0 * fine, "CDA": 2 * coarse + 4.0 * fine}


def source_hash():
    h = hashlib.sha256()
    for f in ("stencil_kernels.hip", "solve_kernels.hip", "fused_kernels.hip", "fft_lds.hpp",
              "stencil.hpp", "cgp_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1308_3290_amd", "csrc", f), "rb").read())
    # the compile flags are part of the kernels too
    h.update(open(os.path.join(ROOT, "paper_1308_3290_amd", "build.py"), "rb").read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.trace_tail)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build runs on one GPU only; "
                          "the multi-GPU design is described, not built (use --gpus 1)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import cgp_inputs as ci
    from paper_1308_3290_amd import api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    only = set(filter(None, args.only.split(",")))
    K, W = args.steps, args.warmup

    def timed_run(case, use_graph=True, steps=K, warm=W, dtype="f64"):
        tdt = torch.float64 if dtype == "f64" else torch.float32
        rng = np.random.default_rng(case.seed)
        w0 = ci.initial_field(case, rng)
        F = torch.as_tensor(ci.forcing_field(case), dtype=tdt, device=dev)
        ens = api.Ensemble([api.config_from_case(case, dtype)], device=dev)
        w = torch.as_tensor(w0, dtype=tdt, device=dev).reshape(-1).contiguous()
        Fp = F.reshape(-1).contiguous()
        if case.nlayers == 2:
            Fp = torch.cat([Fp, torch.zeros_like(Fp)])  # layer-2 forcing slot unused
            Fp = Fp[: w.numel()].contiguous()
        # a non-default stream (graphs cannot be captured on the default one);
        # the events are recorded on it
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            ens.step(w, Fp, nsteps=warm, use_graph=use_graph)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s):
            e0.record(s)
            ens.step(w, Fp, nsteps=steps, use_graph=use_graph)
            e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        finite = bool(torch.isfinite(w).all().item())
        return ms, finite, ens, w, Fp

    result = {}
    if args.copy_calibration:
        a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)  # one elementwise kernel: reads and writes COPY_BYTES
        torch.cuda.synchronize()
        del a, b
    # ---------------------------------------------------------------- main line
    rates = {}
    for lv in (1, 0, 2):
        if only and f"l{lv}" not in only:
            continue
        case = ci.case_c1(lv)
        # the same K steps as captured-graph replays and as direct launches;
        # the faster of the two is the level's rate (both are library modes)
        by_mode = {}
        for mode in ("graph", "direct"):
            ms, finite, ens, w, Fp = timed_run(case, use_graph=mode == "graph")
            by_mode[mode] = dict(ms=ms, rate=case.points * K / (ms * 1e-3) / 1e6, finite=finite,
                                 launch=mode)
            log(f"512x1024 FP64 level {lv} ({mode}): {ms / K * 1e3:.1f} us/step, "
                f"{by_mode[mode]['rate']:.0f} Mpoint-steps/s (finite={finite})")
            del ens, w, Fp
        rates[lv] = max(by_mode.values(), key=lambda r: r["rate"])
        rates[lv]["modes"] = {m: round(r["rate"], 1) for m, r in by_mode.items()}
    # ---------------------------------------------------------------- per-pass roofline
    roof = None
    if not only or "timed" in only:
        case = ci.case_c1(1)
        rng = np.random.default_rng(case.seed)
        b = api.Basin(api.config_from_case(case), device=dev)
        w = torch.as_tensor(ci.initial_field(case, rng), device=dev)
        F = torch.as_tensor(ci.forcing_field(case), device=dev)
        b.step(w, F, nsteps=2)  # fills psi, the stage buffers and the spectra
        api.cgp_time_passes(b.handle, w, F, 10)
        ms = api.cgp_time_passes(b.handle, w, F, 200)
        by = pass_bytes(case, 8)
        names = ["A", "B", "C", "D", "CD", "CDA"]
        if ms[4] <= 0:
            names = names[:4]
        # passes a time step launches: B and the fused pass (C, D and the next
        # stage's A) per stage, A once per call; else A, B, C, D per stage
        in_step = ["B", "CDA"] if "CDA" in names else ["A", "B", "C", "D"]
        dom = max(in_step, key=lambda n: ms[names.index(n)])
        i = names.index(dom)
        achieved = by[dom] / (ms[i] * 1e-3) / 1e9
        kernel_names = {"A": "k_restrict_rowdst", "B": "k_col_solve", "C": "k_rowdst_prolong",
                        "D": "k_stencil_rk3", "CD": "k_prolong_stencil<NEXT=false>",
                        "CDA": "k_prolong_stencil<NEXT=true>"}
        passes = {kernel_names[n]: {"us_per_launch": ms[j] * 1e3,
                                    "alg_bytes_per_launch": by[n],
                                    "achieved_GBs": by[n] / (ms[j] * 1e-3) / 1e9,
                                    "in_time_step": n in in_step}
                  for j, n in enumerate(names)}
        log("per-pass: " + json.dumps(passes))
        traffic = None
        tfile = os.path.join(ROOT, "profiles", "traffic_c1_l1.json")
        if os.path.exists(tfile):
            t = json.load(open(tfile))
            # counters are taken on a time-stepping run: the fused kernel there
            # is always the NEXT=true form
            base = kernel_names[dom].split("<")[0]
            if t.get("source_hash") == source_hash() and base in t.get("kernels", {}):
                traffic = t["kernels"][base]["hbm_bytes_per_launch"]
        # achievable HBM bandwidth: 1 GiB read + 1 GiB written by a device
        # copy and by an elementwise kernel, the better of the two
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        best = 0.0
        for op in (lambda: dst.copy_(src), lambda: torch.mul(src, 1.0, out=dst)):
            for _ in range(3):
                op()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                op()
            e1.record()
            torch.cuda.synchronize()
            best = max(best, 10 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        del src, dst
        log(f"achievable HBM bandwidth (1 GiB copy): {best:.0f} GB/s")
        roof = {"bound": "hbm", "kernel": kernel_names[dom], "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic, "alg_bytes_per_launch": by[dom],
                "us_per_launch": round(ms[i] * 1e3, 2),
                "achievable_copy": round(best, 1), "frac_of_achievable": round(achieved / best, 4)}
        result["passes"] = passes
        # diagnostics (E and Z per layer, eq. 26): outside the time step, timed
        # on their own over the same fields; they read psi and omega once
        psi = b.solve(w)
        ez = torch.empty(2, dtype=torch.float64, device=dev)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(5):
                api.cgp_diagnostics(b.handle, w, psi, ez, s)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(200):
                api.cgp_diagnostics(b.handle, w, psi, ez, s)
            e1.record(s)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 200
        dbytes = 2 * w.numel() * 8
        result["diagnostics"] = {"us_per_call": round(us, 2), "alg_bytes_per_call": dbytes,
                                 "achieved_GBs": round(dbytes / (us * 1e-6) / 1e9, 1)}
        log(f"diagnostics: {us:.1f} us per call ({dbytes / (us * 1e-6) / 1e9:.0f} GB/s)")
        del b, w, F, psi
    # ---------------------------------------------------------------- adjoint ratio
    adj = None
    if not args.no_adjoint and (not only or "adj" in only):
        p = ci.adjoint_c4()
        c = p.case
        b = api.Basin(api.config_from_case(c), device=dev)
        w0 = torch.as_tensor(p.omega0, device=dev).requires_grad_(True)
        F = torch.as_tensor(p.forcing, device=dev).requires_grad_(True)
        idx = torch.as_tensor(p.obs_index, device=dev)
        obs = torch.as_tensor(p.obs_value, device=dev)
        for rep in range(2):  # first pass warms up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            wT = api.Trajectory.apply(w0, F, b, c.nsteps, p.ckpt_every)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L = ((wT.view(-1)[idx] - obs) ** 2).mean()
            w0.grad = None
            F.grad = None
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            t3 = time.perf_counter()
        adj = {"forward_ms": (t1 - t0) * 1e3, "backward_ms": (t3 - t2) * 1e3,
               "ratio": (t3 - t2) / (t1 - t0), "workload": "256x512 FP64 CGP factor 2, "
               "200 steps, checkpoint every 20, final-time misfit at 1% of nodes"}
        log(f"adjoint: forward {adj['forward_ms']:.1f} ms, backward {adj['backward_ms']:.1f} ms, "
            f"ratio {adj['ratio']:.2f}")
        del b, w0, F
    # ---------------------------------------------------------------- extras
    extras = {}
    if args.extras:
        # --only may pick extras too: two_layer, l3, mg, adaptive, fp32, ens
        want = (lambda k: not only or k in only)
        for lv in (1, 0, 2):
            if not want("two_layer"):
                break
            case = ci.case_c2(lv)
            ms, finite, *_ = timed_run(case, steps=min(K, 500))
            extras[f"two_layer_l{lv}"] = case.points * min(K, 500) / (ms * 1e-3) / 1e6
        if want("l3"):  # three levels of coarsening (64x128 solve)
            case = ci.case_c1(3)
            ms, finite, *_ = timed_run(case, steps=min(K, 500))
            extras["cgp8_l3"] = case.points * min(K, 500) / (ms * 1e-3) / 1e6
        if want("mg"):  # the multigrid coarse solver (12 V-cycles) at levels 0, 1, 2
            for lv in (0, 1, 2):
                case = ci.case_c1(lv)
                case.solver = 1
                ms, finite, *_ = timed_run(case, steps=20, warm=2)
                extras[f"multigrid_l{lv}"] = case.points * 20 / (ms * 1e-3) / 1e6
        if want("adaptive"):  # the step size of Sec. 4.2 (CFL 0.5, capped at dt)
            case = ci.case_c1(1)
            case.cfl = 0.5
            ms, finite, *_ = timed_run(case)
            extras["adaptive_l1"] = case.points * K / (ms * 1e-3) / 1e6
        for lv in (1, 0):
            if not want("fp32"):
                break
            case = ci.case_c1(lv)
            ms, finite, *_ = timed_run(case, dtype="f32")
            extras[f"fp32_l{lv}"] = case.points * K / (ms * 1e-3) / 1e6
        for dt_ in ("f64", "f32"):
            if not want("ens"):
                break
            members = ci.ensemble_c3(dtype=dt_)
            tdt = torch.float64 if dt_ == "f64" else torch.float32
            ens = api.Ensemble([api.config_from_case(m.case) for m in members], device=dev)
            Wp = ens.pack([m.omega0 for m in members])
            Fp = ens.pack([m.forcing for m in members])
            s = torch.cuda.Stream()  # graphs are captured on a non-default stream
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                ens.step(Wp, Fp, nsteps=5)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            n_ens = 200
            with torch.cuda.stream(s):
                e0.record(s)
                ens.step(Wp, Fp, nsteps=n_ens)
                e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            pts = sum(m.case.points for m in members)
            es = 8 if dt_ == "f64" else 4
            extras[f"ensemble64_{dt_}"] = pts * n_ens / (ms * 1e-3) / 1e6
            # bytes per point-step: the unfused model e (20 + 12/c^2) and the
            # fused path's algorithmic 12 e (1 + 1/c^2), c = 2
            extras[f"ensemble64_{dt_}_GBs_model"] = (pts * n_ens * (20 + 12 / 4) * es
                                                     / (ms * 1e-3) / 1e9)
            extras[f"ensemble64_{dt_}_GBs_alg"] = (pts * n_ens * 12 * (1 + 1 / 4) * es
                                                   / (ms * 1e-3) / 1e9)
            assert tdt == Wp.dtype
            del ens, Wp, Fp
        log("extras: " + json.dumps(extras))
    # ---------------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu and not only:
        from oracle import model as om
        from oracle.grid import Grid
        from oracle.model import Physics
        case = ci.case_c1(1)
        rng = np.random.default_rng(case.seed)
        w = ci.initial_field(case, rng)
        F = ci.forcing_field(case)
        g = Grid(case.nx, case.ny)
        phys = Physics(inv_re=case.inv_re, inv_ro=case.inv_ro)
        n = 0
        t0 = time.perf_counter()
        while n < 3 or time.perf_counter() - t0 < args.cpu_seconds:
            w = om.step(w, F, g, case.level, phys, case.dt)
            n += 1
        dt_cpu = time.perf_counter() - t0
        cpu = {"value": round(case.points * n / dt_cpu / 1e6, 4), "unit": "Mpoint-steps/s",
               "cores": 1, "kind": "oracle",
               "sample": f"{n} steps of the 512x1024 FP64 CGP-factor-2 workload "
                         f"({dt_cpu:.1f} s; NumPy/SciPy single-threaded)"}
        log(f"cpu oracle: {cpu['value']} Mpoint-steps/s over {n} steps")

    main_rate = rates.get(1, {}).get("rate")
    out = {
        "metric": METRIC,
        "value": round(main_rate, 1) if main_rate else None,
        "unit": "Mpoint-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(rates[1]["ms"] / K, 6) if 1 in rates else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "single-layer barotropic QG, 512x1024 fine grid, FP64, "
                               "CGP factor 2 (256x512 sine-transform solve), Re 450, Ro 0.0036, "
                               "dt 2.5e-5, seeded omega0", "global_batch": 1, "seq_len": None,
                   "parallelism": "single GPU",
                   "launch": ("hipGraph replays of a 3-step rotation" if rates[1]["launch"] == "graph"
                              else "direct launches") if 1 in rates else None},
        "full_grid_value": round(rates[0]["rate"], 1) if 0 in rates else None,
        "cgp4_value": round(rates[2]["rate"], 1) if 2 in rates else None,
        "speedup_cgp2_vs_full": round(rates[1]["rate"] / rates[0]["rate"], 3)
        if 0 in rates and 1 in rates else None,
        "speedup_cgp4_vs_full": round(rates[2]["rate"] / rates[0]["rate"], 3)
        if 0 in rates and 2 in rates else None,
        "launch_modes": rates[1]["modes"] if 1 in rates else None,
        "all_finite": all(v["finite"] for v in rates.values()),
        "adjoint_forward_ratio": round(adj["ratio"], 3) if adj else None,
        "adjoint": adj,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if extras:
        out["extras"] = {k: round(v, 1) for k, v in extras.items()}
    if "passes" in result:
        out["passes"] = result["passes"]
    if "diagnostics" in result:
        out["diagnostics"] = result["diagnostics"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
