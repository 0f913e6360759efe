"""Throughput of the CGP QG time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--repeats R] [--no-cpu] [--extras]

Workload (the value): single-layer barotropic QG, 512 x 1024 fine grid, FP64,
CGP factor 2 (256 x 512 coarse solve), Re 450, Ro 0.0036, dt 2.5e-5, seeded
omega0 = 1e-3 N(0,1), forcing (1/Ro) sin(pi y).  Metric: fine-grid
Mpoint-steps/s = 512 * 1024 * K / seconds over K timed steps (inputs resident
in HBM), the median of R timed runs of each launch mode (captured-graph
replays and direct launches), the faster mode's median reported.  Beside it:
the same basin with the full-grid solve (factor 1) and factor 4, the
CGP/full-grid speed-up, the two-layer workload at factors 1, 2, 4, the
64-member ensemble (FP64 and FP32, 200 steps) and a batch of 16 identical
512 x 1024 basins, the adjoint/forward time ratio of the 256 x 512, 200-step
checkpointed adjoint, per-kernel times inside time steps (HIP events around
each launch on the library's stream), the roofline of the dominant kernel and
of the whole step, and the FP64 oracle timed on the host CPU.

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
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs per launch mode and workload (the median is reported)")
    ap.add_argument("--no-tune", action="store_true",
                    help="ensembles: time the reference launch (per-pass graphs) without tuning")
    ap.add_argument("--ens-steps", type=int, default=200,
                    help="timed steps of the 64-member ensemble (the workload's 200)")
    ap.add_argument("--extras", action="store_true",
                    help="also time FP32 single basins, level 3, multigrid and adaptive steps")
    ap.add_argument("--only", default="",
                    help="comma list of sections (profiling runs): l0,l1,l2,timed,adj,c2,ens,"
                         "batch,cpu; with --extras also fp32,l3,mg,adaptive")
    ap.add_argument("--summarize-sq", nargs=2, metavar=("PASS1_CSV", "PASS2_CSV"),
                    help="print the SQ instruction mix, VALUBusy and LDSBankConflict of each "
                         "CGP kernel from two rocprofv3 --pmc passes as a markdown table and "
                         "exit (no GPU needed)")
    ap.add_argument("--tune-child", nargs=3, metavar=("KIND", "DTYPE", "OUT_JSON"),
                    help=argparse.SUPPRESS)  # the autotuner's process (see tune_in_child)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration runs)")
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV",
                    help="print per-kernel launch statistics of a rocprofv3 --kernel-trace CSV "
                         "as a markdown table and exit (no GPU needed)")
    ap.add_argument("--trace-tail", type=int, default=0, metavar="N",
                    help="with --summarize-trace: statistics over each kernel's last N launches "
                         "(the cgp_time_passes launches that end a --only timed run)")
    ap.add_argument("--trace-json", metavar="PATH",
                    help="with --summarize-trace: also write the per-kernel means (with the "
                         "kernel source hash) as JSON to PATH")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) into "
                         "per-kernel HBM bytes (default profiles/traffic_c1_l1.json) and exit")
    ap.add_argument("--pmc-out", metavar="PATH", help="with --summarize-pmc: output path")
    return ap.parse_args()


COPY_BYTES = 256 << 20


def summarize_sq(csv1, csv2):
    """Median per-dispatch SQ counters of each CGP kernel instantiation from two
    rocprofv3 --pmc passes (pass 1: VALUBusy SQ_INSTS_VALU SQ_INSTS_LDS
    SQ_WAVES ...; pass 2: LDSBankConflict SQ_INSTS_VALU_FMA_F64 / ADD / MUL
    SQ_INSTS_SALU ...), per wave where a count, as a markdown table."""
    import csv
    import statistics
    from collections import defaultdict

    def load(path):
        per = defaultdict(lambda: defaultdict(float))
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            if "cgp::" not in name:
                continue
            inst = name.split("cgp::")[1].split("(")[0]
            per[(inst, r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
        by = defaultdict(lambda: defaultdict(list))
        for (inst, _), cs in per.items():
            for c, v in cs.items():
                by[inst][c].append(v)
        return {i: {c: statistics.median(v) for c, v in cs.items()} for i, cs in by.items()}

    a, b = load(csv1), load(csv2)
    print("| kernel | waves | VALU / wave | FP64 FMA / ADD / MUL per wave | LDS / wave "
          "| SALU / wave | VALUBusy | LDSBankConflict |")
    print("|---|---|---|---|---|---|---|---|")
    for inst in sorted(a):
        x, y = a[inst], b.get(inst, {})
        w = x.get("SQ_WAVES", 0.0) or 1.0
        print(f"| {inst} | {w:.0f} | {x.get('SQ_INSTS_VALU', 0) / w:.0f} | "
              f"{y.get('SQ_INSTS_VALU_FMA_F64', 0) / w:.0f} / "
              f"{y.get('SQ_INSTS_VALU_ADD_F64', 0) / w:.0f} / "
              f"{y.get('SQ_INSTS_VALU_MUL_F64', 0) / w:.0f} | "
              f"{x.get('SQ_INSTS_LDS', 0) / w:.0f} | {y.get('SQ_INSTS_SALU', 0) / w:.0f} | "
              f"{x.get('VALUBusy', float('nan')):.1f} % | "
              f"{y.get('LDSBankConflict', float('nan')):.1f} % |")


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
        # the instantiation, e.g. k_prolong_stencil<double, 2, 2, 512, true>
        inst = name.split("cgp::")[1].split("(")[0]
        fb = fetch[name] * 1024.0 * sf
        wb = write.get(name, 0.0) * 1024.0 * sw
        out["kernels"][inst] = {"fetch_bytes": fb, "write_bytes": wb,
                                "hbm_bytes_per_launch": fb + wb}
    path = out_path or os.path.join(ROOT, "profiles", "traffic_c1_l1.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out, indent=1))


def summarize_trace(trace_csv, tail=0, json_out=None):
    """Launch count and duration statistics (us) per kernel of a kernel trace
    (tail > 0: over each kernel's last `tail` launches in start order);
    json_out: also the means, keyed by kernel, with the kernel source hash."""
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
    if json_out:
        doc = {"source_hash": source_hash(), "trace": os.path.basename(trace_csv), "tail": tail,
               "kernels": {k: {"launches": len(d), "mean_us": statistics.mean(d),
                               "median_us": statistics.median(d)} for k, d in per.items()}}
        json.dump(doc, open(json_out, "w"), indent=1)


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
    """Hash of every kernel and runtime source and the build flags: profile
    figures taken with other sources are not used."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1308_3290_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    # the compile flags are part of the kernels too
    h.update(open(os.path.join(ROOT, "paper_1308_3290_amd", "build.py"), "rb").read())
    return h.hexdigest()[:16]


def step_bytes(case, es):
    """Algorithmic bytes of one fused time step (three stages): per stage the
    fused pass reads the psi spectra S, the stage input, the forcing and (in
    stages 2 and 3) omega_n, writes the stage output and the next spectra S;
    pass B reads and writes S.  Over a step: 11 F + 12 S (F a fine field)."""
    fine = (case.nx + 1) * (case.ny + 1) * case.nlayers * es
    c = 2 ** case.level
    coarse = (case.nx // c - 1) * (case.ny // c - 1) * case.nlayers * es
    return {"fine": fine, "coarse": coarse, "step": 11 * fine + 12 * coarse,
            "fused_avg": (11 * fine + 6 * coarse) / 3.0, "B": 2 * coarse}


def model_bytes(c, es):
    """Bytes per fine point-step of the four-pass model, e (20 + 12/c^2)."""
    return es * (20 + 12 / (c * c))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_share():
    """Cores this process may use, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def median(xs):
    import statistics
    return statistics.median(xs)


# the launch a handle starts with (cgp_set_launch is not needed for it)
DEFAULT_LAUNCH = {"mode": 0, "b_tile": 1, "f_tile": 1, "wg_per_cu": 0}


def tune_workload(kind, dtype_):
    """Configs and inputs of a tuned bench workload: "ens" the 64-member
    ensemble, "batch" 16 copies of the 512x1024 level-1 basin."""
    import numpy as np

    import cgp_inputs as ci
    from paper_1308_3290_amd import api
    if kind == "ens":
        members = ci.ensemble_c3(dtype=dtype_)
        return ([api.config_from_case(m.case) for m in members], [m.omega0 for m in members],
                [m.forcing for m in members])
    case = ci.case_c1(1)
    rng = np.random.default_rng(case.seed)
    w0, F = ci.initial_field(case, rng), ci.forcing_field(case)
    return [api.config_from_case(case)] * 16, [w0] * 16, [F] * 16


def tune_child(kind, dtype_, out_json):
    """The autotuner run for one workload (retuned, every candidate timed and
    checked against the reference launch); writes the chosen setting and the
    report to out_json."""
    import torch

    from paper_1308_3290_amd import api, autotune
    cfgs, w0s, Fs = tune_workload(kind, dtype_)
    probe = api.Ensemble(cfgs, device=torch.device("cuda:0"))
    Wp, Fpk = probe.pack(w0s), probe.pack(Fs)
    probe.close()
    report = []
    setting = autotune.tune(cfgs, Wp, Fpk, steps=30, warmup=6, repeats=3, report=report,
                            retune=True)
    with open(out_json, "w") as f:
        json.dump({"setting": setting, "report": report}, f)


def tune_in_child(kind, dtype_):
    """Run tune_child in a child process, so that a failure while the tuner
    creates, steps and destroys its many candidate handles cannot end the
    measurement; returns (setting, report, None), or (None, [], why)."""
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "tune.json")
        cmd = [sys.executable, os.path.abspath(__file__), "--tune-child", kind, dtype_, out]
        try:
            r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
        except subprocess.TimeoutExpired:
            return None, [], "timed out"
        if r.returncode != 0 or not os.path.exists(out):
            log(r.stderr[-2000:])
            return None, [], f"exit status {r.returncode}"
        with open(out) as f:
            doc = json.load(f)
        return doc["setting"], doc["report"], None


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.trace_tail, args.trace_json)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, out_path=args.pmc_out)
        return
    if args.summarize_sq:
        summarize_sq(*args.summarize_sq)
        return
    if args.tune_child:
        tune_child(*args.tune_child)
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
    want = (lambda k: not only or k in only)
    K, W, R = args.steps, args.warmup, max(1, args.repeats)

    def timed_runs(cfgs, w0s, Fs, steps, warm, use_graph, reps, launch=None):
        """reps timed runs of `steps` steps of an ensemble (one member: a single
        basin) on a non-default stream (graphs cannot be captured on the
        default one), HIP events recorded on that stream; ms per run."""
        ens = api.Ensemble(cfgs, device=dev)
        if launch is not None and launch != DEFAULT_LAUNCH:
            ens.set_launch(**launch)
        w = ens.pack(w0s)
        Fp = ens.pack(Fs)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            ens.step(w, Fp, nsteps=warm, use_graph=use_graph)
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(s):
                e0.record(s)
                ens.step(w, Fp, nsteps=steps, use_graph=use_graph)
                e1.record(s)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        finite = bool(torch.isfinite(w).all().item())
        del ens, w, Fp
        return out, finite

    def basin_inputs(case):
        rng = np.random.default_rng(case.seed)
        w0 = ci.initial_field(case, rng)
        F = ci.forcing_field(case)
        if case.nlayers == 2:  # packed fields hold both layers (layer-2 forcing unused)
            F = np.stack([F, np.zeros_like(F)])
        return w0, F

    def rate_both_modes(case, steps, warm, label, dtype="f64"):
        """Median rate of each launch mode; the faster mode's median wins."""
        w0, F = basin_inputs(case)
        cfg = api.config_from_case(case, dtype)
        by_mode = {}
        for mode in ("graph", "direct"):
            ms, finite = timed_runs([cfg], [w0], [F], steps, warm, mode == "graph", R)
            rates = [case.points * steps / (m * 1e-3) / 1e6 for m in ms]
            by_mode[mode] = dict(ms=median(ms), rate=median(rates), finite=finite, launch=mode,
                                 runs=[round(r, 1) for r in rates])
            log(f"{label} ({mode}): {median(ms) / steps * 1e3:.1f} us/step, median "
                f"{median(rates):.0f} Mpoint-steps/s over {R} runs {by_mode[mode]['runs']} "
                f"(finite={finite})")
        best = dict(max(by_mode.values(), key=lambda r: r["rate"]))
        best["modes"] = {m: round(r["rate"], 1) for m, r in by_mode.items()}
        best["runs_by_mode"] = {m: r["runs"] for m, r in by_mode.items()}
        return best

    out = {}
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
        if want(f"l{lv}"):
            rates[lv] = rate_both_modes(ci.case_c1(lv), K, W, f"512x1024 FP64 level {lv}")
    # ---------------------------------------------------------------- kernels in the step
    roof = None
    passes = None
    if want("timed"):
        case = ci.case_c1(1)
        w0, F0 = basin_inputs(case)
        b = api.Basin(api.config_from_case(case), device=dev)
        w = torch.as_tensor(w0, device=dev)
        F = torch.as_tensor(F0, device=dev)
        b.step(w, F, nsteps=2)  # fills psi, the stage buffers and the spectra
        # back-to-back launches of each pass alone (hot inputs)
        api.cgp_time_passes(b.handle, w, F, 10)
        ms = api.cgp_time_passes(b.handle, w, F, 200)
        by = pass_bytes(case, 8)
        names = ["A", "B", "C", "D", "CD", "CDA"]
        kernel_names = {"A": "k_restrict_rowdst", "B": "k_col_solve", "C": "k_rowdst_prolong",
                        "D": "k_stencil_rk3", "CD": "k_prolong_stencil<NEXT=false>",
                        "CDA": "k_prolong_stencil<NEXT=true>"}
        passes = {kernel_names[n]: {"us_back_to_back": round(ms[j] * 1e3, 3),
                                    "alg_bytes_per_launch": by[n]}
                  for j, n in enumerate(names) if ms[j] > 0}
        # diagnostics (E and Z, eq. 26): outside the time step, timed on
        # their own over the same fields; they read psi and omega once
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
        out["diagnostics"] = {"us_per_call": round(us, 2), "alg_bytes_per_call": dbytes,
                              "achieved_GBs": round(dbytes / (us * 1e-6) / 1e9, 1)}
        log(f"diagnostics: {us:.1f} us per call ({dbytes / (us * 1e-6) / 1e9:.0f} GB/s)")
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
        # the kernels inside time steps: HIP events on the library's stream
        # around every pass B and fused launch of IN_STEP steps (the last
        # launches of this section, so that a kernel trace's last 3 * IN_STEP
        # launches of each kernel are these)
        IN_STEP = 100
        api.cgp_time_step_passes(b.handle, w, F, 10)
        mb, mf, mstep = api.cgp_time_step_passes(b.handle, w, F, IN_STEP)
        sb = step_bytes(case, 8)
        passes["k_col_solve"].update(us_in_step=round(mb * 1e3, 3), alg_bytes_in_step=sb["B"])
        passes["k_prolong_stencil<NEXT=true>"].update(us_in_step=round(mf * 1e3, 3),
                                                      alg_bytes_in_step=sb["fused_avg"])
        for k, v in passes.items():
            t = v.get("us_in_step", v["us_back_to_back"])
            nb = v.get("alg_bytes_in_step", v["alg_bytes_per_launch"])
            v["achieved_GBs"] = round(nb / (t * 1e-6) / 1e9, 1)
            v["in_time_step"] = "us_in_step" in v
        log("per-pass: " + json.dumps(passes))
        dom, t_dom, b_dom = max((("k_prolong_stencil<NEXT=true>", mf, sb["fused_avg"]),
                                 ("k_col_solve", mb, sb["B"])), key=lambda x: x[1])
        achieved = b_dom / (t_dom * 1e-3) / 1e9
        def instance(doc):
            """The dominant kernel's entry of a profile summary (the 512-point
            compile-time instantiations that the 512x1024 level-1 step runs)."""
            if doc.get("source_hash") != source_hash():
                return None
            # (the fused kernel's last template argument is the store form)
            want = ("k_prolong_stencil<double, 2, 2, 512, true, "
                    if dom.startswith("k_prolong_stencil") else "k_col_solve<double, 1024, 0>")
            hits = [v for k, v in doc.get("kernels", {}).items() if k.startswith(want)]
            return hits[0] if len(hits) == 1 else None

        traffic = None
        tfile = os.path.join(ROOT, "profiles", "traffic_c1_l1.json")
        if os.path.exists(tfile):
            e = instance(json.load(open(tfile)))
            traffic = e["hbm_bytes_per_launch"] if e else None
        prof_us = None
        pfile = os.path.join(ROOT, "profiles", "trace_c1_l1.json")
        if os.path.exists(pfile):
            e = instance(json.load(open(pfile)))
            prof_us = round(e["mean_us"], 3) if e else None
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic, "alg_bytes_per_launch": round(b_dom),
                "us_per_launch": round(t_dom * 1e3, 3),
                "timing": f"HIP events around each launch inside {IN_STEP} time steps "
                          "(mean over the three stages' launches)",
                "profile_us_per_launch": prof_us,
                "frac_from_profile": round(b_dom / (prof_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)
                if prof_us else None,
                "achievable_copy": round(best, 1), "frac_of_achievable": round(achieved / best, 4)}
        out["in_step_ms_per_step_with_events"] = round(mstep, 6)
        if 1 in rates:
            # the fused pass's share of the step wall time without events:
            # a step is three (pass B, fused pass) pairs; pass B back to back
            t_b = ms[names.index("B")]
            share = rates[1]["ms"] / K / 3.0 - t_b
            roof["us_step_share"] = round(share * 1e3, 3)
        del b, w, F, psi
    # ---------------------------------------------------------------- two layers
    two = {}
    if want("c2"):
        for lv in (1, 0, 2):
            case = ci.case_c2(lv)
            n = min(K, case.nsteps) if K >= 100 else 100
            r = rate_both_modes(case, n, W, f"two-layer 512x1024 FP64 level {lv}")
            two[f"l{lv}"] = {"value": round(r["rate"], 1), "launch": r["launch"],
                             "modes": r["modes"], "us_per_step": round(r["ms"] / n * 1e3, 2),
                             "steps": n,
                             "frac_step_alg": round(step_bytes(case, 8)["step"] / (r["ms"] / n * 1e-3)
                                                    / 1e9 / PEAK_HBM_GBS, 4)}
    # ---------------------------------------------------------------- ensembles
    ens_out = {}

    def tuned_rate(cfgs, w0s, Fs, n_steps, label, kind, dtype_):
        """The autotuner's choice of launch for this workload (every candidate
        checked bit for bit against the reference launch; tuned in a process
        of its own, see tune_in_child), then R timed runs of it; also the best
        time of each launch mode among the candidates."""
        from paper_1308_3290_amd import autotune
        report = []
        if args.no_tune:
            setting = dict(autotune.REFERENCE)
        else:
            setting, report, why = tune_in_child(kind, dtype_)
            if setting is None:
                log(f"{label}: tuning failed ({why}); timing the reference launch")
                setting = dict(autotune.REFERENCE, tuning=f"failed ({why}); reference launch")
        ms, finite = timed_runs(autotune.configs(cfgs, setting), w0s, Fs, n_steps, 5,
                                setting["use_graph"], max(3, R // 2), launch=setting["launch"])
        best_by_mode = {}
        for r in report:
            k = ("persistent" if r["launch"]["mode"] == 1 else
                 ("per-pass graphs" if r["use_graph"] else "per-pass direct"))
            if r.get("fused_rows", 2) == 4:
                k += ", 4 rows per block"
            if r["accepted"] and (k not in best_by_mode or r["ms_per_step"] < best_by_mode[k][0]):
                best_by_mode[k] = (r["ms_per_step"], r["launch"])
        log(f"{label}: tuned {setting} over {len(report)} candidates "
            f"({sum(r['accepted'] for r in report)} accepted); best per mode "
            + json.dumps({k: round(v[0], 4) for k, v in best_by_mode.items()}))
        return ms, finite, setting, best_by_mode

    if want("ens"):
        n_ens = args.ens_steps
        for dt_ in ("f64", "f32"):
            members = ci.ensemble_c3(dtype=dt_)
            cfgs = [api.config_from_case(m.case) for m in members]
            ms, finite, setting, by_mode = tuned_rate(
                cfgs, [m.omega0 for m in members], [m.forcing for m in members], n_ens,
                f"ensemble 64 {dt_}", "ens", dt_)
            pts = sum(m.case.points for m in members)
            es = 8 if dt_ == "f64" else 4
            alg = sum(step_bytes(m.case, es)["step"] for m in members)
            t = median(ms) * 1e-3 / n_ens
            ens_out[dt_] = {"value": round(pts / t / 1e6, 1), "unit": "Mpoint-steps/s",
                            "members": len(members), "points": pts, "steps": n_ens,
                            "runs": [round(pts * n_ens / (m * 1e-3) / 1e6, 1) for m in ms],
                            "alg_bytes_per_step": alg, "GBs_alg": round(alg / t / 1e9, 1),
                            "frac_alg": round(alg / t / 1e9 / PEAK_HBM_GBS, 4),
                            "GBs_model": round(pts * model_bytes(2, es) / t / 1e9, 1),
                            "finite": finite, "launch": setting,
                            "tuning_best_Mpts_by_mode": {
                                k: round(pts / (v[0] * 1e-3) / 1e6, 1)
                                for k, v in by_mode.items()}}
            log(f"ensemble 64 {dt_}: {ens_out[dt_]}")
    batch = None
    if want("batch"):
        # the 512 x 1024 level-1 kernel set as a batch of 16 identical basins
        case = ci.case_c1(1)
        w0, F = basin_inputs(case)
        cfgs = [api.config_from_case(case)] * 16
        n_b = 100
        ms, finite, setting, by_mode = tuned_rate(cfgs, [w0] * 16, [F] * 16, n_b,
                                                  "batch of 16 x 512x1024", "batch", "f64")
        t = median(ms) * 1e-3 / n_b
        sb = step_bytes(case, 8)["step"] * 16
        batch = {"value": round(16 * case.points / t / 1e6, 1), "unit": "Mpoint-steps/s",
                 "basins": 16, "steps": n_b, "GBs_alg": round(sb / t / 1e9, 1),
                 "frac_alg": round(sb / t / 1e9 / PEAK_HBM_GBS, 4), "finite": finite,
                 "launch": setting,
                 "tuning_best_Mpts_by_mode": {k: round(16 * case.points / (v[0] * 1e-3) / 1e6, 1)
                                              for k, v in by_mode.items()}}
        log(f"batch of 16 x 512x1024 level 1: {batch}")
    # ---------------------------------------------------------------- adjoint ratio
    adj = None
    if not args.no_adjoint and want("adj"):
        p = ci.adjoint_c4()
        c = p.case
        b = api.Basin(api.config_from_case(c), device=dev)
        w0 = torch.as_tensor(p.omega0, device=dev).requires_grad_(True)
        F = torch.as_tensor(p.forcing, device=dev).requires_grad_(True)
        idx = torch.as_tensor(p.obs_index, device=dev)
        obs = torch.as_tensor(p.obs_value, device=dev)
        fw, bw = [], []
        for rep in range(1 + max(3, R // 2)):  # the first pass warms up
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
            if rep:
                fw.append((t1 - t0) * 1e3)
                bw.append((t3 - t2) * 1e3)
        adj = {"forward_ms": round(median(fw), 3), "backward_ms": round(median(bw), 3),
               "ratio": round(median(bw) / median(fw), 3),
               "ratios": [round(y / x, 3) for x, y in zip(fw, bw)],
               "workload": "256x512 FP64 CGP factor 2, 200 steps, checkpoint every 20, "
                           "final-time misfit at 1% of nodes"}
        log(f"adjoint: forward {adj['forward_ms']:.1f} ms, backward {adj['backward_ms']:.1f} ms, "
            f"ratio {adj['ratio']:.2f}")
        del b, w0, F
    # ---------------------------------------------------------------- extras
    extras = {}
    if args.extras:
        def rate(case, steps, warm=W, dtype="f64"):
            w0, F = basin_inputs(case)
            ms, _ = timed_runs([api.config_from_case(case, dtype)], [w0], [F], steps, warm, True,
                               3)
            return case.points * steps / (median(ms) * 1e-3) / 1e6
        if want("l3"):  # three levels of coarsening (64x128 solve)
            extras["cgp8_l3"] = rate(ci.case_c1(3), min(K, 500))
        if want("mg"):  # the multigrid coarse solver (12 V-cycles) at levels 0, 1, 2
            for lv in (0, 1, 2):
                case = ci.case_c1(lv)
                case.solver = 1
                extras[f"multigrid_l{lv}"] = rate(case, 20, 2)
        if want("adaptive"):  # the step size of Sec. 4.2 (CFL 0.5, capped at dt)
            case = ci.case_c1(1)
            case.cfl = 0.5
            extras["adaptive_l1"] = rate(case, K)
        for lv in (1, 0):
            if want("fp32"):
                extras[f"fp32_l{lv}"] = rate(ci.case_c1(lv), K, dtype="f32")
        log("extras: " + json.dumps(extras))
    # ---------------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu and want("cpu"):
        import scipy.fft

        from oracle import model as om
        from oracle.grid import Grid
        from oracle.model import Physics
        share = cpu_share()
        table = {}

        def per_step(case, steps=4, reps=3):
            w, F = basin_inputs(case)
            if case.nlayers == 2:
                F = F[0]
            g = Grid(case.nx, case.ny)
            phys = Physics(inv_re=case.inv_re, inv_ro=case.inv_ro, f1=case.f1, f2=case.f2,
                           drag=case.drag)
            fn = om.step if case.nlayers == 1 else om.step_two_layer
            w = fn(w, F, g, case.level, phys, case.dt)  # warm-up
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                for _ in range(steps):
                    w = fn(w, F, g, case.level, phys, case.dt)
                ts.append((time.perf_counter() - t0) / steps)
            return median(ts), steps * reps + 1
        t_all = time.perf_counter()
        total_steps = 0
        for workers in (1, share):
            with scipy.fft.set_workers(workers):
                for name, case in (("c1_l0", ci.case_c1(0)), ("c1_l1", ci.case_c1(1)),
                                   ("c1_l2", ci.case_c1(2)), ("c2_l0", ci.case_c2(0)),
                                   ("c2_l1", ci.case_c2(1)), ("c2_l2", ci.case_c2(2))):
                    t, n = per_step(case)
                    total_steps += n
                    table[f"{name}_workers{workers}"] = round(case.points / t / 1e6, 3)
            if share == 1:
                break
        wall = time.perf_counter() - t_all
        k1 = f"c1_l1_workers{share}"
        head_key = max(("c1_l1_workers1", k1), key=lambda k: table[k])
        cpu = {"value": table[head_key], "unit": "Mpoint-steps/s",
               "cores": 1 if head_key.endswith("workers1") else share, "kind": "oracle",
               "sample": f"FP64 oracle steps of the 512x1024 one-layer workload at level 1 "
                         f"(median of 3 runs of 4 steps after one warm-up step; the table also "
                         f"holds levels 0 and 2 and the two-layer workload, with scipy.fft "
                         f"workers = 1 and = {share}; {total_steps} steps, {wall:.1f} s in all)",
               "table": table, "nproc": os.cpu_count(), "cpu_share": share,
               "cpu_model": cpu_model()}
        log(f"cpu oracle: {json.dumps(cpu)}")

    main_rate = rates.get(1, {}).get("rate")
    c1 = ci.case_c1(1)
    step_roof = None
    if 1 in rates:
        t = rates[1]["ms"] * 1e-3 / K
        sb = step_bytes(c1, 8)["step"]
        step_roof = {"alg_bytes_per_step": sb, "GBs_alg": round(sb / t / 1e9, 1),
                     "frac_alg": round(sb / t / 1e9 / PEAK_HBM_GBS, 4),
                     "model_bytes_per_point_step": model_bytes(2, 8),
                     "frac_model": round(c1.points * model_bytes(2, 8) / t / 1e9 / PEAK_HBM_GBS,
                                         4)}
    res = {
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
                              else "direct launches") if 1 in rates else None,
                   "repeats": R, "statistic": "median of the repeats, faster launch mode"},
        "full_grid_value": round(rates[0]["rate"], 1) if 0 in rates else None,
        "cgp4_value": round(rates[2]["rate"], 1) if 2 in rates else None,
        "speedup_cgp2_vs_full": round(rates[1]["rate"] / rates[0]["rate"], 3)
        if 0 in rates and 1 in rates else None,
        "speedup_cgp4_vs_full": round(rates[2]["rate"] / rates[0]["rate"], 3)
        if 0 in rates and 2 in rates else None,
        "launch_modes": rates[1]["modes"] if 1 in rates else None,
        "runs": rates[1]["runs_by_mode"] if 1 in rates else None,
        "all_finite": all(v["finite"] for v in rates.values()),
        "step_roofline": step_roof,
        "adjoint_forward_ratio": adj["ratio"] if adj else None,
        "adjoint": adj,
        "roofline": roof,
        "cpu_baseline": cpu,
        "two_layer": two or None,
        "ensemble64": ens_out or None,
        "batch16_c1_l1": batch,
    }
    if extras:
        res["extras"] = {k: round(v, 1) for k, v in extras.items()}
    if passes:
        res["passes"] = passes
    res.update(out)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
