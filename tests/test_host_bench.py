"""Host-side checks of bench.py's contract and helpers (no GPU)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import cgp_inputs as ci  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_algorithmic_bytes_of_the_512x1024_step():
    # per launch at l = 1: fused pass 4 fine fields + 2 spectra, pass B 2 spectra
    by = bench.pass_bytes(ci.case_c1(1), 8)
    fine, coarse = 513 * 1025 * 8, 255 * 511 * 8
    assert by["CDA"] == 4 * fine + 2 * coarse == 18911280
    assert by["B"] == 2 * coarse
    assert by["A"] == fine + coarse


def _write_csv(path, rows, fields):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def test_trace_summary_statistics(tmp_path, capsys):
    rows = [{"Kernel_Name": "void cgp::k_col_solve<double, 1024>(x)", "Start_Timestamp": s,
             "End_Timestamp": s + d} for s, d in ((0, 5000), (10000, 7000), (20000, 6000))]
    p = tmp_path / "trace.csv"
    _write_csv(p, rows, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
    bench.summarize_trace(str(p))
    out = capsys.readouterr().out.splitlines()
    assert out[2] == "| k_col_solve<double, 1024> | 3 | 6.00 | 6.00 | 5.00 | 7.00 |"


def test_pmc_summary_scales_by_the_copy(tmp_path):
    copy_kib = bench.COPY_BYTES / 1024.0
    fields = ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"]
    fetch = [{"Kernel_Name": "MulFunctor copy", "Dispatch_Id": 1, "Counter_Name": "FETCH_SIZE",
              "Counter_Value": copy_kib / 2},  # the counter sees half of the copy's reads
             {"Kernel_Name": "cgp::k_col_solve<double, 1024>(x)", "Dispatch_Id": 2,
              "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0}]
    write = [{"Kernel_Name": "MulFunctor copy", "Dispatch_Id": 1, "Counter_Name": "WRITE_SIZE",
              "Counter_Value": copy_kib},
             {"Kernel_Name": "cgp::k_col_solve<double, 1024>(x)", "Dispatch_Id": 2,
              "Counter_Name": "WRITE_SIZE", "Counter_Value": 500.0}]
    pf, pw, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "traffic.json"
    _write_csv(pf, fetch, fields)
    _write_csv(pw, write, fields)
    bench.summarize_pmc(str(pf), str(pw), out_path=str(out))
    t = json.load(open(out))
    assert t["scale_fetch"] == pytest.approx(2.0) and t["scale_write"] == pytest.approx(1.0)
    k = t["kernels"]["k_col_solve<double, 1024>"]
    assert k["fetch_bytes"] == pytest.approx(2000.0 * 1024)
    assert k["hbm_bytes_per_launch"] == pytest.approx(2500.0 * 1024)
    assert t["source_hash"] == bench.source_hash()


def test_sq_summary_is_per_wave_and_median_over_dispatches(tmp_path, capsys):
    fields = ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"]
    name = "void cgp::k_col_solve<double, 1024, 0>(x)"
    p1, p2 = [], []
    # two dispatches of 8 waves; counters split over two rows (shader engines) are summed
    for d, valu in ((1, 800.0), (2, 1200.0)):
        p1 += [{"Kernel_Name": name, "Dispatch_Id": d, "Counter_Name": "SQ_WAVES",
                "Counter_Value": 8}]
        p1 += [{"Kernel_Name": name, "Dispatch_Id": d, "Counter_Name": c, "Counter_Value": v / 2}
               for c, v in (("SQ_INSTS_VALU", valu), ("SQ_INSTS_LDS", 160.0))] * 2
        p1 += [{"Kernel_Name": name, "Dispatch_Id": d, "Counter_Name": "VALUBusy",
                "Counter_Value": 25.0}]
        p2 += [{"Kernel_Name": name, "Dispatch_Id": d, "Counter_Name": c, "Counter_Value": v}
               for c, v in (("SQ_INSTS_VALU_FMA_F64", 80.0), ("SQ_INSTS_VALU_ADD_F64", 40.0),
                            ("SQ_INSTS_VALU_MUL_F64", 16.0), ("SQ_INSTS_SALU", 24.0),
                            ("LDSBankConflict", 2.0))]
    p1.append({"Kernel_Name": "MulFunctor copy", "Dispatch_Id": 3, "Counter_Name": "SQ_WAVES",
               "Counter_Value": 4})
    f1, f2 = tmp_path / "p1.csv", tmp_path / "p2.csv"
    _write_csv(f1, p1, fields)
    _write_csv(f2, p2, fields)
    bench.summarize_sq(str(f1), str(f2))
    out = capsys.readouterr().out.splitlines()
    assert len(out) == 3
    assert out[2] == ("| k_col_solve<double, 1024, 0> | 8 | 125 | 10 / 5 / 2 | 20 | 3 "
                      "| 25.0 % | 2.0 % |")


def test_algorithmic_bytes_per_step_and_in_step_launch():
    """A fused step moves 11 fine fields and 12 coarse spectra: per stage the
    fused pass reads the psi spectra, omega_s, the forcing and (stages 2, 3)
    omega_n, writes the stage output and the next spectra; pass B reads and
    writes the spectra.  That is the fused lower bound e (11 + 12/c^2) per
    point-step of the byte model, up to the ring nodes."""
    fine, coarse = 513 * 1025 * 8, 255 * 511 * 8
    sb = bench.step_bytes(ci.case_c1(1), 8)
    assert sb["step"] == 11 * fine + 12 * coarse
    assert sb["fused_avg"] * 3 + 3 * sb["B"] == sb["step"]
    per_point = sb["step"] / (512 * 1024)
    assert abs(per_point - 8 * (11 + 12 / 4)) / per_point < 0.01
    assert bench.model_bytes(2, 8) == 184.0


def test_tuning_child_failure_falls_back(monkeypatch):
    """bench.tune_in_child: a child that aborts or times out gives no setting
    (the bench then times the reference launch); a child that finishes gives
    the setting and report it wrote."""
    def aborted(cmd, **kw):
        return subprocess.CompletedProcess(cmd, -6, "", "Aborted")
    monkeypatch.setattr(subprocess, "run", aborted)
    setting, report, why = bench.tune_in_child("ens", "f64")
    assert setting is None and report == [] and "-6" in why

    def timed_out(cmd, **kw):
        raise subprocess.TimeoutExpired(cmd, kw.get("timeout", 0))
    monkeypatch.setattr(subprocess, "run", timed_out)
    assert bench.tune_in_child("batch", "f64")[2] == "timed out"

    doc = {"setting": {"launch": dict(bench.DEFAULT_LAUNCH), "use_graph": True,
                       "fused_rows": 4},
           "report": [{"ms_per_step": 0.5, "accepted": True}]}

    def finished(cmd, **kw):
        assert cmd[-4:-1] == ["--tune-child", "ens", "f32"]
        with open(cmd[-1], "w") as f:
            json.dump(doc, f)
        return subprocess.CompletedProcess(cmd, 0, "", "")
    monkeypatch.setattr(subprocess, "run", finished)
    setting, report, why = bench.tune_in_child("ens", "f32")
    assert why is None and setting == doc["setting"] and report == doc["report"]
