"""Counter summaries of the profiling tools on small synthetic counter files."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FIELDS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
          "End_Timestamp"]


def _write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_mfma_util_summary(tmp_path):
    gemm = "void ptebd::zgemm_kernel<0, 64, 64, 16, 2, 2>(ptebd::ZGemmArgs)"
    rows = []
    # an earlier dispatch (outside the timed region) and two timed ones
    for did, util, fl, t0, t1 in [(1, 99.0, 1e9, 0, 10), (5, 20.0, 2e9, 100, 200), (9, 60.0, 6e9, 300, 600)]:
        for name, val in [("MfmaUtil", util), ("MfmaFlopsF64", fl)]:
            rows.append({"Correlation_Id": did, "Dispatch_Id": did, "Kernel_Name": gemm, "Counter_Name": name,
                         "Counter_Value": val, "Start_Timestamp": t0, "End_Timestamp": t1})
    rows.append({"Correlation_Id": 7, "Dispatch_Id": 7, "Kernel_Name": "herm_apply", "Counter_Name": "MfmaUtil",
                 "Counter_Value": 1.0, "Start_Timestamp": 0, "End_Timestamp": 1})
    pmc = tmp_path / "c.csv"
    _write_csv(pmc, rows)
    bench = tmp_path / "b.log"
    bench.write_text("[bench] noise\n" + json.dumps({"roofline": {"launches": 2, "flops_per_launch": 4e9}}) + "\n")
    out = tmp_path / "summary"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "paper_2401_05301_amd", "mfma_util.py"), "--bench-json",
                        str(bench), "--pmc", str(pmc), "--out", str(out)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    s = json.loads((tmp_path / "summary.json").read_text())
    assert s["launches"] == 2
    assert abs(s["mfma_util_percent_mean"] - 40.0) < 1e-12
    assert abs(s["mfma_util_percent_time_weighted"] - (20.0 * 100 + 60.0 * 300) / 400) < 1e-12
    assert abs(s["mfma_flops_fp64_per_launch"] - 4e9) < 1e-3
    assert abs(s["executed_over_algorithmic"] - 1.0) < 1e-12
    assert abs(s["serialised_rate_TFLOPs"] - 8e9 / 400 / 1e3) < 1e-12
    assert "MfmaUtil" in (tmp_path / "summary.md").read_text()


def test_mfma_util_rejects_missing_dispatches(tmp_path):
    pmc = tmp_path / "c.csv"
    _write_csv(pmc, [])
    bench = tmp_path / "b.log"
    bench.write_text(json.dumps({"roofline": {"launches": 3, "flops_per_launch": 1.0}}) + "\n")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "paper_2401_05301_amd", "mfma_util.py"), "--bench-json",
                        str(bench), "--pmc", str(pmc), "--out", str(tmp_path / "s")], capture_output=True, text=True)
    assert r.returncode != 0 and "expected 3 GEMM dispatches" in r.stderr
