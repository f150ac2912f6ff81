"""Kernel statistics of a profiled bench.py run, reduced to a short summary.

    python paper_2401_05301_amd/kernel_stats.py --stats S_kernel_stats.csv \\
        [--trace T_kernel_trace.csv] --bench-json B.json --command "<profiled command>" \\
        --title "<workload>" --out profiles/<name>

Inputs are the CSV files of ``rocprofv3 --kernel-trace --stats
--output-format csv`` and the JSON line the same bench.py run printed.
Writes <out>.md (the per-kernel table, largest first, and the FP64 GEMM
averages) and <out>.json.  With a trace, the average duration of the last N
dispatches of the FP64 GEMM kernel is given next to the one bench.py measured
with HIP events, N being the launches of bench.py's profiled step (its last
GEMM-launching phase when the auxiliary legs are switched off).
"""
from __future__ import annotations

import argparse
import csv
import json
import re

GEMM = "zgemm_kernel<0"


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("ptebd::", "")
    name = re.sub(r"^void ", "", name)
    depth, out = 0, []
    for ch in name:        # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def col(row: dict, *names):
    for n in names:
        for k in row:
            if k.lower() == n.lower():
                return row[k]
    raise KeyError(names)


def read_bench(path: str):
    bench = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{"):
                bench = json.loads(line)
    if bench is None:
        raise SystemExit(f"no JSON line in {path}")
    return bench


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--trace")
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    rows = []
    with open(a.stats, newline="") as f:
        for r in csv.DictReader(f):
            rows.append((short_name(col(r, "Name", "Kernel_Name")), int(col(r, "Calls")),
                         float(col(r, "TotalDurationNs", "Total_Duration_Ns")) / 1e6))
    total_ms = sum(r[2] for r in rows)
    rows.sort(key=lambda r: -r[2])
    gemm_calls = sum(r[1] for r in rows if r[0].startswith(GEMM))
    gemm_ms = sum(r[2] for r in rows if r[0].startswith(GEMM))

    bench = read_bench(a.bench_json)
    roof = bench.get("roofline", {})
    out = {"title": a.title, "command": a.command, "kernel_total_ms": total_ms,
           "gemm_fp64_calls": gemm_calls, "gemm_fp64_avg_ms": gemm_ms / max(gemm_calls, 1),
           "bench_value": bench.get("value"), "bench_ms_per_step": bench.get("ms_per_step"),
           "bench_gemm_launches": roof.get("launches"), "bench_gemm_avg_launch_ms": roof.get("avg_launch_ms"),
           "kernels": [{"name": n, "calls": c, "ms": t} for n, c, t in rows[:a.top]]}
    if a.trace and roof.get("launches"):
        n = int(roof["launches"])
        disp = []
        with open(a.trace, newline="") as f:
            for r in csv.DictReader(f):
                if GEMM in col(r, "Kernel_Name"):
                    disp.append((int(col(r, "Dispatch_Id")),
                                 (int(col(r, "End_Timestamp")) - int(col(r, "Start_Timestamp"))) / 1e6))
        disp.sort()
        last = disp[-n:]
        out["trace_last_n_gemm_dispatches"] = len(last)
        out["trace_last_n_gemm_avg_ms"] = sum(d for _, d in last) / max(len(last), 1)

    with open(a.out + ".json", "w") as f:
        json.dump(out, f, indent=1)
    md = [f"# Kernel statistics: {a.title}", "", "Command (repository root, one MI355X; "
          "`cd /tmp && export TMPDIR=/tmp && cd /root/repo` first):", "", "```", a.command, "```", "",
          "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for n, c, t in rows[:a.top]:
        md.append(f"| `{n}` | {c} | {t:.1f} | {1e3 * t / max(c, 1):.1f} | {100 * t / total_ms:.2f} |")
    md += ["", f"All kernels: {total_ms:.0f} ms. FP64 GEMM (`zgemm_kernel<0, ...>`, both tile shapes): "
               f"{gemm_calls} launches, {gemm_ms:.0f} ms, average {out['gemm_fp64_avg_ms']:.3f} ms (whole program)."]
    if "trace_last_n_gemm_avg_ms" in out:
        md.append(f"FP64 GEMM over the last {out['trace_last_n_gemm_dispatches']} dispatches (bench.py's profiled "
                  f"step): average {out['trace_last_n_gemm_avg_ms']:.3f} ms from the trace, against "
                  f"{roof['avg_launch_ms']:.3f} ms from bench.py's HIP events over the same "
                  f"{roof['launches']} launches.")
    if bench.get("value") is not None:
        md.append(f"Bench line of the same run: {bench['value']:.3f} gate-updates/s, "
                  f"{bench.get('ms_per_step', 0) / 1e3:.1f} s per step; GEMM roofline achieved "
                  f"{roof.get('achieved', 0):.1f} TFLOP/s ({100 * roof.get('frac', 0):.1f}% of {roof.get('peak')}).")
    md.append("")
    with open(a.out + ".md", "w") as f:
        f.write("\n".join(md))
    print(json.dumps({k: v for k, v in out.items() if k != "kernels"}))


if __name__ == "__main__":
    main()
