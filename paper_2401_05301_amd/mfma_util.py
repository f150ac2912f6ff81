"""Matrix-core utilisation of the FP64 complex GEMM from rocprofv3 counters.

    python paper_2401_05301_amd/mfma_util.py --bench-json B.json \\
        --pmc P_counter_collection.csv --out profiles/zgemm_mfma_bulk_L64_chi1024

The counters come from one ``rocprofv3 --pmc MfmaUtil MfmaFlopsF64`` run of
``bench.py`` restricted to the GEMM kernel.  MfmaUtil is the share of SIMD
cycles the matrix cores were busy during a dispatch (summed busy cycles over
all SIMDs, divided by the active cycles times the SIMD count); MfmaFlopsF64
counts the FP64 flops the matrix cores executed (512 per counted operation),
zero-padded tile edges and whole diagonal tiles of Hermitian outputs
included.  The figures average the last N dispatches of
``zgemm_kernel<0, ...>``, N being the number of GEMM launches of the timed
region (so the bench runs without the square-GEMM reference, the U(1) sample
and the serving sample, which launch GEMMs after it).  Writes <out>.json and
<out>.md (the summary).
"""
from __future__ import annotations

import argparse
import csv
import json
from collections import defaultdict

COMMAND = (
    "rocprofv3 --pmc MfmaUtil MfmaFlopsF64 --kernel-include-regex zgemm_kernel --output-format csv "
    "-d <dir>/mfma -o bench_mfma -- python -u bench.py --no-cpu-baseline --serve 0 --no-u1-sample "
    "--no-square-gemm"
)


def dispatches(path: str, name_part: str):
    """Per dispatch id: kernel name, duration in ns (0 if the file has no
    timestamps) and every counter value."""
    out = defaultdict(lambda: {"name": "", "ns": 0.0, "c": {}})
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if name_part not in r["Kernel_Name"]:
                continue
            d = out[int(r["Dispatch_Id"])]
            d["name"] = r["Kernel_Name"]
            d["c"][r["Counter_Name"]] = float(r["Counter_Value"])
            if r.get("Start_Timestamp") and r.get("End_Timestamp"):
                d["ns"] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    return [out[k] for k in sorted(out)]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--pmc", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    bench = None
    with open(a.bench_json) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{"):
                bench = json.loads(line)
    roof = bench["roofline"]
    n = int(roof["launches"])
    rows = dispatches(a.pmc, "zgemm_kernel<0")[-n:]
    if len(rows) != n:
        raise SystemExit(f"expected {n} GEMM dispatches, found {len(rows)}")
    util = [r["c"]["MfmaUtil"] for r in rows]
    flops = [r["c"]["MfmaFlopsF64"] for r in rows]
    ns = [r["ns"] for r in rows]
    timed = sum(ns) > 0
    util_mean = sum(util) / n
    util_w = sum(u * t for u, t in zip(util, ns)) / sum(ns) if timed else None
    flops_launch = sum(flops) / n
    out = {
        "kernel": "zgemm_kernel<0, ...> (FP64 complex GEMM, all tile shapes)",
        "launches": n,
        "mfma_util_percent_mean": util_mean,
        "mfma_util_percent_time_weighted": util_w,
        "mfma_flops_f64_per_launch": flops_launch,
        "algorithmic_flops_per_launch": roof["flops_per_launch"],
        "executed_over_algorithmic": flops_launch / roof["flops_per_launch"],
        "serialised_rate_TFLOPs": (sum(flops) / sum(ns) / 1e3) if timed else None,
    }
    with open(a.out + ".json", "w") as f:
        json.dump(out, f, indent=1)
    md = [
        "# Matrix-core utilisation of the FP64 complex GEMM, bulk chain L=64, d=5, chi=1024",
        "",
        "Commands (repository root, one MI355X; `cd /tmp && export TMPDIR=/tmp && cd /root/repo` first):",
        "",
        "```",
        COMMAND,
        "python paper_2401_05301_amd/mfma_util.py --bench-json <bench line of the same run> "
        "--pmc <dir>/mfma/bench_mfma_counter_collection.csv --out profiles/zgemm_mfma_bulk_L64_chi1024",
        "```",
        "",
        f"- GEMM launches of the timed step: {n}.",
        f"- MfmaUtil (matrix cores busy, share of SIMD cycles): {util_mean:.1f}% averaged over launches"
        + (f", {util_w:.1f}% weighted by launch duration." if timed else "."),
        f"- FP64 flops executed on the matrix cores per launch: {flops_launch / 1e9:.2f} GFLOP, "
        f"{out['executed_over_algorithmic']:.3f} times the {roof['flops_per_launch'] / 1e9:.2f} GFLOP algorithmic "
        "count (the excess is the whole diagonal tiles of the Hermitian Gram products, which count as half, and "
        "the zero-padded edges of partial tiles).",
    ]
    if timed:
        md.append(f"- Executed rate over the profiled dispatches: {out['serialised_rate_TFLOPs']:.1f} TFLOP/s "
                  "(counter collection runs the dispatches one at a time, so the four gate workers do not overlap "
                  "here).")
    md.append("")
    with open(a.out + ".md", "w") as f:
        f.write("\n".join(md))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
