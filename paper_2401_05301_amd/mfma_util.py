"""Matrix-core utilisation of the complex GEMM from rocprofv3 counters.

    python paper_2401_05301_amd/mfma_util.py [--prec fp64|fp32] --bench-json B.json \\
        --pmc P_counter_collection.csv --out profiles/zgemm_mfma_bulk_L64_chi1024

The counters come from one ``rocprofv3 --pmc MfmaUtil MfmaFlopsF64`` run of
``bench.py`` restricted to the GEMM kernel (``MfmaFlopsF32`` and
``bench.py --prec fp32`` for the FP32 theta and gate GEMMs).  MfmaUtil is the share of SIMD
cycles the matrix cores were busy during a dispatch (summed busy cycles over
all SIMDs, divided by the active cycles times the SIMD count); MfmaFlopsF64
(F32) counts the FP64 (FP32) flops the matrix cores executed (512 per counted operation),
zero-padded tile edges and whole diagonal tiles of Hermitian outputs
included.  The figures average the last N dispatches of
``zgemm_kernel<0, ...>`` (``<1, ...>`` for FP32), N being the number of GEMM launches of the timed
region (so the bench runs without the square-GEMM reference, the U(1) sample
and the serving sample, which launch GEMMs after it).  Writes <out>.json and
<out>.md (the summary).
"""
from __future__ import annotations

import argparse
import csv
import json
from collections import defaultdict

SETTINGS = {
    # counter, kernel prefix, bench flags, kernel description
    "fp64": ("MfmaFlopsF64", "zgemm_kernel<0", "", "FP64 complex GEMM, all tile shapes"),
    "fp32": ("MfmaFlopsF32", "zgemm_kernel<1", " --prec fp32", "FP32 complex GEMM of the theta and gate products"),
}


def launch_flops(roof: dict) -> float:
    """Algorithmic flops one GEMM launch issues on average in the profiled
    step (bench.py's issued_flops_per_launch; older lines: flops_per_launch)."""
    return float(roof.get("issued_flops_per_launch", roof.get("flops_per_launch")))


def command(prec: str) -> str:
    counter, _, flags, _ = SETTINGS[prec]
    return (f"rocprofv3 --pmc MfmaUtil {counter} --kernel-include-regex zgemm_kernel --output-format csv "
            f"-d <dir>/mfma -o bench_mfma -- python -u bench.py --workers 1 --steps 1 --warmup 0 --no-cpu-baseline "
            f"--serve 0 --no-u1-sample --no-square-gemm --no-precision-leg --no-fused-sample{flags}")


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
    ap.add_argument("--prec", choices=sorted(SETTINGS), default="fp64")
    a = ap.parse_args()
    counter, prefix, _, what = SETTINGS[a.prec]
    width = a.prec.upper()

    bench = None
    with open(a.bench_json) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{"):
                bench = json.loads(line)
    roof = bench["roofline"]
    n = int(roof["launches"])
    rows = dispatches(a.pmc, prefix)[-n:]
    if len(rows) != n:
        raise SystemExit(f"expected {n} GEMM dispatches, found {len(rows)}")
    util = [r["c"]["MfmaUtil"] for r in rows]
    flops = [r["c"][counter] for r in rows]
    ns = [r["ns"] for r in rows]
    timed = sum(ns) > 0
    util_mean = sum(util) / n
    util_w = sum(u * t for u, t in zip(util, ns)) / sum(ns) if timed else None
    flops_launch = sum(flops) / n
    out = {
        "kernel": f"{prefix}, ...> ({what})",
        "launches": n,
        "mfma_util_percent_mean": util_mean,
        "mfma_util_percent_time_weighted": util_w,
        f"mfma_flops_{a.prec}_per_launch": flops_launch,
        "algorithmic_flops_per_launch": launch_flops(roof),
        "executed_over_algorithmic": flops_launch / launch_flops(roof),
        "serialised_rate_TFLOPs": (sum(flops) / sum(ns) / 1e3) if timed else None,
    }
    with open(a.out + ".json", "w") as f:
        json.dump(out, f, indent=1)
    md = [
        f"# Matrix-core utilisation of the {what}, bulk chain L=64, d=5, chi=1024",
        "",
        "Commands (repository root, one MI355X; `cd /tmp && export TMPDIR=/tmp && cd /root/repo` first):",
        "",
        "```",
        command(a.prec),
        f"python paper_2401_05301_amd/mfma_util.py --prec {a.prec} --bench-json <bench line of the same run> "
        f"--pmc <dir>/mfma/bench_mfma_counter_collection.csv --out {a.out}",
        "```",
        "",
        f"- GEMM launches of the timed step: {n}.",
        f"- MfmaUtil (matrix cores busy, share of SIMD cycles): {util_mean:.1f}% averaged over launches"
        + (f", {util_w:.1f}% weighted by launch duration." if timed else "."),
        f"- {width} flops executed on the matrix cores per launch: {flops_launch / 1e9:.2f} GFLOP, "
        f"{out['executed_over_algorithmic']:.3f} times the {launch_flops(roof) / 1e9:.2f} GFLOP algorithmic "
        + ("count (the excess is the whole diagonal tiles of the Hermitian Gram products, which count as half, "
           "and the zero-padded edges of partial tiles)." if a.prec == "fp64" else
           "count (the excess is the zero-padded edges of partial tiles)."),
    ]
    if timed:
        md.append(f"- Executed rate over the profiled dispatches: {out['serialised_rate_TFLOPs']:.1f} TFLOP/s "
                  "(counter collection runs the dispatches one at a time, so launches do not overlap here).")
    md.append("")
    with open(a.out + ".md", "w") as f:
        f.write("\n".join(md))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
