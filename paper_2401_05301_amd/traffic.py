"""HBM traffic per launch of the FP64 complex GEMM from rocprofv3 counters.

    python paper_2401_05301_amd/traffic.py --bench-json B.json \\
        --fetch F_counter_collection.csv --write W_counter_collection.csv \\
        --copy-fetch CF_counter_collection.csv --copy-write CW_counter_collection.csv \\
        --copy-bytes 1073741824 --out profiles/zgemm_traffic_bulk_L64_chi1024

The counters come from four ``rocprofv3 --pmc`` runs (FETCH_SIZE, then
WRITE_SIZE) of ``bench.py`` and of its device-to-device copy calibration.
FETCH_SIZE and WRITE_SIZE report KiB per dispatch; each is scaled by the
ratio of the known copy size to what the same counter reads for the copy.
The GEMM figures average the last N dispatches of ``zgemm_kernel<0, ...>``,
N being the number of GEMM launches of bench.py's timed region (so the
bench must be run without the square-GEMM reference, the U(1) sample and the
serving sample, which launch GEMMs after it).  Writes <out>.json (read by bench.py) and <out>.md (the summary).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def launch_flops(roof: dict) -> float:
    """Algorithmic flops one GEMM launch issues on average in the profiled
    step (bench.py's issued_flops_per_launch; older lines: flops_per_launch)."""
    return float(roof.get("issued_flops_per_launch", roof.get("flops_per_launch")))


def gemm_source_hash() -> str:
    with open(os.path.join(HERE, "csrc", "gemm.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_rows(path: str, name_part: str):
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if name_part in r["Kernel_Name"]:
                rows.append((int(r["Dispatch_Id"]), float(r["Counter_Value"]), r["Kernel_Name"]))
    rows.sort()
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
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

    cf = [v for _, v, _ in counter_rows(a.copy_fetch, "copyBuffer")]
    cw = [v for _, v, _ in counter_rows(a.copy_write, "copyBuffer")]
    f_scale = a.copy_bytes / (1024.0 * sum(cf) / len(cf))
    w_scale = a.copy_bytes / (1024.0 * sum(cw) / len(cw))

    fr = counter_rows(a.fetch, "zgemm_kernel<0")[-n:]
    wr = counter_rows(a.write, "zgemm_kernel<0")[-n:]
    if len(fr) != n or len(wr) != n:
        raise SystemExit(f"expected {n} GEMM dispatches, found {len(fr)} / {len(wr)}")
    read_b = 1024.0 * sum(v for _, v, _ in fr) / n * f_scale
    write_b = 1024.0 * sum(v for _, v, _ in wr) / n * w_scale
    per_launch = read_b + write_b
    out = {
        "kernel": "zgemm_kernel<0, ...> (FP64 complex GEMM, all tile shapes)",
        "launches": n,
        "hbm_read_bytes_per_launch": read_b,
        "hbm_write_bytes_per_launch": write_b,
        "traffic_bytes_per_launch": per_launch,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "flops_per_launch": launch_flops(roof),
        "flop_per_hbm_byte": launch_flops(roof) / per_launch,
        "gemm_source_sha256": gemm_source_hash(),
    }
    with open(a.out + ".json", "w") as f:
        json.dump(out, f, indent=1)
    md = [
        "# HBM traffic of the FP64 complex GEMM, bulk chain L=64, d=5, chi=1024",
        "",
        "Commands (repository root, one MI355X; `cd /tmp && export TMPDIR=/tmp && cd /root/repo` first):",
        "",
        "```",
        "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex zgemm_kernel --output-format csv -d <dir>/pmc "
        "-o bench_fetch -- python -u bench.py --workers 1 --steps 1 --warmup 0 --no-cpu-baseline --serve 0 --no-u1-sample --no-square-gemm --no-precision-leg --no-fused-sample",
        "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex zgemm_kernel --output-format csv -d <dir>/pmc "
        "-o bench_write -- python -u bench.py --workers 1 --steps 1 --warmup 0 --no-cpu-baseline --serve 0 --no-u1-sample --no-square-gemm --no-precision-leg --no-fused-sample",
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/pmc -o copy_fetch -- python -u bench.py "
        "--copy-calibration 1024",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/pmc -o copy_write -- python -u bench.py "
        "--copy-calibration 1024",
        "python paper_2401_05301_amd/traffic.py --bench-json <bench line of the FETCH run> "
        "--fetch <dir>/pmc/bench_fetch_counter_collection.csv --write <dir>/pmc/bench_write_counter_collection.csv "
        "--copy-fetch <dir>/pmc/copy_fetch_counter_collection.csv --copy-write <dir>/pmc/copy_write_counter_collection.csv "
        "--copy-bytes 1073741824 --out profiles/zgemm_traffic_bulk_L64_chi1024",
        "```",
        "",
        f"- Copy calibration (1 GiB device-to-device copy): FETCH_SIZE reads {sum(cf) / len(cf):.0f} KiB, "
        f"WRITE_SIZE {sum(cw) / len(cw):.0f} KiB per dispatch; scale factors {f_scale:.4f} (fetch) and "
        f"{w_scale:.4f} (write).",
        f"- GEMM launches of the timed step: {n}.",
        f"- Per launch: {read_b / 1e6:.1f} MB read, {write_b / 1e6:.1f} MB written from/to HBM; "
        f"{launch_flops(roof) / 1e9:.2f} GFLOP algorithmic; {out['flop_per_hbm_byte']:.0f} flop per HBM byte "
        "(the FP64 MFMA ridge is 78.6e12 / 8e12 = 9.8).",
        f"- gemm.hip sha256 {out['gemm_source_sha256'][:16]}...: bench.py reports this traffic only while the "
        "kernel source is unchanged.",
        "",
    ]
    with open(a.out + ".md", "w") as f:
        f.write("\n".join(md))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
