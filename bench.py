#!/usr/bin/env python
"""Three-site TEBD throughput on one MI355X: gate-updates/s at chi = 1024, d = 5.

One timed "step" is one second-order Trotter step of the whole chain (five
commuting layers, 104 three-site gate updates at L = 64) followed by the local
measurement of n_i, <b+_i b_{i+1}> and <b+_i b_{i+2}>, on a synthetic state of
the bulk chi = 1024 workload (L = 64, d = 5, U = 2, J_NNN = 0.1, K = 0,
dt = 0.01, w_max = 1e-12).  The state, the gates and all workspace are
resident in HBM before the timed region starts.  Prints one JSON line on
stdout; progress on stderr.

A step takes tens of seconds at chi = 1024, so the run is bounded by wall
clock: at most one warmup step, then timed steps while they fit in
--budget seconds (at least one); the JSON reports the steps actually run and
the ones requested.  Kernel timing (HIP events per launch) is switched on
only for one extra step after the timed region, which supplies the roofline
and the per-kernel breakdown.

    python bench.py [--steps K] [--warmup W] [--budget S] [--svd gram|jacobi] [--prec fp64|fp32|split]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "3-site TEBD gate-updates/s at χ=1024,d=5 (MFMA roofline %); quench p50/p99"
PEAK_FP64 = 78.6      # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32 = 157.3     # TFLOP/s, MI355X dense FP32 matrix


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gate_updates_per_step(L: int) -> int:
    layers = [(0, 0.5), (1, 0.5), (2, 1.0), (1, 0.5), (0, 0.5)]
    return sum(len(range(g, L - 2, 3)) for g, _ in layers)


def unit_flops(chi: int = 1024, d: int = 5):
    """Algorithmic flops of one bulk gate update (all four bonds at chi), by
    term: theta assembly, gate, and per SVD the Gram product, the
    tridiagonal reduction, the back-transformation of the kept k = chi
    eigenvectors and the projection onto them (complex 8 flop per
    multiply-add, Hermitian products 4 m^2 n).  The GEMM-shaped terms are
    what the GEMM kernel's roofline is credited with."""
    m1, n1 = chi * d, d * d * chi
    m2 = n2 = chi * d
    k = chi
    t = {
        "theta": 8.0 * chi ** 3 * (d ** 2 + d ** 3),
        "gate": 8.0 * d ** 6 * chi ** 2,
        "svd1_gram": 4.0 * m1 * m1 * n1, "svd1_tri": 16.0 / 3.0 * m1 ** 3,
        "svd1_back": 8.0 * m1 * m1 * k, "svd1_project": 8.0 * k * m1 * n1,
        "svd2_gram": 4.0 * m2 * m2 * n2, "svd2_tri": 16.0 / 3.0 * m2 ** 3,
        "svd2_back": 8.0 * m2 * m2 * k, "svd2_project": 8.0 * k * m2 * n2,
    }
    total = sum(t.values())
    gemm = total - t["svd1_tri"] - t["svd2_tri"]
    return total, gemm, t


def cpu_baseline(chi: int):
    """Time the FP64 CPU oracle on one bulk gate update at bond dimension chi
    and scale its rate by (chi / 1024)^3 to the chi = 1024 unit."""
    from oracle import model as mdl
    from oracle import tebd as otebd
    from workloads import Model, Trunc, random_mps
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads") or 0) for i in threadpool_info()) or None
    except Exception:
        threads = None
    L = 14
    B, lam = random_mps(L, 5, chi, seed=0, tau=110.0)
    mps = otebd.MPS(B, lam)
    m = Model(L=L, d=5, U=2.0, J=1.0, Jnnn=0.1, K=0.0)
    G = mdl.gate(m, 5, 0.005)
    t0 = time.perf_counter()
    otebd.apply_gate(mps, 5, G, Trunc(chi_max=chi))
    dt = time.perf_counter() - t0
    rate = (1.0 / dt) * (chi / 1024.0) ** 3
    return {"value": rate, "unit": "gate-updates/s", "cores": threads or os.cpu_count(), "kind": "oracle",
            "sample": (f"one bulk gate update (bonds {chi},{chi},{chi},{chi}, d=5) of the same Hamiltonian on a "
                       f"random right-orthonormal L=14 chain took {dt:.1f} s; its rate is scaled by "
                       f"({chi}/1024)^3 to the chi=1024 unit (the oracle's cost is cubic in chi), since one "
                       f"chi=1024 gate update takes minutes in the oracle")}


def measured_gemm_peak(pt, torch, n: int = 4096):
    """Square complex GEMM rates on this device, n x n x n, 8 n^3 flops each:
    this library's kernel and torch's matmul (rocBLAS), in complex128 (FP64
    matrix cores) and complex64 (FP32 matrix cores)."""
    fl = 8.0 * n ** 3

    def torch_rate(dtype):
        a = torch.randn(n, n, dtype=dtype, device="cuda")
        b = torch.randn(n, n, dtype=dtype, device="cuda")
        torch.matmul(a, b)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            torch.matmul(a, b)
        e1.record()
        torch.cuda.synchronize()
        return fl / (e0.elapsed_time(e1) / 5 / 1e3) / 1e12

    return {"n": n,
            "zgemm_kernel_TFLOPs": fl / (pt.tebd_diag_zgemm_time(n, n, n, pt.FP64, 5) / 1e3) / 1e12,
            "rocblas_zgemm_TFLOPs": torch_rate(torch.complex128),
            "zgemm_kernel_fp32_TFLOPs": fl / (pt.tebd_diag_zgemm_time(n, n, n, pt.FP32, 5) / 1e3) / 1e12,
            "rocblas_cgemm_TFLOPs": torch_rate(torch.complex64)}


def quench_run(pt, torch, args):
    """The growing-chi quench: CDW start of the L = 64, d = 5 chain (U = 3,
    J_NNN = 0.1, K = 0.002 centred at 32.5), truncation 1e-10, chi <= 512,
    dt = 0.01; every step is timed and measured."""
    import numpy as np
    from workloads import CONFIGS
    cfg = CONFIGS["batched_L64_chi512"]
    m, tr, dt = cfg["model"], cfg["trunc"], cfg["dt"]
    svd = {"gram": pt.SVD_GRAM_EIG, "jacobi": pt.SVD_JACOBI}[args.svd]
    eps = max(tr.eps, pt.GRAM_EPS_MIN) if svd == pt.SVD_GRAM_EIG else tr.eps
    stream = torch.cuda.Stream()
    opts = pt.make_opts(tr.chi_max, tr.w_max, eps, svd=svd, stream=stream.cuda_stream, workers=args.workers,
                        u1=args.u1)
    g = pt.MPS.cdw(pt.make_model(m.L, m.d, m.U, m.J, m.Jnnn, m.K, m.centre()), opts)
    g.prepare(dt)
    per_step = gate_updates_per_step(m.L)
    times, chis = [], []
    t_all = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        g.step(dt)
        n, C, D = g.measure()
        times.append(time.perf_counter() - t0)
        chis.append(max(g.bond_dims()))
        if (k + 1) % 10 == 0 or k + 1 == args.steps:
            log(f"quench step {k + 1}/{args.steps}: max bond {chis[-1]}, {times[-1]:.3f} s")
    wall = time.perf_counter() - t_all
    out = {
        "metric": "gate-updates/s of the growing-chi quench (CDW start)",
        "value": per_step * args.steps / wall, "unit": "gate-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 0, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched_L64_chi512", "L": m.L, "d": m.d, "U": m.U, "Jnnn": m.Jnnn, "K": m.K,
                   "jc": m.centre(), "chi_max": tr.chi_max, "w_max": tr.w_max, "eps": eps, "dt": dt,
                   "svd": args.svd, "u1": bool(args.u1)},
        "max_bond_per_step": chis,
        "seconds_per_step": [round(t, 4) for t in times],
        "discarded_weight": g.discarded_weight(),
        "trunc_rule_counts": g.trunc_stats(),
        "n_total": float(np.sum(n)),
    }
    g.close()
    print(json.dumps(out), flush=True)


def u1_sample(pt, torch, args, eps):
    """One timed Strang step of the same chain (L, d = 5, chi) with U(1)
    sectors: a random state of L/2 bosons (sector width sigma), canonicalised
    and evolved by one untimed step, tebd_opts.u1 = 1, Gram route."""
    from workloads import CONFIGS, random_mps_u1
    cfg = CONFIGS["bulk_L64_chi1024"]
    mdl, dt = cfg["model"], cfg["dt"]
    L, d, chi = args.L, mdl.d, args.chi
    B, lam, _ = random_mps_u1(L, d, chi, L // 2, seed=args.seed, tau=args.tau, sigma=args.sigma, bias=args.bias)
    stream = torch.cuda.Stream()
    opts = pt.make_opts(chi, 1e-12, eps, svd=pt.SVD_GRAM_EIG, stream=stream.cuda_stream, workers=args.workers,
                        u1=True)
    g = pt.MPS.from_tensors(pt.make_model(L, d, mdl.U, mdl.J, mdl.Jnnn, mdl.K, mdl.centre()), opts, B, lam)
    del B, lam
    g.canonicalize()
    g.prepare(dt)
    g.step(dt)      # untimed: the first step after a canonicalisation, and the tile tuner's first look at new shapes
    g.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    g.step(dt)
    g.measure()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out = {"value": gate_updates_per_step(L) / (ms / 1e3), "unit": "gate-updates/s", "ms_per_step": ms,
           "input": f"random right-orthonormal MPS of {L // 2} bosons (seed {args.seed}, sector width sigma "
                    f"{args.sigma:g}, right-index weight exp(-b/{args.bias:g})), canonicalised, one untimed step",
           "max_bond": max(g.bond_dims())}
    g.close()
    return out


def fused_sample(pt, workers: int = 0, chi: int = 32, steps: int = 4):
    """Fused layers against concurrent workers on the same small-chi state:
    the L = 64, d = 5 chain from a random right-orthonormal MPS at bond
    dimension chi (cap chi, so every gate truncates), Jacobi route, one
    untimed step, then `steps` timed Strang steps each way.  `workers` is
    tebd_opts.workers of the unfused run (0: the library's default); the
    fused run issues everything from one host thread."""
    import numpy as np
    from workloads import Model, random_mps
    L, d, dt = 64, 5, 0.01
    m = Model(L=L, d=d, U=3.0, J=1.0, Jnnn=0.1, K=0.002)
    B, lam = random_mps(L, d, chi, seed=2, tau=8.0)
    res, obs = {}, {}
    for name, fuse in (("workers", False), ("fused", True)):
        g = pt.MPS.from_tensors(pt.make_model(L, d, m.U, m.J, m.Jnnn, m.K, m.centre()),
                                pt.make_opts(chi, 1e-10, 1e-10, fuse=fuse, workers=0 if fuse else workers), B, lam)
        g.prepare(dt)
        g.step(dt)
        g.sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.step(dt)
        g.sync()
        sec = (time.perf_counter() - t0) / steps
        obs[name] = g.measure()
        res[name] = {"ms_per_step": 1e3 * sec, "gate_updates_per_s": gate_updates_per_step(L) / sec}
        g.close()
    res["speedup"] = res["workers"]["ms_per_step"] / res["fused"]["ms_per_step"]
    res["bit_identical"] = all(np.array_equal(a, b) for a, b in zip(obs["workers"], obs["fused"]))
    res["input"] = (f"L={L}, d={d}, random right-orthonormal MPS at chi={chi} (seed 2), cap {chi}, Jacobi route, "
                    f"w_max = eps = 1e-10, dt={dt}; "
                    + (f"{workers} worker(s)" if workers > 0 else "the default six workers")
                    + " against one fused batch per layer")
    return res


def precision_batching(pt, torch, args):
    """The same chi = 1024 state stepped four ways with one library: FP64 with
    one gate worker (the plain per-gate form), FP64 with six concurrent
    workers (the batched form), and the batched form with the theta/gate
    products in FP32 and in split FP32.  Chain L = 16, d = 5 (its central
    bonds at chi = 1024), one Strang step each from the same state (a
    canonicalised random state after one FP64 step).  Rates in
    gate-updates/s; for each FP32 form the largest differences of n, C and
    D from the FP64 result on the same state (the per-observable errors
    against the oracle at chi = 1024 are what the full-size parity test
    checks)."""
    import numpy as np
    from workloads import CONFIGS, random_mps_device
    cfg = CONFIGS["bulk_L64_chi1024"]
    mdl, dt = cfg["model"], cfg["dt"]
    L, d, chi = 16, mdl.d, args.chi
    model = pt.make_model(L, d, mdl.U, mdl.J, mdl.Jnnn, mdl.K, (L + 1) / 2.0)
    B, lam = random_mps_device(L, d, chi, seed=args.seed, tau=args.tau, bias=args.bias)
    stream = torch.cuda.Stream()

    def opts(prec, workers):
        return pt.make_opts(chi, 1e-12, pt.GRAM_EPS_MIN, prec=prec, svd=pt.SVD_GRAM_EIG, stream=stream.cuda_stream,
                            workers=workers)

    g = pt.MPS.from_tensors(model, opts(pt.FP64, 6), B, lam)
    del B, lam
    g.canonicalize()
    g.prepare(dt)
    g.step(dt)      # the first gates after a canonicalisation converge slowest: start from a step later
    g.sync()
    Bc = [g.site(i) for i in range(L)]
    lc = [g.lam(b) for b in range(L + 1)]
    g.close()
    per_step = gate_updates_per_step(L)
    res, obs = {}, {}
    for name, prec, workers in [("fp64_plain_1_worker", pt.FP64, 1), ("fp64_batched_6_workers", pt.FP64, 6),
                                ("fp32_batched_6_workers", pt.FP32, 6), ("split_batched_6_workers", pt.FP32_SPLIT, 6)]:
        h = pt.MPS.from_tensors(model, opts(prec, workers), Bc, lc)
        h.prepare(dt)
        h.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        h.step(dt)
        n, C, D = h.measure()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        obs[name] = (np.asarray(n), np.asarray(C), np.asarray(D))
        res[name] = {"gate_updates_per_s": per_step / (ms / 1e3), "ms_per_step": ms,
                     "discarded_weight": h.discarded_weight()}
        h.close()
        log(f"precision/batching leg: {name} {res[name]['gate_updates_per_s']:.2f} gate-updates/s")
    ref = obs["fp64_batched_6_workers"]
    for name in res:
        if name == "fp64_batched_6_workers":
            continue
        n, C, D = obs[name]
        res[name]["max_abs_diff_vs_fp64_batched"] = {
            "n": float(np.abs(n - ref[0]).max()), "C": float(np.abs(C - ref[1]).max()),
            "D": float(np.abs(D - ref[2]).max())}
    plain = res["fp64_plain_1_worker"]["gate_updates_per_s"]
    best = max(res[k]["gate_updates_per_s"] for k in res if k != "fp64_plain_1_worker")
    return {"workload": f"L={L}, d={d}, chi={chi}, one Strang step ({per_step} gate updates) from the same "
                        f"state: a canonicalised random state (seed {args.seed}) after one FP64 step",
            "forms": res, "batched_over_plain": best / plain,
            "batched_mixed_precision_beats_plain_fp64": bool(
                max(res["fp32_batched_6_workers"]["gate_updates_per_s"],
                    res["split_batched_6_workers"]["gate_updates_per_s"]) > plain)}


def measured_traffic():
    """HBM bytes per launch of the FP64 GEMM from the committed rocprofv3
    counter summary, or None when it is missing or the kernel source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "zgemm_traffic_bulk_L64_chi1024.json")
    if not os.path.exists(path):
        return None
    from paper_2401_05301_amd.traffic import gemm_source_hash
    with open(path) as f:
        t = json.load(f)
    if t.get("gemm_source_sha256") != gemm_source_hash():
        return None
    return t["traffic_bytes_per_launch"]


def serving_sample(pt, n: int, scale: float, eps: float, svd: int = None, batched: bool = False):
    """Quench requests of the serving workload (Poisson arrivals, L in
    {16..64}, U in [2, 10], K in [0, 0.01], J_NNN = 0.1, dt = 0.01), with the
    small bond caps {16, 32, 64} and each horizon scaled by `scale`, served
    concurrently by the library; p50/p99 time from arrival to horizon.
    `batched` serves them by continuous batching (Jacobi route only)."""
    if svd is None:
        svd = pt.SVD_GRAM_EIG
    import numpy as np
    from workloads import serving_requests
    rate = 2.0
    reqs = []
    for r in serving_requests(n=n, seed=5, rate=rate, small=True):
        m = r["model"]
        steps = max(1, int(round(r["horizon"] / r["dt"] * scale)))
        reqs.append(dict(model=pt.make_model(m.L, m.d, m.U, m.J, m.Jnnn, m.K, m.centre()), chi_max=r["chi_max"],
                         dt=r["dt"], steps=steps, arrival=r["arrival"]))
    t0 = time.perf_counter()
    if batched:
        res = pt.tebd_serve(reqs, max_active=8, svd=svd, eps=eps, batched=True, workers_per_request=0)
    else:
        res = pt.tebd_serve(reqs, max_active=8, svd=svd, eps=eps)
    wall = time.perf_counter() - t0
    if any(x["status"] != 0 for x in res):
        raise RuntimeError("a served request failed: " + str([x["status"] for x in res]))
    lat = np.array([x["finished"] - x["arrival"] for x in res])
    span = max(x["finished"] for x in res) - min(x["arrival"] for x in res)
    gu = sum(x["gate_updates"] for x in res)
    return {"requests": n, "arrival_rate_per_s": rate, "max_active": 8, "chi_max_set": [16, 32, 64],
            "horizon_scale": scale, "steps_total": sum(r["steps"] for r in reqs),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "gate_updates_per_s": gu / span, "wall_s": wall,
            "note": "time-to-horizon = finish - arrival; " + ("Gram" if svd != pt.SVD_JACOBI else "Jacobi") +
                    (" route; continuous batching: every admitted request stepped together, one fused batch per "
                     "layer" if batched else " route; each request on its own handle, stream and thread")}


def main():
    T_START = time.perf_counter()
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed steps requested (capped by --budget)")
    ap.add_argument("--warmup", type=int, default=1, help="warmup steps requested (at most one is run)")
    ap.add_argument("--budget", type=float, default=100.0,
                    help="seconds of timed steps: no further step starts once the next would end past it")
    ap.add_argument("--aux-budget", type=float, default=420.0,
                    help="auxiliary legs (profiled step, U(1), serving, square GEMM, CPU oracle) start only "
                         "while the whole run is below this many seconds")
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--svd", choices=["gram", "jacobi"], default="gram")
    ap.add_argument("--prec", choices=["fp64", "fp32", "split"], default="fp64")
    ap.add_argument("--tau", type=float, default=110.0, help="decay length of the imposed Lambda profile")
    ap.add_argument("--bias", type=float, default=150.0,
                    help="decay length of the right-index weighting that shapes the canonical Schmidt spectra")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-input", action="store_true",
                    help="draw the input with numpy on the host (slow at chi=1024) instead of torch on the GPU")
    ap.add_argument("--no-canonicalize", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-chi", type=int, default=512)
    ap.add_argument("--workers", type=int, default=0, help="concurrent gate workers per layer (0: library default)")
    ap.add_argument("--serve", type=int, default=16, help="requests in the serving sample (0: skip it)")
    ap.add_argument("--no-profile-step", action="store_true", help="skip the profiled step (no roofline)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (the reference for the HBM counters) and exit")
    ap.add_argument("--quench", action="store_true",
                    help="time the growing-chi CDW quench (L=64, chi<=512, truncation 1e-10) instead")
    ap.add_argument("--u1", action="store_true",
                    help="U(1) block-sparse SVDs on a random state of L/2 bosons with definite numbers per bond index")
    ap.add_argument("--no-square-gemm", action="store_true",
                    help="skip the square-GEMM reference (it launches this library's GEMM after the timed step)")
    ap.add_argument("--no-precision-leg", action="store_true",
                    help="skip the plain/batched FP64 vs batched FP32 comparison on an L = 16 chain")
    ap.add_argument("--no-fused-sample", action="store_true",
                    help="skip the fused-layer sample (chi = 32, fused against concurrent workers)")
    ap.add_argument("--no-u1-sample", action="store_true",
                    help="skip the U(1) step reported under u1_sample in the default run")
    ap.add_argument("--sigma", type=float, default=2.0,
                    help="--u1: width of the particle-number distribution over each bond's indices")
    ap.add_argument("--serve-scale", type=float, default=0.1,
                    help="fraction of each request's horizon served in the sample")
    args = ap.parse_args()

    if args.copy_calibration > 0:
        import torch
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": nbytes, "dispatches": 5}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library evolves one chain per GPU and has no multi-GPU path "
              "(see the sharding design); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2401_05301_amd as pt
    from workloads import CONFIGS, random_mps, random_mps_device, random_mps_u1

    torch.cuda.set_device(0)
    if args.quench:
        quench_run(pt, torch, args)
        return
    stream = torch.cuda.Stream()
    cfg = CONFIGS["bulk_L64_chi1024"]
    mdl = cfg["model"]
    dt = cfg["dt"]
    L, d, chi = args.L, mdl.d, args.chi
    prec = {"fp64": pt.FP64, "fp32": pt.FP32, "split": pt.FP32_SPLIT}[args.prec]
    svd = {"gram": pt.SVD_GRAM_EIG, "jacobi": pt.SVD_JACOBI}[args.svd]
    w_max = cfg["trunc"].w_max
    # The Gram route refuses eps below TEBD_GRAM_EPS_MIN; at chi = 1024 the
    # bond cap sets every cut of this workload (trunc_rule_counts shows it),
    # so the result is the one eps = 1e-12 would give.
    eps = pt.GRAM_EPS_MIN if svd == pt.SVD_GRAM_EIG else cfg["trunc"].eps

    t0 = time.perf_counter()
    if args.u1:
        B, lam, _ = random_mps_u1(L, d, chi, L // 2, seed=args.seed, tau=args.tau, sigma=args.sigma, bias=args.bias)
        recipe = "random_mps_u1 (numpy)"
    elif args.cpu_input:
        B, lam = random_mps(L, d, chi, seed=args.seed, tau=args.tau, bias=args.bias)
        recipe = "random_mps (numpy)"
    else:
        B, lam = random_mps_device(L, d, chi, seed=args.seed, tau=args.tau, bias=args.bias)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        recipe = "random_mps_device (torch on the GPU)"
    log(f"synthetic input L={L} d={d} chi={chi} u1={args.u1} ({recipe}) generated in {time.perf_counter() - t0:.1f} s")
    model = pt.make_model(L, d, mdl.U, mdl.J, mdl.Jnnn, mdl.K, mdl.centre())
    opts = pt.make_opts(chi, w_max, eps, prec=prec, svd=svd, stream=stream.cuda_stream, workers=args.workers,
                        u1=args.u1)
    keep = pt.torch_allocator(opts, stream=stream)
    g = pt.MPS.from_tensors(model, opts, B, lam)
    g._keep = keep
    del B, lam
    if not args.no_canonicalize:
        t0 = time.perf_counter()
        g.canonicalize()
        g.sync()
        log(f"canonicalised by an identity sweep in {time.perf_counter() - t0:.1f} s, max bond {max(g.bond_dims())}")
    g.prepare(dt)
    nsteps_gu = gate_updates_per_step(L)

    warm_run, t_warm = 0, None
    for w in range(min(args.warmup, 1)):
        # the warmup step runs its five layers one call at a time (the same
        # work as tebd_step), reporting each
        t0 = time.perf_counter()
        for grp, tau in [(0, 0.5 * dt), (1, 0.5 * dt), (2, dt), (1, 0.5 * dt), (0, 0.5 * dt)]:
            tl = time.perf_counter()
            g.layer(grp, tau)
            g.sync()
            log(f"warmup layer {grp} ({tau:g}) done in {time.perf_counter() - tl:.1f} s")
        g.measure()
        t_warm = time.perf_counter() - t0
        warm_run += 1
        log(f"warmup step {w + 1} done in {t_warm:.1f} s")

    w0 = g.discarded_weight()
    sweeps0 = pt.mps_sweep_stats(g.h)[1]
    rules0 = g.trunc_stats()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    steps_run = 0
    est = t_warm
    step_s = []
    for k in range(max(1, args.steps)):
        if steps_run >= 1 and est is not None and (time.perf_counter() - t0) + est > args.budget:
            break
        ts = time.perf_counter()
        g.step(dt)
        n, C, D = g.measure()
        steps_run += 1
        est = time.perf_counter() - ts
        step_s.append(est)
        log(f"timed step {k + 1}/{args.steps} done ({time.perf_counter() - t0:.1f} s)")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = e0.elapsed_time(e1)
    w1 = g.discarded_weight()
    sweeps1 = pt.mps_sweep_stats(g.h)[1]
    rules1 = g.trunc_stats()
    chis = g.bond_dims()
    lam_min = min(float(np.min(g.lam(b))) / float(np.max(g.lam(b))) for b in range(1, L) if chis[b] > 1)

    secs = dev_ms / 1e3
    value = nsteps_gu * steps_run / secs
    F_GU, F_GEMM, terms = unit_flops(1024, 5)
    peak = PEAK_FP64 if prec == pt.FP64 else PEAK_FP32
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "gate-updates/s",
        "n_gpus": 1,
        "steps": steps_run,
        "warmup": warm_run,
        "requested": {"steps": args.steps, "warmup": args.warmup, "budget_s": args.budget},
        "ms_per_step": dev_ms / steps_run,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == pt.FP64 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "bulk_L64_chi1024" + ("_u1" if args.u1 else ""), "L": L, "d": d, "chi_max": chi,
                   "U": mdl.U, "J": mdl.J, "Jnnn": mdl.Jnnn, "K": mdl.K, "dt": dt, "svd": args.svd,
                   "theta_gate_prec": args.prec, "gate_updates_per_step": nsteps_gu, "w_max": w_max, "eps": eps,
                   "u1": bool(args.u1),
                   "input": (f"{recipe}: random right-orthonormal MPS (seed {args.seed}, right-index weight "
                             f"exp(-b/{args.bias:g})"
                             + (f", {L // 2} bosons, sector width sigma {args.sigma:g}" if args.u1 else "") + "), "
                             + ("canonicalised by an identity sweep" if not args.no_canonicalize else "as generated"))},
        "path_roofline": {"unit_flops": F_GU, "achieved_TFLOPs": F_GU * value / 1e12, "peak": PEAK_FP64,
                          "frac": F_GU * value / 1e12 / PEAK_FP64,
                          # with --u1 the sector SVDs do far less than the dense count F_GU: the
                          # figure is then a dense-equivalent rate, not work done
                          "dense_equivalent": bool(args.u1)},
        "wall_s": wall,
        # host wall time of every timed step (step plus measurement, which reads the
        # observables back): the spread of the timed steps
        "seconds_per_step": [round(t, 3) for t in step_s],
        "discarded_weight_per_step": (w1 - w0) / steps_run,
        "trunc_rule_counts": {k: rules1[k] - rules0[k] for k in rules1},
        "smallest_kept_lambda_ratio": lam_min,
        "jacobi_sweeps_per_gate_update": (sweeps1 - sweeps0) / (nsteps_gu * steps_run),
        "theta_tile_tuner": g.tile_tuner(),
        "max_bond": max(chis),
    }

    def time_left():
        return time.perf_counter() - T_START < args.aux_budget

    # the fused-layer sample runs before the profiled step, so that the profiled
    # step stays the last GEMM work of a run without the later legs
    if not args.no_fused_sample and time_left():
        log("fused layers against concurrent workers at chi = 32")
        out["fused_layers"] = fused_sample(pt, args.workers)
    # one more step with per-launch HIP events: kernel breakdown and roofline
    if not args.no_profile_step and time_left():
        g.profile(True)
        tp = time.perf_counter()
        g.step(dt)
        g.measure()
        g.sync()
        prof = g.profile_read()
        busy = g.profile_busy()
        sites = g.profile_sites()
        g.profile(False)
        log(f"profiled step done in {time.perf_counter() - tp:.1f} s")
        key = "gemm_fp64" if prec == pt.FP64 else "gemm_fp32"
        gemm_ms, gemm_n, gemm_fl = prof["gemm_fp64"]
        gemm_busy = busy["gemm_fp64"]
        # credited: the GEMM-shaped terms of the unit (theta, gate, Gram products,
        # back-transformation, projections) for the step's gate updates; in the
        # FP32 theta/gate path those two terms run on the FP32 GEMM instead
        credited = F_GEMM * nsteps_gu
        if prec != pt.FP64:
            credited -= (terms["theta"] + terms["gate"]) * nsteps_gu
        roof = {"bound": "mfma", "kernel": "zgemm_kernel<FP64>", "achieved": credited / (gemm_ms / 1e3) / 1e12,
                "peak": PEAK_FP64, "unit": "TFLOP/s", "frac": credited / (gemm_ms / 1e3) / 1e12 / PEAK_FP64,
                "traffic": None, "launches": gemm_n, "avg_launch_ms": gemm_ms / max(gemm_n, 1),
                "credited_flops_per_launch": credited / max(gemm_n, 1),
                "issued_flops_per_launch": gemm_fl / max(gemm_n, 1),
                "issued_over_credited": gemm_fl / credited,
                "issued_TFLOPs": gemm_fl / (gemm_ms / 1e3) / 1e12,
                "busy_ms": gemm_busy, "summed_launch_ms": gemm_ms,
                "achieved_over_busy_TFLOPs": credited / (gemm_busy / 1e3) / 1e12,
                "frac_over_busy": credited / (gemm_busy / 1e3) / 1e12 / PEAK_FP64,
                "note": ("achieved = credited GEMM flops of the profiled step (algorithmic unit terms x gate "
                         "updates) / summed HIP-event launch time; gate workers run concurrently, so "
                         "launches overlap: busy_ms is the union of the launch intervals")}
        if prec == pt.FP64 and L == 64 and chi == 1024 and args.svd == "gram" and not args.u1:
            roof["traffic"] = measured_traffic()
        out["roofline"] = roof
        out["kernel_ms"] = {k: v[0] for k, v in prof.items()}
        out["kernel_launches"] = {k: v[1] for k, v in prof.items()}
        out["kernel_busy_ms"] = busy
        out["gemm_sites"] = {k: {"launches": v[0], "ms": v[1], "TFLOP": v[2] / 1e12} for k, v in sites.items()}
        out["dominant_kernel_class"] = max(prof.items(), key=lambda kv: kv[1][0])[0]
        if key != "gemm_fp64":
            out["roofline_fp32_gemm"] = {"achieved": (terms["theta"] + terms["gate"]) * nsteps_gu
                                         / (prof[key][0] / 1e3) / 1e12, "peak": PEAK_FP32}
    g.close()
    if not args.no_square_gemm and time_left():
        out["measured_square_gemm"] = measured_gemm_peak(pt, torch)
    if not args.u1 and not args.no_precision_leg and args.prec == "fp64" and time_left():
        log("precision/batching leg: plain FP64, batched FP64, batched FP32 and split FP32 on one state")
        out["precision_batching"] = precision_batching(pt, torch, args)
    if not args.u1 and not args.no_u1_sample and time_left():
        log("U(1) sample: one step of the same chain with particle-number sectors")
        out["u1_sample"] = u1_sample(pt, torch, args, pt.GRAM_EPS_MIN)
    if args.serve > 0 and time_left():
        log(f"serving sample: {args.serve} requests")
        out["serving"] = serving_sample(pt, args.serve, args.serve_scale, pt.GRAM_EPS_MIN)
    if not args.no_cpu_baseline and time_left():
        log(f"timing the CPU oracle on one chi={args.cpu_chi} gate update")
        out["cpu_baseline"] = cpu_baseline(args.cpu_chi)
    if args.serve > 0 and time_left():
        # the same requests and truncation on the Jacobi route, thread per
        # request against continuous batching
        log("serving sample, Jacobi route: threads, then continuous batching")
        out["serving_batching"] = {
            "threads": serving_sample(pt, args.serve, args.serve_scale, pt.GRAM_EPS_MIN, svd=pt.SVD_JACOBI),
            "batched": serving_sample(pt, args.serve, args.serve_scale, pt.GRAM_EPS_MIN, svd=pt.SVD_JACOBI,
                                      batched=True)}
    out["bench_wall_s"] = time.perf_counter() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
