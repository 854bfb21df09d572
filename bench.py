"""Benchmark: TT-SVD effective GB/s against the HBM roofline on one MI355X.

A step is one full TT-SVD (Algorithm 2 of arXiv 2102.00104: for every TT step
the Q-less TSQR, the small SVD with truncation and the fused TSMM + reshape)
of a 2^28-element FP64 tensor (2 GiB) that is already resident in HBM:
i.i.d. U[0, 1) entries (seed 0), no tolerance, r_max = 32, viewed as
d = 28, n_i = 2 (the headline shape) and d = 7, n_i = 16 (reported beside it).

value = algorithmic bytes / time per step, where the algorithmic bytes are the
paper's data-volume model (each step reads its work matrix twice and writes the
reduced one, Sec. 4.2).  The roofline object reports the dominant kernel's
achieved rate from HIP events recorded on the decomposition's stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector / matrix, published


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def workload(name):
    if name == "d28n2":
        return [2] * 28
    if name == "d7n16":
        return [16] * 7
    raise SystemExit("unknown workload " + name)


def time_decompose(tt, X, dims, r_max, tol, steps, warmup):
    import torch
    for _ in range(warmup):
        tt.ttsvd_decompose(X, dims, r_max, tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(steps):
        res = tt.ttsvd_decompose(X, dims, r_max, tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, res


def kernel_profile(tt, X, dims, r_max, tol, steps):
    """Per-kernel event timings over `steps` decompositions."""
    import torch
    tt.ttsvd_profile_reset()
    tt.ttsvd_profile_enable(True)
    try:
        for _ in range(steps):
            tt.ttsvd_decompose(X, dims, r_max, tol)
        torch.cuda.synchronize()
        stats = tt.ttsvd_profile_read()
    finally:
        tt.ttsvd_profile_enable(False)
        tt.ttsvd_profile_reset()
    return stats


def roofline_of(stats):
    dom = max(stats, key=lambda s: s["total_ms"])
    secs = dom["total_ms"] / 1e3
    intensity = dom["flops"] / dom["bytes"] if dom["bytes"] else float("inf")
    balance = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity < balance:
        ach = dom["bytes"] / secs / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4)}
    else:
        ach = dom["flops"] / secs / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4)}
    roof.update({"kernel": dom["name"], "launches": dom["launches"],
                 "avg_launch_us": round(dom["total_ms"] * 1e3 / dom["launches"], 2),
                 "traffic": None})
    return roof


def precision_forms(tt, X64, dims, r_max, steps, warmup, f64_sec, f64_res):
    """FP32 / BF16 storage forms of the same workload: speed at full size and
    accuracy (singular values against the FP64 run; reconstruction of a 2^20
    exact TT + 1e-4 noise tensor against the FP64 oracle)."""
    import numpy as np
    import torch

    import oracle
    from paper_2102_00104_amd import model, synth
    out = {}
    dsmall = [2] * 20
    Xs = synth.exact_tt(dsmall, 16, seed=61, noise=1e-4, noise_seed=62, unit_variance=True,
                        relative_noise=True)
    o = oracle.ttsvd(Xs, dsmall, r_max, 0.0)
    e_or = oracle.rel_error(Xs, oracle.tt_full(o.cores))
    for name, dt, eb in (("f32", torch.float32, 4), ("bf16", torch.bfloat16, 2)):
        Xl = X64.to(dt)
        sec, res = time_decompose(tt, Xl, dims, r_max, 0.0, steps, warmup)
        dev = 0.0
        for j in range(1, len(dims)):
            a, b = np.asarray(res.sigma[j]), np.asarray(f64_res.sigma[j])
            r = f64_res.ranks[j]
            dev = max(dev, float(np.max(np.abs(a[:r] - b[:r])) / b[0]))
        g = tt.ttsvd_decompose(torch.from_numpy(Xs).to(X64.device).to(dt), dsmall, r_max, 0.0)
        cores = [tt.core_array(c, (g.ranks[j], dsmall[j], g.ranks[j + 1]))
                 for j, c in enumerate(g.cores)]
        e = oracle.rel_error(Xs, oracle.tt_full(cores))
        ab = model.algorithmic_bytes(dims, f64_res.ranks, eb)
        out[name] = {"value": round(ab / sec / 1e9, 2), "unit": "GB/s",
                     "ms_per_step": round(sec * 1e3, 3),
                     "speedup_vs_f64": round(f64_sec / sec, 3),
                     "max_kept_sigma_dev_vs_f64_rel_sigma1": dev,
                     "exact_tt_2e20_rel_error": e, "exact_tt_2e20_rel_error_fp64_oracle": e_or}
        log("%s: %.3f ms/step (%.2fx FP64), sigma dev %.2e, rel. error %.3e (oracle %.3e)" % (
            name, sec * 1e3, f64_sec / sec, dev, e, e_or))
        del Xl
    return out


def cpu_baseline(d_sample, r_max):
    """The CPU FP64 oracle on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    from paper_2102_00104_amd import model
    dims = [2] * d_sample
    X = np.random.default_rng(0).random(2 ** d_sample)
    t0 = time.perf_counter()
    o = oracle.ttsvd(X, dims, r_max, 0.0)
    dt = time.perf_counter() - t0
    b = model.algorithmic_bytes(dims, o.ranks, 8)
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    return {"value": round(b / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "2^%d-element U[0,1) FP64 tensor, d=%d, n_i=2, r_max=%d, no tol "
                      "(1/%d of the workload); %.2f s" % (d_sample, d_sample, r_max,
                                                          2 ** (28 - d_sample), dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--r-max", type=int, default=32)
    ap.add_argument("--workloads", default="d28n2,d7n16")
    ap.add_argument("--cpu-sample-d", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU path (row slabs of the "
              "unfoldings with an exchange of the triangular factors) is not built; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2102_00104_amd as tt
    from paper_2102_00104_amd import model

    tt.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    log("generating 2^28 U[0,1) values (seed 0)")
    X = torch.from_numpy(np.random.default_rng(0).random(2 ** 28)).to(dev)
    torch.cuda.synchronize()

    results = []
    for wname in args.workloads.split(","):
        dims = workload(wname)
        ranks = model.no_tol_ranks(dims, args.r_max)
        abytes = model.algorithmic_bytes(dims, ranks, 8)
        aflops = model.flops(dims, ranks)
        log("%s: %d warmup + %d timed steps" % (wname, args.warmup, args.steps))
        sec, res = time_decompose(tt, X, dims, args.r_max, 0.0, args.steps, args.warmup)
        assert res.ranks == ranks, (res.ranks, ranks)
        log("%s: %.3f ms/step, %.1f GB/s" % (wname, sec * 1e3, abytes / sec / 1e9))
        stats = kernel_profile(tt, X, dims, args.r_max, 0.0, max(1, min(args.steps, 3)))
        for s in sorted(stats, key=lambda s: -s["total_ms"]):
            log("  %-40s n=%4d  %9.3f ms  %8.1f GB/s  %6.2f TF/s" % (
                s["name"], s["launches"], s["total_ms"],
                s["bytes"] / (s["total_ms"] / 1e3) / 1e9 if s["total_ms"] else 0,
                s["flops"] / (s["total_ms"] / 1e3) / 1e12 if s["total_ms"] else 0))
        results.append(dict(workload=wname, dims=dims, ranks=ranks, ms_per_step=sec * 1e3,
                            value=abytes / sec / 1e9, bytes=abytes, flops=aflops,
                            roofline=roofline_of(stats), kernels=stats, sec=sec, res=res))

    head = results[0]
    line = {
        "metric": "TT-SVD effective GB/s vs 2-read HBM roofline",
        "value": round(head["value"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain FP64 TT-SVD of 2^28 i.i.d. U[0,1) values (2 GiB), "
                               "d=%d, n_i=%d, r_max=%d, no tol" % (len(head["dims"]), head["dims"][0],
                                                                  args.r_max),
                   "algorithmic_bytes": head["bytes"], "flops": head["flops"],
                   "hbm_roofline_frac": round(head["value"] / HBM_PEAK_GBS, 4)},
        "roofline": head["roofline"],
        "others": [{"workload": r["workload"], "value": round(r["value"], 2), "unit": "GB/s",
                    "ms_per_step": round(r["ms_per_step"], 3),
                    "hbm_roofline_frac": round(r["value"] / HBM_PEAK_GBS, 4),
                    "roofline": r["roofline"]} for r in results[1:]],
    }
    if not args.no_precision:
        line["precision_forms"] = precision_forms(tt, X, head["dims"], args.r_max, args.steps,
                                                  args.warmup, head["sec"], head["res"])
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a 2^%d sample" % args.cpu_sample_d)
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample_d, args.r_max)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
