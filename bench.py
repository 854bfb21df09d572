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


class Decomposer:
    """ttsvd_decompose_ws on one resident tensor with a workspace and a core
    buffer allocated once, so the timed calls make no device allocation; the
    C call is made directly (prebuilt ctypes arguments) and each result's host
    arrays are released right away."""

    def __init__(self, tt, X, dims, r_max, tol):
        import ctypes

        import torch
        self.tt, self.X, self.dims = tt, X, list(dims)
        self.L = tt.lib()
        d = len(dims)
        self.ws = torch.empty(tt.ttsvd_workspace_size(dims, r_max, tt.dtype_code(X)),
                              dtype=torch.uint8, device=X.device)
        self.cores = torch.empty(tt.ttsvd_cores_size(dims, r_max), dtype=torch.float64,
                                 device=X.device)
        self.st = torch.cuda.current_stream().cuda_stream
        self.xs = tt.TensorStruct(X.data_ptr(), tt.dtype_code(X), 0, self.st)
        self.arr = (ctypes.c_int64 * d)(*[int(n) for n in dims])
        self.args = (ctypes.byref(self.xs), self.arr, d, int(r_max), float(tol),
                     self.ws.data_ptr(), self.ws.numel(), self.cores.data_ptr(),
                     self.cores.numel())
        self.out = tt.TTStruct()
        self.ctypes = ctypes

    def once(self):
        rc = self.L.ttsvd_decompose_ws(*self.args, self.ctypes.byref(self.out))
        if rc != 0:
            raise self.tt.TTSVDError(rc, self.L.ttsvd_last_error().decode())
        self.L.ttsvd_tt_free(self.ctypes.byref(self.out))

    def result(self, fetch=False):
        return self.tt.ttsvd_decompose_ws(self.X, self.dims, self.args[3], self.args[4], self.ws,
                                          self.cores, fetch=fetch)


def time_decompose(tt, X, dims, r_max, tol, steps, warmup):
    """Mean seconds per decomposition over `steps` timed calls (after `warmup`
    untimed ones), the per-call median, and the result of one more call."""
    import torch
    dec = Decomposer(tt, X, dims, r_max, tol)
    for _ in range(warmup):
        dec.once()
    torch.cuda.synchronize()
    each = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ta = time.perf_counter()
        dec.once()            # returns after its stream is synchronised
        each.append(time.perf_counter() - ta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    each.sort()
    med = each[len(each) // 2] if len(each) % 2 else 0.5 * (each[len(each) // 2 - 1] + each[len(each) // 2])
    res = dec.result()
    del dec
    return (t1 - t0) / steps, res, med


def kernel_profile(tt, X, dims, r_max, tol, steps):
    """Per-kernel event timings over `steps` decompositions."""
    import torch
    dec = Decomposer(tt, X, dims, r_max, tol)
    tt.ttsvd_profile_reset()
    tt.ttsvd_profile_enable(True)
    try:
        for _ in range(steps):
            dec.once()
        torch.cuda.synchronize()
        stats = tt.ttsvd_profile_read()
    finally:
        tt.ttsvd_profile_enable(False)
        tt.ttsvd_profile_reset()
    return stats


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/traffic_*.json), or None when there is none for this
    kernel and workload or its sources changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("kernel") != kernel or rec.get("workload") != workload:
            continue
        h = hashlib.sha1()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() == rec["source_digest"]:
            return float(rec["traffic_bytes_per_launch"])
    return None


def roofline_of(stats, workload=None):
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
    traffic = measured_traffic(dom["name"], workload)
    roof.update({"kernel": dom["name"], "launches": dom["launches"],
                 "avg_launch_us": round(dom["total_ms"] * 1e3 / dom["launches"], 2),
                 "algorithmic_bytes_per_launch": round(dom["bytes"] / dom["launches"]),
                 "traffic": round(traffic) if traffic is not None else None})
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
        sec, res, _ = time_decompose(tt, Xl, dims, r_max, 0.0, steps, warmup)
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


def thick_bounds(tt, model, X, dims, r_max, steps, warmup, plain_sec, plain_res,
                 m_min=16, f1_min=0.5):
    """Algorithm 3 (thick bounds) on the headline tensor: the k right-most
    modes combined (smallest k with m >= max(m_min, r_max / f1_min); m_min = 16
    and f1_min = 1/2 are the paper's Table 2 setting), timed like the plain path
    and checked against it at full size (same ranks; same singular values at
    and left of the block boundary, where no rank inside the block is cut)."""
    import torch
    k, m = tt.thick_bounds_k(dims, m_min, f1_min, r_max)
    for _ in range(warmup):
        tt.ttsvd_decompose_thick(X, dims, r_max, 0.0, m_min=m_min, f1_min=f1_min)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(steps):
        res = tt.ttsvd_decompose_thick(X, dims, r_max, 0.0, m_min=m_min, f1_min=f1_min)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    d = len(dims)
    dims_w = list(dims[:d - k]) + [m]
    abytes = model.algorithmic_bytes(dims_w, model.no_tol_ranks(dims_w, r_max), 8)
    r = res.ranks[d - k]
    dims_b = [r * dims[d - k]] + list(dims[d - k + 1:])
    abytes += model.algorithmic_bytes(dims_b, model.no_tol_ranks(dims_b, r_max), 8)
    plain_bytes = model.algorithmic_bytes(dims, model.no_tol_ranks(dims, r_max), 8)
    dev = 0.0
    for j in range(1, d - k + 1):
        a, b = res.sigma[j], plain_res.sigma[j]
        dev = max(dev, max(abs(x - y) for x, y in zip(a, b)) / b[0])
    ok = res.ranks == plain_res.ranks and dev <= 1e-10
    log("thick bounds: k=%d m=%d, %.3f ms/step (%.2fx plain), ranks %s, sigma dev %.1e" % (
        k, m, sec * 1e3, plain_sec / sec, "equal" if res.ranks == plain_res.ranks else "DIFFER", dev))
    return {"value": round(abytes / sec / 1e9, 2), "unit": "GB/s", "ms_per_step": round(sec * 1e3, 3),
            "k": k, "m": m, "m_min": m_min, "f1_min": f1_min, "algorithmic_bytes": abytes,
            "hbm_roofline_frac": round(abytes / sec / 1e9 / HBM_PEAK_GBS, 4),
            "speedup_vs_plain": round(plain_sec / sec, 3),
            "plain_bytes_per_time_GBs": round(plain_bytes / sec / 1e9, 2),
            "parity_vs_plain": {"ranks_equal": res.ranks == plain_res.ranks,
                                "max_sigma_dev_rel_sigma1": dev, "passed": ok}}


def batched(tt, steps, warmup, count=512, parity_elems=1 << 24):
    """Many-tensor form: 512 FP32 exact-TT tensors of mixed shapes (d ~
    U{6..20}, n_i in {2, 4, 8}, 4 KiB .. 64 MiB, bond ranks U{2..16}, unit-
    variance cores, 1e-6 relative noise), r_max = 16, tol = 1e-5, decomposed
    in one persistent launch after autotuning; aggregate effective GB/s, a
    per-tensor parity check against the FP64 oracle on a bounded sample, and
    the same tensors decomposed one by one with the single-tensor path."""
    import ctypes

    import numpy as np
    import torch

    import oracle
    from paper_2102_00104_amd import model, synth
    dev = torch.device("cuda:0")
    specs = synth.batch_specs(count=count, seed=3)
    dims_list = [d for d, _ in specs]
    Xs = [synth.exact_tt_device(d, r, seed=10000 + i, noise=1e-6, noise_seed=20000 + i,
                                device=dev, dtype=torch.float32)
          for i, (d, r) in enumerate(specs)]
    torch.cuda.synchronize()
    in_bytes = sum(4 * synth.prod(d) for d in dims_list)
    log("batched: %d tensors, %.1f MiB FP32; autotuning" % (len(Xs), in_bytes / 2 ** 20))
    cfg, tune_ms = tt.ttsvd_batch_autotune(Xs, dims_list, 16, 1e-5)
    log("batched: best %s (%.3f ms)" % (cfg.as_dict(), tune_ms))
    st = torch.cuda.current_stream().cuda_stream
    n, xs, d, dims, rm, tl = tt._batch_args(Xs, dims_list, 16, 1e-5, st)
    outs = (tt.TTStruct * n)()
    L = tt.lib()

    def once():
        rc = L.ttsvd_decompose_batch(n, xs, d, dims, rm, tl, ctypes.byref(cfg), st, outs)
        if rc != 0:
            raise tt.TTSVDError(rc, L.ttsvd_last_error().decode())

    def free():
        for t in range(n):
            L.ttsvd_tt_free(ctypes.byref(outs[t]))

    for _ in range(warmup):
        once()
        free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        once()
        if k + 1 < steps:
            free()
    sec = (time.perf_counter() - t0) / steps
    ranks = [[int(outs[t].ranks[i]) for i in range(d[t] + 1)] for t in range(n)]
    free()
    # time per phase kind, from the kernel's device clock
    tt.ttsvd_profile_reset()
    tt.ttsvd_profile_enable(True)
    try:
        once()
        free()
        phases = {s_["name"]: round(s_["total_ms"], 3) for s_ in tt.ttsvd_profile_read()}
    finally:
        tt.ttsvd_profile_enable(False)
        tt.ttsvd_profile_reset()
    log("batched: phases %s" % phases)
    abytes = sum(model.algorithmic_bytes(dl, rk, 4) for dl, rk in zip(dims_list, ranks))
    log("batched: %.3f ms per batch, %.1f GB/s" % (sec * 1e3, abytes / sec / 1e9))

    # parity on a bounded sample: smallest tensors first, up to parity_elems elements
    res = tt.ttsvd_decompose_batch(Xs, dims_list, 16, 1e-5, cfg=cfg)
    order = sorted(range(n), key=lambda t: synth.prod(dims_list[t]))
    checked = passed = 0
    budget = parity_elems
    u = 2.0 ** -24
    t_or = time.perf_counter()
    for t in order:
        size = synth.prod(dims_list[t])
        if size > budget:
            break
        budget -= size
        Xh = Xs[t].to(torch.float64).cpu().numpy()
        o = oracle.ttsvd(Xh, dims_list[t], 16, 1e-5)
        g = res[t]
        c = (len(dims_list[t]) - 1) * u + 1e-5
        ok = g.ranks == o.ranks
        if ok:
            for j in range(1, len(dims_list[t])):
                r = o.ranks[j]
                ok &= bool(np.max(np.abs(np.asarray(g.sigma[j])[:r] - o.sigma[j][:r]))
                           <= c * o.sigma[j][0])
            cores = [tt.core_array(cc, (g.ranks[j], g.dims[j], g.ranks[j + 1]))
                     for j, cc in enumerate(g.cores)]
            e = oracle.rel_error(Xh, oracle.tt_full(cores))
            ok &= abs(e - oracle.rel_error(Xh, oracle.tt_full(o.cores))) <= c
        checked += 1
        passed += int(ok)
    t_or = time.perf_counter() - t_or
    log("batched: parity %d / %d tensors (%.1f s of oracle)" % (passed, checked, t_or))

    # the same tensors one by one through the single-tensor path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for X, dl in zip(Xs, dims_list):
        tt.ttsvd_decompose(X, dl, 16, 1e-5)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    log("batched: one by one %.1f ms" % (seq * 1e3))
    return {"value": round(abytes / sec / 1e9, 2), "unit": "GB/s", "ms_per_batch": round(sec * 1e3, 3),
            "tensors": n, "input_bytes": in_bytes, "algorithmic_bytes": abytes,
            "hbm_roofline_frac": round(abytes / sec / 1e9 / HBM_PEAK_GBS, 4),
            "config": cfg.as_dict(), "autotune_best_ms": round(tune_ms, 3), "phases_ms": phases,
            "parity": {"checked": checked, "passed": passed,
                       "sample": "smallest tensors up to %d elements in total" % parity_elems},
            "one_by_one_ms": round(seq * 1e3, 3), "speedup_vs_one_by_one": round(seq / sec, 2)}


def serve_trace(tt, trace, workers, max_batch, live_cap=48 << 30, ahead_s=1.0):
    """Replay a request trace in real time against a Server.  Each request's
    FP32 tensor (``synth.serving_tensor``: its exact TT contracted in FP32
    plus 1e-6 relative noise) is synthesised on the device by a producer
    stream ahead of its
    arrival (at most `ahead_s` seconds ahead, and only while the tensors
    alive -- synthesised, queued or running -- stay within `live_cap` bytes),
    then submitted at its scheduled arrival time; the server's work on it
    waits on the synthesis through an event, never on the host.  A request
    whose tensor could not be enqueued by its arrival (memory cap) is
    submitted late; the lateness counts in its latency.  Returns per-request
    records."""
    import collections

    import torch

    from paper_2102_00104_amd import synth
    dev = torch.device("cuda:0")
    cfg = tt.server_default_config()
    cfg.workers, cfg.max_batch = workers, max_batch
    syn = torch.cuda.Stream()    # producer: tensor synthesis
    hand = torch.cuda.Stream()   # hand-off: waits for one tensor's synthesis event
    ahead = collections.deque()  # (index, tensor, event, bytes): synthesised, not submitted
    live = {}                    # ticket -> (tensor, bytes, request index)
    state = {"bytes": 0, "next": 0}
    rec = {}

    def nbytes(q):
        return synth.prod(q["dims"]) * 4

    # every request's cores on the device before the replay starts: the loop
    # below then only enqueues device work
    cores = [synth.serving_cores_device(q["dims"], q["ranks"], 40000 + i, dev)
             for i, q in enumerate(trace)]
    torch.cuda.synchronize()

    def produce():
        i = state["next"]
        with torch.cuda.stream(syn):
            X = synth.serving_tensor(cores[i], 1e-6, 50000 + i, dev)
            ev = torch.cuda.Event()
            ev.record(syn)
        b = nbytes(q)
        ahead.append((i, X, ev, b))
        state["bytes"] += b
        state["next"] = i + 1

    def collect(srv, wait_ms):
        for c in srv.poll(max_n=512, wait_ms=wait_ms):
            X, b, i = live.pop(c["ticket"])
            state["bytes"] -= b
            r = c["result"]
            if c["status"] != 0:
                log("serving: request %d failed (%d): %s" % (i, c["status"], c["message"]))
            rec[i].update(status=c["status"], t_submit=c["t_submit"], t_start=c["t_start"],
                          t_done=c["t_done"], batch=c["batch_size"], batched=c["batched"],
                          ranks=r.ranks if r is not None else None)
            del X

    with tt.Server(cfg) as srv:
        t0 = tt.server_clock() + 0.05
        for i, q in enumerate(trace):
            while True:
                now = tt.server_clock()
                left = t0 + q["t"] - now
                nxt = state["next"]
                if nxt <= i:
                    # this request's tensor is not enqueued yet: enqueue it as
                    # soon as memory allows (nothing alive: always)
                    if state["bytes"] + nbytes(trace[nxt]) <= live_cap or state["bytes"] == 0:
                        produce()
                    else:
                        collect(srv, 1)
                    continue
                if left <= 0:
                    break
                if (nxt < len(trace) and trace[nxt]["t"] <= now - t0 + ahead_s
                        and state["bytes"] + nbytes(trace[nxt]) <= live_cap):
                    produce()
                    continue
                collect(srv, max(1, min(20, int(left * 1e3))))
            j, X, ev, b = ahead.popleft()
            assert j == i
            hand.wait_event(ev)
            now = tt.server_clock()
            rec[i] = dict(arrival=t0 + q["t"], ready=now)
            ticket = srv.submit(X, q["dims"], q["r_max"], q["tol"], stream=hand)
            live[ticket] = (X, b, i)
        while srv.pending() > 0 or live:
            collect(srv, 50)
    return [rec[i] for i in range(len(trace))]


def serving(tt, duration):
    """Serving workload: Poisson arrivals at 200/s over `duration` seconds,
    sizes 1 MiB .. 4 GiB (FP32), r_max U{4..64}, tol log-uniform in
    [1e-5, 1e-2]; the batching server (4 workers) against one worker that
    runs every request alone (the sequential plain path), same trace."""
    import numpy as np

    from paper_2102_00104_amd import model, synth
    trace = synth.serving_trace(duration_s=duration, rate=200.0, seed=4)

    def summary(recs):
        ok = [r for r in recs if r.get("status") == 0]
        lat = np.array([r["t_done"] - r["ready"] for r in ok])
        lat_arr = np.array([r["t_done"] - r["arrival"] for r in ok])
        span = max(r["t_done"] for r in ok) - min(r["ready"] for r in ok)
        abytes = sum(model.algorithmic_bytes(q["dims"], r["ranks"], 4)
                     for q, r in zip(trace, recs) if r.get("status") == 0)
        batches = [r["batch"] for r in ok if r["batched"]]
        return {"completed": len(ok), "failed": len(recs) - len(ok),
                "late_submissions": sum(1 for r in recs if r["ready"] - r["arrival"] > 5e-3),
                "p50_ms": round(float(np.percentile(lat_arr, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat_arr, 99)) * 1e3, 3),
                "p50_ms_from_ready": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms_from_ready": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "aggregate_GBs": round(abytes / span / 1e9, 2), "span_s": round(span, 3),
                "batched_requests": len(batches),
                "mean_batch_of_batched": round(float(np.mean(batches)), 2) if batches else 0.0,
                "max_batch_seen": max(r["batch"] for r in ok)}

    log("serving: %d requests over %.1f s (%.1f GiB FP32)" % (
        len(trace), duration, sum(synth.prod(q["dims"]) for q in trace) * 4 / 2 ** 30))
    fast = summary(serve_trace(tt, trace, workers=4, max_batch=512))
    log("serving: batching server %s" % fast)
    seq = summary(serve_trace(tt, trace, workers=1, max_batch=1))
    log("serving: sequential %s" % seq)
    return {"requests": len(trace), "duration_s": duration, "rate_per_s": 200.0,
            "latency": "p50/p99: scheduled arrival -> cores ready (queueing included); "
                       "*_from_ready: submission -> cores ready (tensors are synthesised "
                       "ahead and submitted at their arrival unless the memory cap delays "
                       "them: late_submissions)",
            "offered_input_GBs": round(sum(synth.prod(q["dims"]) for q in trace) * 4 / duration / 1e9, 2),
            "server": fast, "sequential": seq}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of this process (the oracle's C code)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def cpu_baseline(d_sample, r_max, d_single=25):
    """The CPU FP64 oracle on bounded samples of the same workload: all host
    cores on a 2^d_sample tensor, and one thread on a 2^d_single tensor."""
    import numpy as np

    import oracle
    from paper_2102_00104_amd import model

    def run(d):
        dims = [2] * d
        X = np.random.default_rng(0).random(2 ** d)
        t0 = time.perf_counter()
        o = oracle.ttsvd(X, dims, r_max, 0.0)
        dt = time.perf_counter() - t0
        return model.algorithmic_bytes(dims, o.ranks, 8) / dt / 1e9, dt

    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    gbs, dt = run(d_sample)
    single = None
    if _omp_threads(1):
        try:
            g1, dt1 = run(d_single)
            single = {"value": round(g1, 4), "unit": "GB/s", "cores": 1,
                      "sample": "2^%d-element tensor, d=%d, n_i=2, r_max=%d; %.2f s" % (
                          d_single, d_single, r_max, dt1)}
        finally:
            _omp_threads(threads)
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "2^%d-element U[0,1) FP64 tensor, d=%d, n_i=2, r_max=%d, no tol "
                      "(1/%d of the workload); %.2f s" % (d_sample, d_sample, r_max,
                                                          2 ** (28 - d_sample), dt),
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "single_thread": single}


def machine(tt):
    """Measured roofline denominators (the analog of the paper's Table 1):
    load, store, copy and triad HBM bandwidth over 3 GiB, and the FP64 FMA
    rate, from the library's micro-benchmark kernels."""
    import torch
    buf = torch.zeros(3 * 2 ** 27, dtype=torch.float64, device="cuda:0")
    res = {}
    for kind, name in ((tt.MB_LOAD, "load"), (tt.MB_STORE, "store"), (tt.MB_COPY, "copy"),
                       (tt.MB_TRIAD, "triad")):
        ms, by = tt.ttsvd_machine_bench(kind, buf, 20)
        res[name + "_GBs"] = round(by / ms / 1e6, 1)
    ms, fl = tt.ttsvd_machine_bench(tt.MB_FMA, buf, 10)
    res["fp64_fma_TFs"] = round(fl / ms / 1e9, 2)
    del buf
    torch.cuda.empty_cache()
    return res


def family_split(stats, ndec):
    """Milliseconds per decomposition spent in each building block (the
    analog of the paper's per-function timings): TSQR, small SVD, TSMM."""
    fam = {"tsqr": 0.0, "svd": 0.0, "tsmm": 0.0, "other": 0.0}
    for s in stats:
        n = s["name"]
        key = ("tsqr" if n.startswith("tsqr") else "svd" if n.startswith("svd")
               else "tsmm" if n.startswith("tsmm") else "other")
        fam[key] += s["total_ms"]
    return {k + "_ms": round(v / ndec, 3) for k, v in fam.items()}


def small_latency(tt, steps, warmup):
    """The d = 12 exact-TT workload (4096 values): latency of one
    decomposition in microseconds."""
    import torch

    from paper_2102_00104_amd import synth
    dims, X, r_max, tol = synth.small_exact_tt_workload()
    Xd = torch.from_numpy(X).to("cuda:0")
    n = max(steps, 20)
    sec, res, med = time_decompose(tt, Xd, dims, r_max, tol, n, max(warmup, 3))
    return {"workload": "d=12, n_i=2 exact TT (ranks 4, Gaussian cores) + 1e-8 noise, "
                        "r_max=8, tol=1e-10, FP64", "median_us": round(med * 1e6, 1),
            "mean_us": round(sec * 1e6, 1), "calls": n, "ranks": res.ranks}


def two_sided(tt, model, X, dims, r_max, steps, warmup, plain_sec, plain_res):
    """Algorithm 4 (two-sided) on the resident tensor: time per decomposition
    (C call with prebuilt arguments), its effective GB/s over its own
    algorithmic bytes (TSQR read + TSMM read/write of every step, plus the
    transposes' read and write of the remainder), and its result beside the
    plain one's."""
    import ctypes

    import numpy as np
    import torch
    L = tt.lib()
    d = len(dims)
    st = torch.cuda.current_stream().cuda_stream
    xs = tt.TensorStruct(X.data_ptr(), tt.dtype_code(X), 0, st)
    arr = (ctypes.c_int64 * d)(*dims)
    out = tt.TTStruct()

    def once():
        rc = L.ttsvd_decompose_two_sided(ctypes.byref(xs), arr, d, r_max, 0.0, ctypes.byref(out))
        if rc != 0:
            raise tt.TTSVDError(rc, L.ttsvd_last_error().decode())
        L.ttsvd_tt_free(ctypes.byref(out))
    for _ in range(warmup):
        once()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        once()
        ts.append(time.perf_counter() - t0)
    med = sorted(ts)[len(ts) // 2]
    g = tt.ttsvd_decompose_two_sided(X, dims, r_max, 0.0)
    # algorithmic bytes of the two-sided order at the ranks it chose
    e = X.element_size()
    size, lo, hi, right, ab = X.numel(), 0, d - 1, True, 0.0
    while lo < hi:
        m = dims[hi] * g.ranks[hi + 1] if right else g.ranks[lo] * dims[lo]
        r = g.ranks[hi] if right else g.ranks[lo + 1]
        nxt = size // m * r
        last = (hi - 1 == lo) if right else (lo + 1 == hi)
        ab += e * (2 * size + nxt) + (0 if last else 2 * e * nxt)
        size = nxt
        if right:
            hi -= 1
        else:
            lo += 1
        right = not right
    return {"ms_per_step": round(med * 1e3, 3), "value": round(ab / med / 1e9, 2), "unit": "GB/s",
            "algorithmic_bytes": ab, "speedup_vs_plain": round(plain_sec / med, 3),
            "ranks": g.ranks, "ranks_equal_plain": g.ranks == plain_res.ranks,
            "err_bound_rel": g.err_bound / g.norm_sigma,
            "plain_err_bound_rel": plain_res.err_bound / plain_res.norm_sigma}


def alg1_comparator(tt, d=24, r_max=32):
    """Algorithm 1 (full SVD of every unfolding, rocSOLVER GESVD without QR
    preprocessing) against Algorithm 2 on the same 2^d U[0,1) FP64 tensor
    (d modes of size 2, r_max, no tol): the speed-up of the QR trick."""
    import numpy as np
    import torch
    X = torch.from_numpy(np.random.default_rng(0).random(2 ** d)).to("cuda:0")
    dims = [2] * d
    tt.ttsvd_decompose_alg1(X, dims, r_max, 0.0)          # warm-up
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        g1 = tt.ttsvd_decompose_alg1(X, dims, r_max, 0.0)
        ts.append(time.perf_counter() - t0)
    t1 = sorted(ts)[1]
    sec2, g2, med2 = time_decompose(tt, X, dims, r_max, 0.0, 10, 2)
    dev = max(float(np.max(np.abs(np.asarray(g1.sigma[j]) - np.asarray(g2.sigma[j])))) /
              float(g1.sigma[j][0]) for j in range(1, d))
    del X
    torch.cuda.empty_cache()
    return {"workload": "2^%d U[0,1) FP64, d=%d, n_i=2, r_max=%d, no tol" % (d, d, r_max),
            "alg1_ms": round(t1 * 1e3, 2), "alg2_ms": round(med2 * 1e3, 3),
            "qr_trick_speedup": round(t1 / med2, 1), "ranks_equal": g1.ranks == g2.ranks,
            "max_sigma_dev_rel_sigma1": dev,
            "paper_context": "about 50x for TSQR with the QR trick against a plain LAPACK SVD "
                             "(10^7 x m, m <= 50, one 14-core Skylake-SP socket)"}


def sweeps(tt):
    """GB/s and TFLOP/s of ttsvd_tsqr_r and ttsvd_gemm_reshape against the
    column count m on 1 GiB FP64 inputs (rows = 2^27 / m; the product has
    k = max(1, m / 2) columns and n_next = 2), the analog of the paper's
    roofline plots of the two building blocks (median of 5 calls)."""
    import torch
    out = {"tsqr_r": [], "gemm_reshape": []}
    dev = torch.device("cuda:0")
    for m in (1, 2, 4, 8, 16, 32, 50, 64, 100, 128):
        rows = (2 ** 27 // m) // 2 * 2
        W = torch.rand(rows * m, dtype=torch.float64, device=dev)
        R = torch.empty(m * m, dtype=torch.float64, device=dev)
        need = tt.ttsvd_tsqr_workspace_size(tt.TTSVD_F64, rows, m)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        k = max(1, m // 2)
        V = torch.rand(m * k, dtype=torch.float64, device=dev)
        Y = torch.empty(rows * k, dtype=torch.float64, device=dev)

        def med(fn):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(5):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return sorted(ts)[2]
        t = med(lambda: tt.ttsvd_tsqr_r(W, tt.TTSVD_F64, rows, m, rows, R, m, ws, need))
        out["tsqr_r"].append({"m": m, "rows": rows, "ms": round(t * 1e3, 3),
                              "GBs": round(8.0 * rows * m / t / 1e9, 1),
                              "TFs": round(2.0 * rows * m * m / t / 1e12, 2)})
        t = med(lambda: tt.ttsvd_gemm_reshape(W, tt.TTSVD_F64, rows, m, rows, V, m, k, 2, Y,
                                              rows // 2))
        out["gemm_reshape"].append({"m": m, "k": k, "rows": rows, "ms": round(t * 1e3, 3),
                                    "GBs": round(8.0 * rows * (m + k) / t / 1e9, 1),
                                    "TFs": round(2.0 * rows * m * k / t / 1e12, 2)})
        del W, R, ws, V, Y
    torch.cuda.empty_cache()
    return out


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
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-thick", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--no-machine", action="store_true")
    ap.add_argument("--no-sweeps", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-alg1", action="store_true")
    ap.add_argument("--no-two-sided", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (counter calibration)")
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
        sec, res, med = time_decompose(tt, X, dims, args.r_max, 0.0, args.steps, args.warmup)
        assert res.ranks == ranks, (res.ranks, ranks)
        log("%s: %.3f ms/step (median %.3f ms), %.1f GB/s" % (wname, sec * 1e3, med * 1e3,
                                                             abytes / sec / 1e9))
        nprof = max(1, min(args.steps, 3))
        stats = kernel_profile(tt, X, dims, args.r_max, 0.0, nprof)
        for s in sorted(stats, key=lambda s: -s["total_ms"]):
            log("  %-40s n=%4d  %9.3f ms  %8.1f GB/s  %6.2f TF/s" % (
                s["name"], s["launches"], s["total_ms"],
                s["bytes"] / (s["total_ms"] / 1e3) / 1e9 if s["total_ms"] else 0,
                s["flops"] / (s["total_ms"] / 1e3) / 1e12 if s["total_ms"] else 0))
        results.append(dict(workload=wname, dims=dims, ranks=ranks, ms_per_step=sec * 1e3,
                            median_ms=med * 1e3, value_median=abytes / med / 1e9,
                            value=abytes / sec / 1e9, bytes=abytes, flops=aflops,
                            roofline=roofline_of(stats, wname), kernels=stats, sec=sec, res=res,
                            split=family_split(stats, nprof)))

    if args.copy_calibration:
        # a plain copy of known size: reads 2^27 doubles, writes 2^27 doubles
        Y = torch.empty(2 ** 27, dtype=torch.float64, device=dev)
        Y.copy_(X[: 2 ** 27])
        torch.cuda.synchronize()
        del Y

    head = results[0]
    line = {
        "metric": "TT-SVD effective GB/s vs 2-read HBM roofline",
        "value": round(head["value"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "median_ms_per_step": round(head["median_ms"], 3),
        "value_median": round(head["value_median"], 2),
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
        "time_split": head["split"],
        "others": [{"workload": r["workload"], "value": round(r["value"], 2), "unit": "GB/s",
                    "ms_per_step": round(r["ms_per_step"], 3),
                    "median_ms_per_step": round(r["median_ms"], 3),
                    "hbm_roofline_frac": round(r["value"] / HBM_PEAK_GBS, 4),
                    "roofline": r["roofline"], "time_split": r["split"]} for r in results[1:]],
    }
    if not args.no_machine:
        mach = machine(tt)
        log("machine: %s" % mach)
        mach["headline_frac_of_measured_load"] = round(head["value"] / mach["load_GBs"], 4)
        line["machine"] = mach
    if not args.no_small:
        line["small_latency"] = small_latency(tt, args.steps, args.warmup)
        log("small workload: %s" % line["small_latency"])
    if not args.no_alg1:
        line["alg1_comparator"] = alg1_comparator(tt)
        log("alg1 comparator: %s" % line["alg1_comparator"])
    if not args.no_sweeps:
        line["sweeps"] = sweeps(tt)
        log("sweeps: %s" % line["sweeps"])
    if not args.no_precision:
        line["precision_forms"] = precision_forms(tt, X, head["dims"], args.r_max, args.steps,
                                                  args.warmup, head["sec"], head["res"])
    if not args.no_thick:
        line["thick_bounds"] = thick_bounds(tt, model, X, head["dims"], args.r_max, args.steps,
                                            args.warmup, head["sec"], head["res"])
    if not args.no_two_sided:
        line["two_sided"] = two_sided(tt, model, X, head["dims"], args.r_max, max(args.steps, 5),
                                      args.warmup, head["sec"], head["res"])
        log("two-sided: %s" % line["two_sided"])
    if not args.no_batched:
        line["batched"] = batched(tt, args.steps, args.warmup)
    if not args.no_serving:
        line["serving"] = serving(tt, args.serve_seconds)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a 2^%d sample" % args.cpu_sample_d)
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample_d, args.r_max)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
