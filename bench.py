"""Benchmark: truncated vs full product on one MI355X.

A step is one low product, one high product and one full product of the same
two n-bit operands (n = 2^30 by default, the largest single instance:
uniform random 64-bit limbs from a fixed seed), inputs resident in HBM.
Prints one JSON line with

* value: whole-step operand throughput, 3 n bits / step time, in Mbit/s;
* per-kind time and Mbit/s, and the lo/full and hi/full time ratios;
* per-kernel times (HIP events on the launch stream), each kernel's
  algorithmic GB/s against the 8 TB/s HBM peak and a measured copy ceiling;
* roofline: algorithmic bytes / time of the dominant (longest) kernel;
* n2_24: the same step at n = 2^24 (operands and transforms fit the 256 MiB
  last-level cache, so its GB/s are effective figures);
* precision: rounding distances at n = 2^26 for several digit sizes, and
  the edge-digit pattern through the checked entry point;
* serving: throughput (saturated) and p50 / p99 latency (Poisson arrivals)
  of a mixed stream of requests (n from 2^12 to 2^22 bits, all three kinds)
  through the library's continuous-batching server;
* cpu_baseline: the CPU oracle (Karatsuba on 64-bit limbs) on the host cores.

Every guard of the timed products is read; a tripped guard aborts the run.
Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "mul_hi/mul_lo vs mul_full time ratio; operand Mbit/s; p50/p99 latency batched"


def kernel_bytes(plan, n_bits, kind):
    """Algorithmic HBM bytes per launch of each kernel (reads + writes).

    With N real coefficients and M = N/2 complex points: K1 reads both
    operands (n/8 bytes each) and writes two packed spectra (2 M 16 = 16 N
    bytes); K2 reads them (16 N) and writes the product spectrum (8 N); K3
    reads and writes one complex array (8 N + 8 N); K4 reads the real
    convolution (8 N) and writes the result limbs.  With the three-pass
    split the middle passes read and write both spectra (32 N) forward and
    the product (16 N) inverse."""
    N = plan["N"]
    L = (n_bits + 63) // 64
    out = 16 * L if kind == "full" else 8 * L
    return {"fused_fft": 2 * 8 * L + 8 * N,
            "split_map_colfft": 2 * 8 * L + 16 * N,
            "mid_colfft": 32 * N,
            "rowfft_pointwise_rowifft": 24 * N,
            "mid_colifft": 16 * N,
            "col_ifft": 16 * N,
            "backmap_round_carry": 8 * N + out}


def source_hash():
    """sha1 of the HIP sources and the C header (ties stored counter figures
    to the kernels they were taken on)."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_1703_00640_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc)) + [
        os.path.join(ROOT, "include", "tmul.h")]
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(log2n):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
    (profiles/traffic_n2_<log2n>.txt), keyed by kind:kernel, or {} when the
    file is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_n2_%d.txt" % log2n)
    if not os.path.exists(path):
        return {}
    out, src = {}, None
    for line in open(path):
        f = line.split()
        if len(f) == 2 and f[0] == "source_hash:":
            src = f[1]
        elif len(f) == 4 and f[0] == "traffic:":
            out[f[1]] = int(f[2]) + int(f[3])
    return out if src == source_hash() else {}


def pmc_pass(n_bits, reps=2):
    """Workload for rocprofv3 runs (kernel trace and counter passes): the
    autotuner's timing runs for every kind (the benchmark's FFT splits) and
    untimed products of each kind, then a marker dispatch (a fill of a
    16-bit integer tensor, the only one in the run), then `reps` steps of one
    product of each kind, then a plain 256 MiB device copy (the calibration kernel for
    FETCH_SIZE and WRITE_SIZE).
    Summaries take the dispatches between the marker and the copy."""
    import torch
    import paper_1703_00640_amd as tm
    from paper_1703_00640_amd import inputs
    dev = torch.device("cuda:0")
    u, v = inputs.operand_pair(n_bits, 5)
    du = torch.from_numpy(u.view(np.int64)).to(dev)
    dv = torch.from_numpy(v.view(np.int64)).to(dev)
    kinds = ("lo", "hi", "full")
    for k in kinds:
        tm.autotune(k, n_bits)  # the same FFT split as the benchmark
    ws = {k: torch.empty(tm.plan(k, n_bits)["workspace_bytes"], dtype=torch.uint8, device=dev)
          for k in kinds}
    # untimed steps first, so no kind runs cold (the VALU-bound kernels of a
    # kind run back to back after another kind's took several launches to
    # settle; interleaved steps, as in the benchmark, do not show this)
    for _ in range(max(reps, 8)):
        for k in kinds:
            tm.mul(k, du, dv, n_bits, workspace=ws[k])
    torch.cuda.synchronize()
    torch.full((1,), 3, dtype=torch.int16, device=dev)  # marker
    for _ in range(reps):  # interleaved like the benchmark's step
        for k in kinds:
            tm.mul(k, du, dv, n_bits, workspace=ws[k])
    a = torch.ones(1 << 25, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    print("pmc pass done", flush=True)


def copy_ceiling_gb_s(mib=256, reps=10):
    """Achieved bandwidth of a plain device-to-device copy of `mib` MiB
    (read + write bytes per second): the practical ceiling the kernels'
    algorithmic GB/s is also compared against."""
    import torch
    dev = torch.device("cuda:0")
    a = torch.ones(mib << 17, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(gbs, 1)


def serving_bench(count=4096, n_streams=4):
    """Mixed-request serving through the continuous-batching server: count
    requests, n log-uniform over [2^12, 2^22] bits (whole limbs), kind
    uniform over lo / hi / full, uniform random operands in pinned host
    memory (copies in and out are part of every request).  After one
    untimed pass, all requests at t = 0 (saturation throughput R), then
    Poisson arrivals at 0.5 R and 0.9 R; latency = completion seen on the
    host - arrival."""
    import paper_1703_00640_amd as tm
    from paper_1703_00640_amd import inputs, serving
    mix = inputs.serving_mix(count, seed=6)
    m = serving.Mix(mix, seed=7)
    # warm-up pass over the same mix (first launches of every kernel
    # instance load its code; pinned staging buffers are allocated)
    serving.run(m, np.zeros(count), n_streams=n_streams)
    sat, _, _ = serving.run(m, np.zeros(count), n_streams=n_streams)
    # every request arrives at t = 0 here: the spread of completion times is
    # queueing, not latency, so only throughput is kept from this run
    sat = {k: v for k, v in sat.items() if k not in ("p50_ms", "p99_ms")}
    out = {"workload": "%d requests, n log-uniform over [2^12, 2^22] bits, kind uniform "
                       "lo/hi/full, host operands (pinned), pool 1 GiB, %d streams"
                       % (count, n_streams),
           "saturated": sat}
    for frac in (0.5, 0.9):
        rate = frac * sat["throughput_rps"]
        arr = inputs.poisson_arrivals(count, rate, seed=8)
        st, _, _ = serving.run(m, arr, n_streams=n_streams)
        st["offered_rps"] = rate
        out["poisson_%.1f" % frac] = st
    # the same server with batches captured into HIP graphs: every batch of
    # two or more requests, and only batches of 16 or more
    for mode, key in ((True, "graph_mode"), ("auto", "graph_mode_auto")):
        gsat, _, _ = serving.run(m, np.zeros(count), n_streams=n_streams, graphs=mode)
        rate = 0.5 * sat["throughput_rps"]
        gp, _, _ = serving.run(m, inputs.poisson_arrivals(count, rate, seed=8), n_streams=n_streams,
                               graphs=mode)
        gq, _, _ = serving.run(m, inputs.poisson_arrivals(count, 1.8 * rate, seed=8),
                               n_streams=n_streams, graphs=mode)
        out[key] = {"saturated_throughput_rps": gsat["throughput_rps"],
                    "poisson_0.5": {"p50_ms": gp["p50_ms"], "p99_ms": gp["p99_ms"],
                                    "throughput_rps": gp["throughput_rps"]},
                    "poisson_0.9": {"p50_ms": gq["p50_ms"], "p99_ms": gq["p99_ms"],
                                    "throughput_rps": gq["throughput_rps"]},
                    "guard_flags": gsat["guard_flags"] | gp["guard_flags"] | gq["guard_flags"],
                    "failed": gsat["failed"] + gp["failed"] + gq["failed"]}
    # storage: the truncated products' transforms hold N = 3n/b' reals
    # against 2N for the full product; admission capacity of a 1 GiB pool
    cap = {}
    for lg in (16, 22, 26):
        nb = 1 << lg
        row = {}
        for k in ("lo", "hi", "full"):
            fp = tm.server_footprint(k, nb)
            row[k] = {"workspace_bytes": tm.workspace_bytes(k, nb), "footprint_bytes": fp,
                      "per_gib": (1 << 30) // fp if fp else 0}
        row["lo_full_workspace_ratio"] = round(row["lo"]["workspace_bytes"] / row["full"]["workspace_bytes"], 4)
        cap["n=2^%d" % lg] = row
    out["admission_capacity"] = cap
    for v in out.values():
        if isinstance(v, dict):
            for k in list(v):
                if isinstance(v[k], float):
                    v[k] = round(v[k], 6)
    return out


def small_latency_bench(log2n=16, reps=200):
    """One small multiplication at a time (n = 2^16, the smallest benchmark
    size): microseconds per call for back-to-back eager calls (launch-bound
    at this size) and for replays of the same call captured in a HIP graph;
    then 256 such products of one kind in packed launches, microseconds of
    GPU time per product."""
    import torch
    import paper_1703_00640_amd as tm
    from paper_1703_00640_amd import inputs
    n = 1 << log2n
    L = n // 64
    dev = torch.device("cuda:0")
    u, v = inputs.operand_pair(n, 2)
    du = torch.from_numpy(u.view(np.int64)).to(dev)
    dv = torch.from_numpy(v.view(np.int64)).to(dev)
    res = {"n_bits": n, "eager_us": {}, "graph_us": {}}
    for k in ("lo", "hi", "full"):
        tm.prepare(k, n)
        out = torch.empty(2 * L if k == "full" else L, dtype=torch.int64, device=dev)
        ws = torch.empty(tm.plan(k, n)["workspace_bytes"], dtype=torch.uint8, device=dev)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                tm.mul(k, du, dv, n, out=out, workspace=ws)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            tm.mul(k, du, dv, n, out=out, workspace=ws)
        stream = torch.cuda.current_stream(dev)
        for name, fn in (("eager_us", lambda: tm.mul(k, du, dv, n, out=out, workspace=ws)),
                         ("graph_us", graph.replay)):
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res[name][k] = round(e0.elapsed_time(e1) * 1e3 / reps, 2)
        del graph
    # many small products in packed launches (tm_mul_batched: one launch per
    # stage for the whole batch), GPU time per product
    nb, breps = 256, 20
    pool_u = torch.from_numpy(inputs.operand_pair(n * nb, 3)[0].view(np.int64)).to(dev)
    pool_v = torch.from_numpy(inputs.operand_pair(n * nb, 4)[0].view(np.int64)).to(dev)
    res["batched_us_per_product"] = {"batch": nb}
    for k in ("lo", "hi", "full"):
        nout = 2 * L if k == "full" else L
        outs = torch.empty(nb * nout, dtype=torch.int64, device=dev)
        reqs = [(k, pool_u[i * L:(i + 1) * L], pool_v[i * L:(i + 1) * L], n, outs[i * nout:(i + 1) * nout])
                for i in range(nb)]
        ws = torch.empty(tm.workspace_bytes_batched(reqs), dtype=torch.uint8, device=dev)
        for _ in range(3):
            tm.mul_batched(reqs, workspace=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(breps):
            tm.mul_batched(reqs, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        res["batched_us_per_product"][k] = round(e0.elapsed_time(e1) * 1e3 / (breps * nb), 3)
    return res


def mulmod_bench(log2n=24, reps=10):
    """Barrett modular multiplication (tm_mulmod: one full, one high and one
    low product plus carry fixups) at n = 2^24 with the modulus 2^n - 1,
    whose reciprocal floor(2^(2n) / m) is 2^n + 1; time against one full
    product of the same size."""
    import torch
    import paper_1703_00640_amd as tm
    from paper_1703_00640_amd import inputs
    n = 1 << log2n
    L = n // 64
    dev = torch.device("cuda:0")
    a, b = inputs.operand_pair(n, 9)
    da = torch.from_numpy(a.view(np.int64)).to(dev)
    db = torch.from_numpy(b.view(np.int64)).to(dev)
    m = torch.full((L,), -1, dtype=torch.int64, device=dev)
    mu = torch.zeros(n // 64 + 1, dtype=torch.int64, device=dev)
    mu[0] = 1
    mu[L] = 1
    ws = torch.empty(tm._load().tm_workspace_bytes_mulmod(n), dtype=torch.uint8, device=dev)
    out = torch.empty(L, dtype=torch.int64, device=dev)
    out_full = torch.empty(2 * L, dtype=torch.int64, device=dev)
    ws_full = torch.empty(tm.plan("full", n)["workspace_bytes"], dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    res = {"n_bits": n, "modulus": "2^n - 1"}
    for name, fn in (("mulmod_ms", lambda: tm.mulmod(da, db, m, mu, n, out=out, workspace=ws)),
                     ("full_ms", lambda: tm.mul("full", da, db, n, out=out_full, workspace=ws_full))):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = round(e0.elapsed_time(e1) / reps, 4)
    res["ratio_to_full"] = round(res["mulmod_ms"] / res["full_ms"], 3)
    return res


def precision_bench(log2n=26, reps=5):
    """The high product at n = 2^26 (the precision-comparison size): the
    maximum rounding distance over all coefficients (the guard) and the time
    for FP64 digit sizes b = 10..13 on uniform random operands, for the
    default b on the edge-digit pattern (every digit 2^(b-1)) with the
    checked call's fallback, whether the worst-case bound admits a plan at
    this size, and the FP32 path (double-float FFT passes, b = 9)."""
    import torch
    import paper_1703_00640_amd as tm
    from paper_1703_00640_amd import inputs
    n = 1 << log2n
    dev = torch.device("cuda:0")
    u, v = inputs.operand_pair(n, 4)
    du = torch.from_numpy(u.view(np.int64)).to(dev)
    dv = torch.from_numpy(v.view(np.int64)).to(dev)
    stream = torch.cuda.current_stream(dev)

    def measure(a, b, guaranteed=False):
        g = tm.new_guard(dev)
        out = tm.mul("hi", a, b, n, guard=g, guaranteed=guaranteed)
        torch.cuda.synchronize()
        gd = tm.read_guard(g)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            tm.mul("hi", a, b, n, out=out, guaranteed=guaranteed)
        e1.record(stream)
        torch.cuda.synchronize()
        return {"b": gd.b, "lam": gd.lam, "N": gd.N, "max_dist": round(gd.max_dist, 6),
                "flags": gd.flags, "ms": round(e0.elapsed_time(e1) / reps, 4)}

    res = {"n_bits": n, "kind": "hi", "fp64_random": []}
    prev = os.environ.get("TM_FORCE_B")
    try:
        for b in (10, 11, 12, 13):
            os.environ["TM_FORCE_B"] = str(b)
            res["fp64_random"].append(measure(du, dv))
    finally:
        if prev is None:
            os.environ.pop("TM_FORCE_B", None)
        else:
            os.environ["TM_FORCE_B"] = prev
    # edge digits: every b-bit field of the high product's split (u 2^s,
    # s = (N + 1) b - n) equal to 2^(b-1), so each balanced digit sits at
    # the edge of its range; the default plan's guard reports it and the
    # checked call recomputes with its guaranteed fallback
    pl = tm.plan("hi", n)
    b0, s0 = pl["b"], (pl["N"] + 1) * pl["b"] - n
    adv = torch.from_numpy(inputs.digit_pattern(n, b0, 1 << (b0 - 1), s0).view(np.int64)).to(dev)
    res["fp64_edge_digits"] = measure(adv, adv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, gck = tm.mul_checked("hi", adv, adv, n)
    res["fp64_edge_digits_checked"] = {"b": gck.b, "N": gck.N, "max_dist": round(gck.max_dist, 6),
                                       "flags": gck.flags,
                                       "ms_incl_sync": round((time.perf_counter() - t0) * 1e3, 3),
                                       "fallback": "full product's guaranteed plan + extraction"}
    try:
        gp = tm.plan("hi", n, guaranteed=True)
        res["fp64_guaranteed"] = measure(du, dv, guaranteed=True)
        res["fp64_guaranteed"]["bound"] = gp["rounding_bound"]
    except tm.TmulError as e:
        res["fp64_guaranteed"] = {"supported": False, "reason": str(e)}
    # FP32 path: double-float FFT passes, digit sizes for its ~48-bit
    # arithmetic (tm_mul_fp32c), random operands and the edge pattern of its
    # own plan
    g = tm.new_guard(dev)
    out = tm.mul("hi", du, dv, n, guard=g, fp32c=True)
    torch.cuda.synchronize()
    gd = tm.read_guard(g)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        tm.mul("hi", du, dv, n, out=out, fp32c=True)
    e1.record(stream)
    torch.cuda.synchronize()
    pf = tm.plan("hi", n, fp32c=True)
    res["fp32_compensated"] = {"b": gd.b, "lam": gd.lam, "N": gd.N, "max_dist": round(gd.max_dist, 6),
                               "flags": gd.flags, "ms": round(e0.elapsed_time(e1) / reps, 4),
                               "worst_case_bound": pf["rounding_bound"],
                               "arithmetic": "double-float FFT passes; FP64 twiddle generation, "
                                             "maps, theta, scaling, rounding"}
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_bits, threads, n_single):
    """The oracle (oracle/: schoolbook + Karatsuba on 64-bit limbs) timed on
    the host cores: one full product of the benchmark's operand pair at
    n_bits on `threads` threads (the oracle computes the low and high
    products by extraction from the same full product, so its lo + hi + full
    step is three of these), and one single-threaded full product at
    n_single bits."""
    import oracle
    from paper_1703_00640_amd import inputs
    u, v = inputs.operand_pair(n_bits, 5)
    t0 = time.perf_counter()
    oracle.mul_full(u, v, n_bits, threads)
    dt = time.perf_counter() - t0
    del u, v
    u1, v1 = inputs.operand_pair(n_single, 2)
    t1 = time.perf_counter()
    oracle.mul_full(u1, v1, n_single, 1)
    dt1 = time.perf_counter() - t1
    return {"value": round(n_bits / dt / 1e6, 3), "unit": "operand Mbit/s",
            "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": "one full product of the n=2^%d operand pair on %d threads (%.1f s); the "
                      "oracle's lo+hi+full step is three such products"
                      % (n_bits.bit_length() - 1, threads, dt),
            "single_thread": {"n_bits": n_single, "seconds": round(dt1, 3),
                              "value": round(n_single / dt1 / 1e6, 3)}}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_bench(tm, torch, n, steps, warmup, stage_reps, tag):
    """Time one lo + hi + full step at n bits (autotuned splits), each kind
    alone, squarings, and every kernel by HIP events on the launch stream.
    Raises if any guard reports a flag."""
    from paper_1703_00640_amd import inputs
    L = n // 64
    dev = torch.device("cuda:0")
    u, v = inputs.operand_pair(n, tag)
    du = torch.from_numpy(u.view(np.int64)).to(dev)
    dv = torch.from_numpy(v.view(np.int64)).to(dev)
    del u, v
    kinds = ("lo", "hi", "full")
    stream = torch.cuda.current_stream(dev)
    plans = {k: tm.autotune(k, n, stream=stream) for k in kinds}
    ws = {k: torch.empty(plans[k]["workspace_bytes"], dtype=torch.uint8, device=dev) for k in kinds}
    outs = {k: torch.empty(2 * L if k == "full" else L, dtype=torch.int64, device=dev) for k in kinds}
    guards = {k: tm.new_guard(dev) for k in kinds}

    def one(k, a=du, b=dv):
        tm.mul(k, a, b, n, out=outs[k], workspace=ws[k], stream=stream, guard=guards[k])

    def timed(fn, reps):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    for _ in range(warmup):
        for k in kinds:
            one(k)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ms_step = timed(lambda: [one(k) for k in kinds], steps)
    wall = time.perf_counter() - t_wall
    gd = {k: tm.read_guard(guards[k]).as_dict() for k in kinds}
    per = {k: timed(lambda k=k: one(k), steps) for k in kinds}
    per_sq = {k: timed(lambda k=k: one(k, du, du), steps) for k in kinds}
    # one call at a time (each bracketed by its own events): median, p10, p90
    calls = {k: [timed(lambda k=k: one(k), 1) for _ in range(steps)] for k in kinds}
    for k in kinds:
        g = tm.read_guard(guards[k])
        if g.flags or g.max_dist >= 0.25:
            raise SystemExit("guard tripped at n=%d (%s): %s" % (n, k, g.as_dict()))
    stage = {}
    for k in kinds:
        acc = {}
        for _ in range(stage_reps):
            for name, ms in tm.profile_stages(k, du, dv, n, outs[k], ws[k], stream=stream):
                acc.setdefault(name, []).append(ms)
        stage[k] = {name: float(np.median(vv)) for name, vv in acc.items()}
    nbytes = {k: kernel_bytes(plans[k], n, k) for k in kinds}
    res = {
        "n_bits": n,
        "ms_per_step": ms_step, "wall_s_timed": wall,
        "plans": {k: {x: plans[k][x] for x in ("b", "lam", "N", "L1", "Lm", "L2", "via_full")}
                  for k in kinds},
        "ms": {k: round(per[k], 5) for k in kinds},
        "mbit_s": {k: round(n / (per[k] * 1e-3) / 1e6, 1) for k in kinds},
        "ratio_lo_full": round(per["lo"] / per["full"], 4),
        "ratio_hi_full": round(per["hi"] / per["full"], 4),
        "square_ms": {k: round(per_sq[k], 5) for k in kinds},
        "call_ms": {k: {"median": round(float(np.median(calls[k])), 5),
                        "p10": round(float(np.percentile(calls[k], 10)), 5),
                        "p90": round(float(np.percentile(calls[k], 90)), 5)} for k in kinds},
        "ratio_median_lo_full": round(float(np.median(calls["lo"]) / np.median(calls["full"])), 4),
        "ratio_median_hi_full": round(float(np.median(calls["hi"]) / np.median(calls["full"])), 4),
        "stage_ms": {k: {s_: round(t, 5) for s_, t in stage[k].items()} for k in kinds},
        "stage_gb_s": {k: {nm: round(nbytes[k][nm] / (t * 1e-3) / 1e9, 1) for nm, t in stage[k].items()}
                       for k in kinds},
        "hbm_frac": {k: {nm: round(nbytes[k][nm] / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)
                         for nm, t in stage[k].items()} for k in kinds},
        "guard_max_dist": {k: gd[k]["max_dist"] for k in kinds},
        "guard_flags": {k: gd[k]["flags"] for k in kinds},
    }
    best = None
    for k in kinds:
        for name, ms in stage[k].items():
            if best is None or ms > best[2]:
                best = (k, name, ms, nbytes[k][name])
    del ws, outs, du, dv
    torch.cuda.empty_cache()
    return res, best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=30,
                    help="operand size of the timed step (default 2^30, the largest single instance)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-log2n", type=int, default=30,
                    help="operand size of the oracle timing (the benchmark size by default; "
                         "about a minute on 16 cores at 2^30)")
    ap.add_argument("--no-serve", action="store_true", help="skip the mixed-request serving runs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the n = 2^24 step, precision, small-n and mulmod sections")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="run the counter-collection workload instead of the benchmark")
    args = ap.parse_args()
    if args.pmc_pass:
        pmc_pass(1 << args.log2n, args.steps)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent products would shard by request; nothing here splits one product "
              "over several GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1703_00640_amd as tm

    n = 1 << args.log2n
    log("[bench] step at n=2^%d" % args.log2n)
    head, best = step_bench(tm, torch, n, args.steps, args.warmup, 10, 5)
    k_dom, name_dom, ms_dom, bytes_dom = best
    achieved = bytes_dom / (ms_dom * 1e-3) / 1e9
    traffic = stored_traffic(args.log2n).get("%s:%s" % (k_dom, name_dom))
    ms_step = head.pop("ms_per_step")
    wall = head.pop("wall_s_timed")
    result = {
        "metric": METRIC,
        "value": round(3 * n / (ms_step * 1e-3) / 1e6, 3),
        "unit": "operand Mbit/s (lo+hi+full step)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: uniform random limbs, PCG64 streams 10 and 11",
        "config": {"workload": "one mul_lo, mul_hi and mul_full of two n=2^%d-bit operands "
                               "(largest single instance)" % args.log2n,
                   "n_bits": n, "limbs": n // 64, "plans": head.pop("plans")},
        "roofline": {"bound": "hbm", "kernel": "%s:%s" % (k_dom, name_dom),
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": bytes_dom, "ms_per_launch": round(ms_dom, 5)},
        "source_hash": source_hash(),
        "wall_s_timed": round(wall, 3),
    }
    result.update(head)
    log("[bench] copy ceiling")
    ceil = copy_ceiling_gb_s()
    result["copy_ceiling_gb_s"] = ceil
    result["copy_frac"] = {k: {nm: round(g / ceil, 3) for nm, g in v.items()}
                           for k, v in result["stage_gb_s"].items()}
    if not args.no_extra:
        log("[bench] step at n=2^24")
        r24, _ = step_bench(tm, torch, 1 << 24, 50, 5, 20, 2)
        r24["ms_per_step"] = round(r24["ms_per_step"], 5)
        result["n2_24"] = r24
        log("[bench] precision at n=2^26")
        result["precision"] = precision_bench()
        log("[bench] small n")
        result["small_n"] = small_latency_bench()
        log("[bench] mulmod")
        result["mulmod"] = mulmod_bench()
    if not args.no_serve:
        log("[bench] serving")
        result["serving"] = serving_bench()
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        log("[bench] cpu oracle at n=2^%d on %d threads" % (args.cpu_log2n, threads))
        result["cpu_baseline"] = cpu_baseline(1 << args.cpu_log2n, threads, 1 << 24)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
