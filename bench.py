"""Benchmark of the batched homogeneous-support DFT on one MI355X.

Workload: N = 2^20, k = 2^12, one seeded homogeneous support J shared by 4096
signals (the batched single-plan configuration), complex64 samples drawn as
CN(0, k/N^2), resident in HBM before timing starts.

A step is one call of hidft_execute on the whole batch: one fused kernel that
gathers the samples, runs the s = 12 radix-2 stages, scales by N/k and stores
the coefficients in the caller's order of J.  Consecutive steps cycle through
--sets independent (input, output) buffer pairs (default 4, 1 GiB in all), so
that each launch reads samples that are no longer held in the 256 MB
last-level (Infinity) cache: the timed traffic goes to HBM.  The plan (validation, pivots,
sample set, orders, twiddles: the paper's preprocessing) is built once before
timing; its own cost is reported separately as plan_create_ms.

Prints one JSON line.  Modes for profiling runs:
  --mode copy      a plain device copy of the same byte count (counter scale)
  --mode execute   warmup + steps of the fused kernel only (no baselines)
  --mode grouped   the uneven configuration: 2048 instances with their own J
                   (N = 2^12..2^24, k = 2^6..2^14) in one grouped launch
  --mode serve     the serving configuration: Poisson arrivals (20k/s) of
                   requests over 256 supports reused Zipf(1.1), through the
                   continuous-batching server
  --mode precision the precision configuration (N = 2^22, k = 2^14, 1024
                   signals, |c| log-uniform on [1e-3, 1e3]): FP32 butterflies
                   against the FP16 / BF16 split-precision matrix-core group
                   (radix-16 and radix-32 first groups)
  --mode inverse   the inverse map (coefficients -> samples) on the headline
                   workload's shape
  --mode sas       Shift-and-Sample on a random half of a homogeneous set
  --mode gap       GAP and arithmetic-progression supports through
                   Shift-and-Sample
  --mode large     transforms of 2^15..2^22 points (N = 2^24), which run in
                   passes through a workspace
The full run also reports the autotuned variant of the headline workload
(hidft_autotune, then hidft_execute_config with the tuned variant).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "transforms/s and HBM GB/s vs plain GPU path at rel-L2≤1e-5; p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
WORKLOAD = dict(workload="batched single plan: N=2^20, k=2^12, 4096 signals, complex64",
                N=1 << 20, log2_n=20, k=1 << 12, batch=4096, support="seeded homogeneous J")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "hidft_fused_k4096_b4096_counters.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2211_15299_amd", "csrc", "kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--mode", choices=["full", "execute", "copy", "grouped", "serve", "precision",
                                       "inverse", "sas", "gap", "large"],
                    default="full")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="duration of the Poisson arrival process (serving)")
    ap.add_argument("--serve-rate", type=float, default=20000.0, help="arrivals per second")
    ap.add_argument("--no-serve-sweep", action="store_true",
                    help="serving: skip the load curve after the --serve-rate run")
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="signals the oracle runs for cpu_baseline (default: the whole batch)")
    ap.add_argument("--plain-signals", type=int, default=4096,
                    help="signals timed on the plain per-signal path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--sets", type=int, default=4,
                    help="buffer pairs cycled through by consecutive steps (1 = same buffers)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def load_traffic(launch_bytes_alg):
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current kernel source (else None)."""
    try:
        with open(COUNTERS_FILE) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return c.get("traffic_bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the batched "
              "transform shards by splitting the batch across GPUs with no exchange; "
              "this benchmark runs on one GPU.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2211_15299_amd import native
    from workloads import homogeneous_support, rng_for, sample_values

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    M, k, batch = WORKLOAD["log2_n"], WORKLOAD["k"], WORKLOAD["batch"]
    rng = rng_for(2, 0)
    sup = homogeneous_support(M, k.bit_length() - 1, rng)
    J = sup.J.tolist()
    f_host = sample_values(M, k, batch, rng)
    x = torch.from_numpy(f_host).to(dev)
    y = torch.empty_like(x)
    xs = [x] + [x.clone() for _ in range(args.sets - 1)]
    ys = [y] + [torch.empty_like(x) for _ in range(args.sets - 1)]
    bytes_per_launch = batch * k * 16  # read 8 B + write 8 B per point

    if args.mode == "copy":
        # Plain copy of the same number of bytes, for counter calibration.
        for i in range(args.warmup):
            ys[i % args.sets].copy_(xs[i % args.sets])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.steps):
            ys[i % args.sets].copy_(xs[i % args.sets])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        print(json.dumps({"mode": "copy", "sets": args.sets, "bytes_per_launch": bytes_per_launch,
                          "ms_per_copy": ms, "GBps": bytes_per_launch / ms / 1e6}), flush=True)
        return

    if args.mode == "grouped":
        del xs, ys, x, y
        print(json.dumps(grouped_bench(args, native, torch, stream)), flush=True)
        return
    if args.mode == "serve":
        del xs, ys, x, y
        print(json.dumps(serve_bench(args, native)), flush=True)
        return
    if args.mode == "precision":
        del xs, ys, x, y
        print(json.dumps(precision_bench(args, native, torch, stream)), flush=True)
        return
    if args.mode in ("inverse", "sas", "gap", "large"):
        del xs, ys, x, y
        if args.mode == "inverse":
            r = inverse_bench(args, native, torch, stream, steps=args.steps)
        elif args.mode == "large":
            r = large_bench(native, torch, stream, steps=args.steps)
        elif args.mode == "sas":
            r = sas_bench(native, torch, stream, steps=args.steps)
        else:
            r = gap_bench(native, torch, stream, steps=args.steps)
        print(json.dumps(r), flush=True)
        return

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = native.Plan(M, J, stream=stream)
    plan_ms = (time.perf_counter() - t0) * 1e3
    # plan creation cost, steady state (tables re-derived and re-uploaded)
    t0 = time.perf_counter()
    n_rep = 20
    for _ in range(n_rep):
        native.Plan(M, J, stream=stream).close()
    plan_ms_steady = (time.perf_counter() - t0) * 1e3 / n_rep

    def step(i):
        j = i % args.sets
        plan.execute_ptr(xs[j].data_ptr(), k, ys[j].data_ptr(), k, batch, stream)

    for i in range(args.warmup):
        step(i)
    # Throughput: K back-to-back launches between two events on the launch stream.
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    g0.record(stream)
    for i in range(args.steps):
        step(i)
    g1.record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - wall0
    total_ms = g0.elapsed_time(g1)
    ms_per_step = total_ms / args.steps
    kernel_ms = ms_per_step  # one kernel launch per step
    # Latency: each launch between its own pair of events (a separate loop).
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for i in range(args.steps):
        starts[i].record(stream)
        step(i)
        ends[i].record(stream)
    torch.cuda.synchronize()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    transforms_per_s = batch / (ms_per_step * 1e-3)
    achieved_gbps = bytes_per_launch / (kernel_ms * 1e-3) / 1e9

    result = {
        "metric": METRIC,
        "value": transforms_per_s,
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded homogeneous J; CN(0,k/N^2) complex64 samples)",
        "config": dict(WORKLOAD, buffer_sets=args.sets),
        "hbm_GBps": bytes_per_launch / (ms_per_step * 1e-3) / 1e9,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "one launch (4096 transforms) between its own pair of events"},
        "plan_create_ms": {"first": plan_ms, "steady": plan_ms_steady},
        "wall_s_timed": wall_s,
        "roofline": {
            "bound": "hbm",
            "kernel": "hidft_fused_kernel<12, 0, 4, 0, false>",
            "achieved": achieved_gbps,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved_gbps / HBM_PEAK_GBPS,
            "traffic": load_traffic(bytes_per_launch),
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": kernel_ms,
        },
    }
    if args.mode == "execute":
        print(json.dumps(result), flush=True)
        return

    # Plain per-signal GPU method (baseline of the metric): one launch per signal.
    n_plain = min(args.plain_signals, batch)
    yp = torch.empty_like(x)
    plan.execute_ptr(x.data_ptr(), k, yp.data_ptr(), k, min(n_plain, 64), stream, plain=True)
    torch.cuda.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    plan.execute_ptr(x.data_ptr(), k, yp.data_ptr(), k, n_plain, stream, plain=True)
    p1.record(stream)
    torch.cuda.synchronize()
    plain_ms = p0.elapsed_time(p1)
    plain_tps = n_plain / (plain_ms * 1e-3)
    same = torch.equal(yp[:n_plain], y[:n_plain])
    diff = (yp[:n_plain] - y[:n_plain]).abs().max().item()
    result["plain_gpu"] = {
        "value": plain_tps, "unit": "transforms/s", "signals": n_plain,
        "ms_total": plain_ms, "HBM_GBps": n_plain * k * 16 / (plain_ms * 1e-3) / 1e9,
        "max_abs_diff_vs_fused": diff, "bitwise_equal_to_fused": bool(same),
    }
    result["speedup_vs_plain"] = transforms_per_s / plain_tps

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(M, J, f_host, y, args.cpu_sample)

    # The autotuner on the same workload: search, then the tuned variant timed
    # like the headline loop.
    tuned = native.ExecConfig(native.PREC_FP32, native.SCHED_TUNED, 0, 0)
    t0 = time.perf_counter()
    best, best_us = plan.autotune_ptr(xs[-1].data_ptr(), k, ys[-1].data_ptr(), k, batch,
                                      reps=10, stream=stream)
    search_s = time.perf_counter() - t0
    for i in range(args.warmup):
        j = i % args.sets
        plan.execute_ptr(xs[j].data_ptr(), k, ys[j].data_ptr(), k, batch, stream, config=tuned)
    torch.cuda.synchronize()
    g0.record(stream)
    for i in range(args.steps):
        j = i % args.sets
        plan.execute_ptr(xs[j].data_ptr(), k, ys[j].data_ptr(), k, batch, stream, config=tuned)
    g1.record(stream)
    torch.cuda.synchronize()
    tuned_ms = g0.elapsed_time(g1) / args.steps
    result["autotuned"] = {
        "config": {"precision": best.precision, "schedule": best.schedule, "radix": best.radix,
                   "blocks_per_cu": best.blocks_per_cu},
        "search_us_per_launch": best_us, "search_s": search_s,
        "ms_per_step": tuned_ms, "transforms_per_s": batch / (tuned_ms * 1e-3),
        "hbm_GBps": bytes_per_launch / (tuned_ms * 1e-3) / 1e9,
    }
    plan.close()
    del xs, ys, x, y, yp
    torch.cuda.empty_cache()
    # The other configurations, reported beside the headline (not the metric):
    # the uneven batch in one grouped launch, and Poisson-arrival serving.
    gsteps = args.steps
    args.steps, args.warmup = 20, 3
    result["config1_single_signal"] = single_signal_bench(native, torch, stream)
    result["config3_grouped"] = grouped_bench(args, native, torch, stream)
    args.steps = gsteps
    result["config5_serving"] = serve_bench(args, native)
    result["config4_precision"] = precision_bench(args, native, torch, stream, steps=20)
    result["gap_supports"] = gap_bench(native, torch, stream)
    result["inverse"] = inverse_bench(args, native, torch, stream)
    result["shift_and_sample"] = sas_bench(native, torch, stream)
    result["large"] = large_bench(native, torch, stream)
    if not args.no_cpu:
        result["cpu_baseline"]["precision_vs_oracle"] = precision_vs_oracle(native, torch, stream)
    print(json.dumps(result), flush=True)


def grouped_instances(n):
    """(M, J) of the uneven configuration (workloads.uneven_instances): N
    log-uniform over 2^12..2^24 and k over 2^6..2^14 with k <= N/4, each with
    its own seeded J, the first 64 direct sums of homogeneous blocks."""
    from workloads import uneven_instances
    return [(M, sup.J.tolist()) for M, sup in uneven_instances(n)]


def grouped_bench(args, native, torch, stream):
    """Throughput of one grouped launch over 2048 uneven instances."""
    from workloads import rng_for, sample_values
    insts = grouped_instances(2048)
    rng = rng_for(3, 99999)
    plans = [native.Plan(M, J, stream=stream) for M, J in insts]
    ks = np.array([p.k for p in plans], dtype=np.int64)
    total = int(ks.sum())
    offs = np.concatenate([[0], np.cumsum(ks)])
    host = np.concatenate([sample_values(M, len(J), 1, rng)[0] for M, J in insts])
    sets = max(args.sets, 1)
    xs = [torch.from_numpy(host).cuda()] + []
    xs += [xs[0].clone() for _ in range(sets - 1)]
    ys = [torch.empty_like(xs[0]) for _ in range(sets)]
    groups = []
    for j in range(sets):
        items = [(p, xs[j].data_ptr() + 8 * int(offs[i]), p.k, ys[j].data_ptr() + 8 * int(offs[i]),
                  p.k, 1) for i, p in enumerate(plans)]
        groups.append(native.Group(items, stream=stream))
    for i in range(args.warmup):
        groups[i % sets].execute(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        groups[i % sets].execute(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    byts = total * 16
    # Per-instance plans: the minimum plan input is J as uint32 (4 B per
    # point); the tables the kernel actually reads are the twiddles and the
    # gather positions (8 (k - 1) + 2 k B per instance).
    table_bytes = int(sum(8 * (kk - 1) + 2 * kk for kk in ks.tolist()))
    out = {"mode": "grouped", "instances": len(plans), "points": total, "packs": groups[0].n_packs,
           "k_min": int(ks.min()), "k_max": int(ks.max()), "ms_per_launch": ms,
           "transforms_per_s": len(plans) / (ms * 1e-3), "GBps": byts / (ms * 1e-3) / 1e9,
           "GBps_data_plus_plan": (byts + 4 * total) / (ms * 1e-3) / 1e9,
           "table_bytes_per_launch": table_bytes,
           "frac_of_8TBps": byts / (ms * 1e-3) / 8e12, "sets": sets}
    # The group autotuner (schedule and pack order), then the tuned launch
    # timed like the default one.
    t0 = time.perf_counter()
    cfg, tune_us = groups[0].autotune(reps=10, stream=stream)
    search_s = time.perf_counter() - t0
    for g in groups[1:]:
        g.set_config(cfg.schedule, cfg.order, stream)
    for i in range(args.warmup):
        groups[i % sets].execute(stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(args.steps):
        groups[i % sets].execute(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    tms = e0.elapsed_time(e1) / args.steps
    out["autotuned"] = {"schedule": cfg.schedule, "order": cfg.order, "search_s": search_s,
                        "search_us_per_launch": tune_us, "ms_per_launch": tms,
                        "transforms_per_s": len(plans) / (tms * 1e-3),
                        "GBps": byts / (tms * 1e-3) / 1e9}
    return out


SERVE_SWEEP_RATES = (20000.0, 50000.0, 100000.0, 200000.0, 500000.0, 1000000.0, 2000000.0)


def _serve_supports():
    """256 supports (M uniform on 10..22, s uniform on 6..13 with s <= M-2)
    and one sample vector per support."""
    from workloads import homogeneous_support, rng_for, sample_values
    sups, vecs = [], []
    for i in range(256):
        rng = rng_for(5, i)
        M = int(rng.integers(10, 23))
        s = int(rng.integers(6, min(13, M - 2) + 1))
        sup = homogeneous_support(M, s, rng)
        sups.append((M, np.ascontiguousarray(sup.J, dtype=np.uint64)))
        vecs.append(sample_values(M, len(sup.J), 1, rng)[0])
    return sups, vecs


def serve_run(native, srv, sups, vecs, rate, seconds, seed):
    """Poisson arrivals at `rate` requests/s for `seconds`, supports drawn by
    a Zipf(1.1) law over their rank.  Requests whose arrival time has passed
    go to the server in one hidft_server_submit_many call; results are
    polled between bursts.  Latency is the server's (submit to coefficients
    in the request's host buffer); the client's own lag behind the arrival
    times is reported beside it."""
    from workloads import rng_for
    rng = rng_for(5, seed)
    n = max(1, int(rate * seconds))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    pz = np.arange(1, 257, dtype=np.float64) ** -1.1
    which = rng.choice(256, size=n, p=pz / pz.sum())
    pool_n, width = 4096, 1 << 13
    pool = np.zeros((pool_n, width), dtype=np.complex64)
    recs = np.zeros(n, dtype=native.REQUEST_DTYPE)
    recs["log2_n"] = np.array([M for M, _ in sups], dtype=np.uint32)[which]
    recs["J"] = np.array([J.ctypes.data for _, J in sups], dtype=np.uint64)[which]
    ks = np.array([len(J) for _, J in sups], dtype=np.uint64)[which]
    recs["k"] = ks
    recs["host_samples"] = np.array([v.ctypes.data for v in vecs], dtype=np.uint64)[which]
    recs["host_coefs"] = (pool.ctypes.data + (np.arange(n) % pool_n) * width * 8).astype(np.uint64)
    done = np.zeros(n, dtype=bool)
    idx_of_rank = np.zeros(n, dtype=np.int64)
    lat, bsz = [], []
    state = {"id0": None, "rank": 0, "rejected": 0, "failed": 0, "lag": 0.0,
             "submit_s": 0.0, "poll_s": 0.0}

    def collect(wait_us=0):
        tp = time.perf_counter()
        res = srv.poll(wait_us)
        state["poll_s"] += time.perf_counter() - tp
        if len(res):
            r = (res["id"].astype(np.int64) - state["id0"])
            done[idx_of_rank[r]] = True
            ok = res["status"] == 0
            state["failed"] += int((~ok).sum())
            lat.append(res["latency_us"][ok])
            bsz.append(res["batch_size"][ok])
        return len(res)

    st0 = srv.stats()
    t0 = time.perf_counter()
    i = 0
    while i < n:
        now = time.perf_counter() - t0
        j = int(np.searchsorted(arrivals, now, side="right"))
        j = min(j, i + 4096)
        if j > pool_n:  # request x reuses the buffer of request x - pool_n
            lo = max(i - pool_n, 0)
            seg = done[lo: j - pool_n]
            if not seg.all():
                j = lo + int(np.argmin(seg)) + pool_n
        if j > i:
            ts = time.perf_counter()
            ids, sts = srv.submit_many(recs[i:j])
            state["submit_s"] += time.perf_counter() - ts
            acc = sts == 0
            if state["id0"] is None and acc.any():
                state["id0"] = int(ids[acc][0])
            na = int(acc.sum())
            idx_of_rank[state["rank"]: state["rank"] + na] = np.arange(i, j)[acc]
            state["rank"] += na
            done[np.arange(i, j)[~acc]] = True
            state["rejected"] += j - i - na
            state["lag"] = max(state["lag"], now - arrivals[i])
            i = j
        collect()
    srv.drain()
    wall = time.perf_counter() - t0
    while collect():
        pass
    st = srv.stats()
    lat = np.concatenate(lat) if lat else np.zeros(1)
    bsz = np.concatenate(bsz) if bsz else np.zeros(1)
    return {"offered_per_s": rate, "requests": n, "seconds": seconds,
            "completed": int(st["completed"] - st0["completed"]),
            "rejected": state["rejected"], "failed": state["failed"],
            "transforms_per_s": n / wall, "wall_s": wall,
            "data_GBps": float(ks.sum()) * 16 / wall / 1e9,
            "latency_us": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean()), "max": float(lat.max())},
            "batch_size_mean": float(bsz.mean()), "batches": int(st["batches"] - st0["batches"]),
            "max_client_lag_us": state["lag"] * 1e6,
            "client_time_s": {"submit_many": state["submit_s"], "poll": state["poll_s"]}}


def serve_bench(args, native, seconds=None):
    """The serving configuration through the continuous-batching server:
    Poisson arrivals at --serve-rate (20 000 requests/s) for --serve-seconds
    over 256 supports reused Zipf(1.1), then a load curve (2 s per rate) up
    to 2 * 10^6 requests/s.  Plans are made resident before the clock starts
    (their creation is timed separately)."""
    seconds = args.serve_seconds if seconds is None else seconds
    sups, vecs = _serve_supports()
    srv = native.Server(data_bytes=512 << 20, plan_bytes=256 << 20, slots=4, max_batch=1024)
    warm = np.zeros(1 << 13, dtype=np.complex64)
    t0 = time.perf_counter()
    for (M, J), f in zip(sups, vecs):  # make every plan resident
        srv.submit(M, J, f, warm[:len(J)])
        srv.drain()
    srv.poll()
    plan_warm_s = time.perf_counter() - t0
    st = srv.stats()
    out = serve_run(native, srv, sups, vecs, args.serve_rate, seconds, 10 ** 6)
    out.update({"mode": "serve", "rate_per_s": args.serve_rate, "supports": 256, "zipf": 1.1,
                "plan_warmup_s": plan_warm_s, "plans_resident": int(st["plans_resident"]),
                "plan_bytes_resident": int(st["plan_bytes_resident"])})
    curve = []
    for q, rate in enumerate(() if args.no_serve_sweep else SERVE_SWEEP_RATES):
        r = serve_run(native, srv, sups, vecs, rate, 2.0, 2 * 10 ** 6 + q)
        curve.append({k: r[k] for k in ("offered_per_s", "transforms_per_s", "completed",
                                        "rejected", "failed", "latency_us", "batch_size_mean",
                                        "data_GBps", "max_client_lag_us", "wall_s",
                                        "client_time_s")})
        print(f"serve sweep: offered {rate:.0f}/s sustained {r['transforms_per_s']:.0f}/s "
              f"p50 {r['latency_us']['p50']:.1f} us p99 {r['latency_us']['p99']:.1f} us "
              f"batch {r['batch_size_mean']:.1f}", file=sys.stderr, flush=True)
    out["load_curve"] = curve
    st = srv.stats()
    out["max_inflight_batches"] = int(st["max_inflight_batches"])
    srv.close()
    return out


PRECISION_WORKLOAD = dict(workload="precision: N=2^22, k=2^14, 1024 signals, |c| log-uniform "
                                   "on [1e-3, 1e3] with random phase", log2_n=22, log2_k=14,
                          batch=1024)


def single_signal_bench(native, torch, stream, reps=500):
    """The single-signal configuration: N = 2^10, k = 64, an elementary
    homogeneous J (a seeded odd dilation and translation of {0..63}) and one
    signal of seeded samples.  Latency of one transform per launch, fused
    kernel and plain kernel, each launch between its own pair of events; the
    two results must agree bit for bit (their accuracy against the oracle is
    the single-signal parity test's)."""
    from workloads import elementary_support, rng_for, sample_values
    rng = rng_for(1, 0)
    M, s = 10, 6
    plan = native.Plan(M, elementary_support(M, s, rng).J.tolist(), stream=stream)
    k = plan.k
    x = torch.from_numpy(sample_values(M, k, 1, rng)).cuda()
    out = {"workload": "single signal: N=2^10, k=64, elementary J", "reps": reps}
    res = {}
    for name, plain in (("fused", False), ("plain", True)):
        y = torch.empty_like(x)
        for _ in range(20):
            plan.execute_ptr(x.data_ptr(), k, y.data_ptr(), k, 1, stream, plain=plain)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            plan.execute_ptr(x.data_ptr(), k, y.data_ptr(), k, 1, stream, plain=plain)
            b.record(stream)
        torch.cuda.synchronize()
        lat = np.array([a.elapsed_time(b) for a, b in ev]) * 1e3
        out[name] = {"latency_us": {"p50": float(np.percentile(lat, 50)),
                                    "p99": float(np.percentile(lat, 99))}}
        res[name] = y
    out["fused_equals_plain"] = bool(torch.equal(res["fused"], res["plain"]))
    plan.close()
    return out


def precision_variants(native):
    """(name, precision, radix) of the group-1 arithmetics compared on the
    precision workload: FP32 butterflies and the two matrix-core splits, with
    a radix-16 and a radix-32 first group."""
    return (("fp32", native.PREC_FP32, 16), ("f16x2", native.PREC_F16X2, 16),
            ("bf16x3", native.PREC_BF16X3, 16), ("fp32_r32", native.PREC_FP32, 32),
            ("f16x2_r32", native.PREC_F16X2, 32), ("bf16x3_r32", native.PREC_BF16X3, 32))


def _precision_setup(native, stream):
    from workloads import homogeneous_support, rng_for
    rng = rng_for(4, 0)
    M, s = PRECISION_WORKLOAD["log2_n"], PRECISION_WORKLOAD["log2_k"]
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    return M, J, native.Plan(M, J, stream=stream), rng


def precision_bench(args, native, torch, stream, steps=None):
    """Launch time of each precision of group 1 on the precision workload.

    Samples of the workload's magnitude: per signal, CN(0, 1) scaled by
    10^U(-3, 3) sqrt(k) / N (the size of samples of coefficients with that
    spread).  Reports the FP32 path and the two split-precision matrix-core
    paths, and how far each result is from the FP32 one.
    """
    from workloads import complex_normal
    M, J, plan, rng = _precision_setup(native, stream)
    k, batch, N = plan.k, PRECISION_WORKLOAD["batch"], float(1 << M)
    f = complex_normal((batch, k), rng) * (10.0 ** rng.uniform(-3, 3, (batch, 1))) * np.sqrt(k) / N
    sets = max(args.sets, 1)
    xs = [torch.from_numpy(f.astype(np.complex64)).cuda()]
    xs += [xs[0].clone() for _ in range(sets - 1)]
    ys = [torch.empty_like(xs[0]) for _ in range(sets)]
    steps = steps or args.steps
    out = {"config": PRECISION_WORKLOAD, "sets": sets, "steps": steps}
    ref = None
    for name, prec, radix in precision_variants(native):
        cfg = native.ExecConfig(prec, native.SCHED_DEFAULT, radix, 0)
        for i in range(3):
            plan.execute_ptr(xs[i % sets].data_ptr(), k, ys[i % sets].data_ptr(), k, batch,
                             stream, config=cfg)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            plan.execute_ptr(xs[i % sets].data_ptr(), k, ys[i % sets].data_ptr(), k, batch,
                             stream, config=cfg)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        plan.execute_ptr(xs[0].data_ptr(), k, ys[0].data_ptr(), k, batch, stream, config=cfg)
        torch.cuda.synchronize()
        y = ys[0].cpu().numpy().astype(np.complex128)
        entry = {"ms_per_launch": ms, "transforms_per_s": batch / (ms * 1e-3),
                 "GBps": batch * k * 16 / (ms * 1e-3) / 1e9}
        if ref is None:
            ref = y
        else:
            d = np.linalg.norm(y - ref, axis=1) / np.linalg.norm(ref, axis=1)
            entry["rel_l2_vs_fp32"] = {"max": float(d.max()), "median": float(np.median(d))}
        out[name] = entry
    plan.close()
    del xs, ys
    torch.cuda.empty_cache()
    return out


def precision_vs_oracle(native, torch, stream, n_exact=8):
    """Per-instance error of each precision against the FP64 oracle on the
    precision workload: n_exact signals synthesised by the oracle from seeded
    coefficients (log-uniform magnitudes, random phase)."""
    import oracle
    from workloads import log_uniform_coefficients
    M, J, plan, rng = _precision_setup(native, stream)
    k = plan.k
    c = log_uniform_coefficients((n_exact, k), rng)
    t0 = time.perf_counter()
    f = oracle.synthesize_samples_fft(M, J, c, plan.samples().tolist())
    synth_s = time.perf_counter() - t0
    x = torch.from_numpy(f.astype(np.complex64)).cuda()
    out = {"instances": n_exact, "synthesis": "oracle.synthesize_samples_fft (FP64)",
           "synthesis_s": synth_s}
    for name, prec, radix in precision_variants(native):
        y = plan.execute(x, config=native.ExecConfig(prec, native.SCHED_DEFAULT, radix, 0),
                         stream=stream)
        torch.cuda.synchronize()
        got = y.cpu().numpy().astype(np.complex128)
        err = oracle.rel_l2(got, c)
        mabs = oracle.max_abs(got, c)
        out[name] = {"rel_l2": [float(e) for e in err], "rel_l2_max": float(err.max()),
                     "max_abs": [float(a) for a in mabs], "max_abs_rel_to_max_coef":
                     float(np.max(mabs / np.max(np.abs(c), axis=1)))}
    plan.close()
    return out


def inverse_bench(args, native, torch, stream, steps=50):
    """The inverse map (coefficients on J -> samples on I_r) on the headline
    workload's shape: N = 2^20, k = 2^12, 4096 signals, rotating buffers."""
    from workloads import complex_normal, homogeneous_support, rng_for
    M, k, batch = WORKLOAD["log2_n"], WORKLOAD["k"], WORKLOAD["batch"]
    rng = rng_for(2, 0)
    J = homogeneous_support(M, k.bit_length() - 1, rng).J.tolist()
    plan = native.Plan(M, J, stream=stream)
    sets = max(args.sets, 1)
    cs = [torch.from_numpy(complex_normal((batch, k), rng).astype(np.complex64)).cuda()]
    cs += [cs[0].clone() for _ in range(sets - 1)]
    fs = [torch.empty_like(cs[0]) for _ in range(sets)]
    for i in range(5):
        plan.inverse_ptr(cs[i % sets].data_ptr(), k, fs[i % sets].data_ptr(), k, batch, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        plan.inverse_ptr(cs[i % sets].data_ptr(), k, fs[i % sets].data_ptr(), k, batch, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # round trip on one set: forward(inverse(c)) = c
    back = torch.empty_like(cs[0])
    plan.inverse_ptr(cs[0].data_ptr(), k, fs[0].data_ptr(), k, batch, stream)
    plan.execute_ptr(fs[0].data_ptr(), k, back.data_ptr(), k, batch, stream)
    torch.cuda.synchronize()
    rt = ((back - cs[0]).abs().pow(2).sum(1).sqrt() / cs[0].abs().pow(2).sum(1).sqrt()).max().item()
    plan.close()
    del cs, fs, back
    torch.cuda.empty_cache()
    return {"workload": "N=2^20, k=2^12, 4096 signals", "ms_per_launch": ms,
            "transforms_per_s": batch / (ms * 1e-3), "GBps": batch * k * 16 / (ms * 1e-3) / 1e9,
            "round_trip_rel_l2_max": rt, "steps": steps, "sets": sets}


def large_bench(native, torch, stream, steps=50):
    """Transforms of 2^15..2^22 points at N = 2^24, 256 MB of samples and
    coefficients per launch, 4 rotating (input, output) sets and one shared
    workspace (hidft_execute_ws: three passes, no allocation).  GB/s counts
    the algorithmic 16 B per point; the passes move about 48 (each reads and
    writes the signal once, the last reads it in gather order)."""
    from workloads import homogeneous_support, rng_for, sample_values
    M = 24
    out = {"workload": "N=2^24, k=2^15..2^22, 256 MB per launch", "steps": steps}
    for s in range(15, 23):
        rng = rng_for(24, s)
        plan = native.Plan(M, homogeneous_support(M, s, rng).J.tolist(), stream=stream)
        k = plan.k
        batch = (256 << 20) // (16 * k)
        sets = ROTATE_SETS
        xs = [torch.from_numpy(sample_values(M, k, batch, rng)).cuda()]
        xs += [xs[0].clone() for _ in range(sets - 1)]
        ys = [torch.empty_like(xs[0]) for _ in range(sets)]
        wb = plan.workspace_bytes(batch)
        work = torch.empty(wb // 8, dtype=torch.complex64, device="cuda")

        def run(i):
            plan.execute_ws_ptr(xs[i % sets].data_ptr(), k, ys[i % sets].data_ptr(), k, batch,
                                work.data_ptr(), wb, stream)

        for i in range(3):
            run(i)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            run(i)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps

        def run_inv(i):  # coefficients -> samples, the adjoint passes
            plan.inverse_ws_ptr(ys[i % sets].data_ptr(), k, xs[i % sets].data_ptr(), k, batch,
                                work.data_ptr(), wb, stream)

        for i in range(3):
            run_inv(i)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(steps):
            run_inv(i)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_inv = e0.elapsed_time(e1) / steps
        out[f"k=2^{s}"] = {"batch": batch, "ms_per_launch": ms,
                           "transforms_per_s": batch / (ms * 1e-3),
                           "GBps": batch * k * 16 / (ms * 1e-3) / 1e9,
                           "inverse_ms_per_launch": ms_inv}
        plan.close()
        del xs, ys, work
        torch.cuda.empty_cache()
    return out


ROTATE_SETS = 4               # input/output buffer sets cycled through by a leg
ROTATE_INPUT_BYTES = 128 << 20  # input bytes per set: 4 sets exceed the 256 MB cache


def _rotating_sas_run(native, torch, stream, plan, batch, rng, steps):
    """Times plan.execute over ROTATE_SETS (input, output) pairs; the
    workspace is shared.  Returns ms per launch and the buffers of set 0."""
    from workloads import sample_values
    n_in = plan.samples_per_signal
    x0 = torch.from_numpy(sample_values(20, n_in, batch, rng).astype(np.complex64)).cuda()
    xs = [x0] + [x0.clone() for _ in range(ROTATE_SETS - 1)]
    ys = [torch.empty((batch, plan.k), dtype=torch.complex64, device="cuda")
          for _ in range(ROTATE_SETS)]
    work = torch.empty(max(plan.workspace_bytes(batch) // 8, 1), dtype=torch.complex64,
                       device="cuda")

    def run(i):
        j = i % ROTATE_SETS
        plan.execute_ptr(xs[j].data_ptr(), n_in, ys[j].data_ptr(), plan.k, batch,
                         work.data_ptr(), stream)

    for i in range(2 * ROTATE_SETS):
        run(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        run(i)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del xs, ys, work
    torch.cuda.empty_cache()
    return ms


def _sas_rates(plan, batch, ms):
    """Rates of a Shift-and-Sample launch: data (samples in, coefficients out)
    and data plus the workspace (the mu* shifted Hi-DFT outputs, written by
    the fused kernel and read by the leaf solves)."""
    n_in = plan.samples_per_signal
    data = batch * (n_in + plan.k) * 8
    work = 2 * plan.workspace_bytes(batch)
    return {"ms_per_launch": ms, "transforms_per_s": batch / (ms * 1e-3),
            "GBps": data / (ms * 1e-3) / 1e9,
            "GBps_with_workspace": (data + work) / (ms * 1e-3) / 1e9}


def sas_bench(native, torch, stream, steps=20, two_pass=False):
    """Shift-and-Sample on a random half of a homogeneous set (N = 2^20, 2^12
    candidate positions, 2048 elements kept), r chosen by Lemma 4's cost: the
    mu* shifted Hi-DFTs and the FP64 leaf solves (one kernel for this plan;
    two launches through a workspace with two_pass).  4096 signals per
    launch, 4 rotating buffer sets."""
    from workloads import homogeneous_support, rng_for
    rng = rng_for(941, 0)
    K = homogeneous_support(20, 12, rng)
    keep = rng.random(len(K.J)) < 0.5
    J = [int(j) for j, kp in zip(K.J, keep) if kp]
    plan = native.SASPlan(20, J, stream=stream, two_pass=two_pass)
    batch = 4096
    ms = _rotating_sas_run(native, torch, stream, plan, batch, rng, steps)
    out = {"k": plan.k, "r": plan.pivots(), "mu_star": plan.mu_max, "nodes": plan.n_nodes,
           "samples_per_transform": plan.samples_per_signal, "lemma4_cost": plan.cost,
           "one_kernel": plan.workspace_bytes(batch) == 0,
           "batch": batch, "sets": ROTATE_SETS, **_sas_rates(plan, batch, ms)}
    plan.close()
    if not two_pass:
        out["two_pass"] = {k: v for k, v in sas_bench(native, torch, stream, steps, True).items()
                           if k in ("ms_per_launch", "transforms_per_s", "GBps",
                                    "GBps_with_workspace")}
    return out


def gap_bench(native, torch, stream, steps=20):
    """Supports with additive structure: a proper 2-dimensional GAP (16 x 16
    terms) and an arithmetic progression (1000 terms, difference 2^5 odd) in
    Z_{2^20}, through Shift-and-Sample with r = all pivots (Lemma 5: 2^n
    samples, mu* = 1) and with Lemma 4's choice of r.  The batch holds 128 MiB
    of samples, 4 rotating buffer sets."""
    from workloads import arithmetic_progression, gap_support, rng_for
    out = {"steps": steps, "sets": ROTATE_SETS}
    cases = {"gap_16x16": gap_support(20, [16, 16], rng_for(940, 0)),
             "ap_1000_alpha5": arithmetic_progression(20, 1000, rng_for(940, 1), 5)}
    for name, sup in cases.items():
        J = sup.J.tolist()
        P, _ = native.analyze(20, J)
        for label, piv in (("all_pivots", P), ("lemma4_r", None)):
            plan = native.SASPlan(20, J, pivots=piv, stream=stream)
            n_in = plan.samples_per_signal
            batch = max(1, ROTATE_INPUT_BYTES // (8 * n_in))
            ms = _rotating_sas_run(native, torch, stream, plan, batch, rng_for(940, 2), steps)
            out[f"{name}/{label}"] = {
                "k": plan.k, "pivots_of_J": len(P), "r": plan.pivots(), "mu_star": plan.mu_max,
                "samples_per_transform": n_in, "batch": batch, **_sas_rates(plan, batch, ms)}
            plan.close()
    return out


def cpu_baseline(M, J, f_host, y_dev, n_sample):
    """The FP64 oracle, as it stands, on the same batch (by default all of it).

    Times oracle.coefficients (dense LU solve of F^{-1}(I_r, J) c = f_I for
    k = 4096, factorisation included) on the first n_sample signals, and
    reports the GPU result's error against those oracle outputs: every
    coefficient of every signal at the default n_sample.
    """
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        threads = len(os.sched_getaffinity(0))
    f = f_host[:n_sample].astype(np.complex128)
    t0 = time.perf_counter()
    c = oracle.coefficients(M, J, f)
    dt = time.perf_counter() - t0
    got = y_dev[:n_sample].cpu().numpy().astype(np.complex128)
    err = oracle.rel_l2(got, c)
    # The oracle's other route on the same sample: c = (N/k) F(J, I_r) f_I.
    t0 = time.perf_counter()
    ca = oracle.coefficients(M, J, f, method="adjoint")
    dta = time.perf_counter() - t0
    return {
        "value": n_sample / dt, "unit": "transforms/s", "cores": int(threads), "kind": "oracle",
        "sample": f"first {n_sample} of the {f_host.shape[0]} signals; oracle.coefficients (LU route, "
                  f"factorisation included), {dt:.1f} s",
        "seconds": dt,
        "adjoint_route": {"value": n_sample / dta, "unit": "transforms/s", "seconds": dta,
                          "rel_l2_vs_lu_max": float(np.max(oracle.rel_l2(ca, c)))},
        "config1_single_thread": oracle_config1_single_thread(oracle),
        "gpu_rel_l2_vs_oracle": {"max": float(np.max(err)), "mean": float(np.mean(err))},
        "gpu_max_abs_vs_oracle": float(np.max(np.abs(got - c))),
    }


def oracle_config1_single_thread(oracle, seconds=1.0):
    """The oracle on the single-signal configuration (N = 2^10, k = 64, an
    odd dilation and translation of {0..63}), one signal per call, one BLAS
    thread: transforms/s."""
    from workloads import elementary_support, rng_for, sample_values
    rng = rng_for(1, 0)
    J = elementary_support(10, 6, rng).J.tolist()
    f = sample_values(10, len(J), 64, rng).astype(np.complex128)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            oracle.coefficients(10, J, f[n % 64:n % 64 + 1])
            n += 1
        dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "transforms/s", "threads": 1, "calls": n,
            "route": "LU (factorisation per call)"}


if __name__ == "__main__":
    main()
