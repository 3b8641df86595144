#!/usr/bin/env python3
"""Throughput of SciFi Seeding + VELO-SciFi Matching on one MI355X.

A step is one pass of the whole path (XZ seeding, clone vote, UV seeding,
matching, output compaction) over one batch of 1000 synthetic min-bias-like
events already resident in HBM.  `value` is events/s of the batched form
(one captured graph of persistent kernels per batch, host sync included);
the plain form (one kernel sequence per event) is timed beside it.  Outputs
are checked against the FP64 oracle before timing; the per-kernel roofline
of the seeding kernel comes from HIP events recorded around it on its stream.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
SERVE_SLOTS = 4   # serving slots: uploads, kernels and result copies of different requests overlap
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

METRIC = ("events/s seeding+matching on 1 MI355X (batched vs plain) at oracle-matched "
          "tracks; p99 latency")
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "minbias": "minbias-{n}: {n} min-bias-like events per batch, Poisson(120) tracks in "
               "acceptance, p 1.5-100 GeV, 2% hit inefficiency, 10% noise hits, 5% ghost VELO "
               "states",
    "uneven": "uneven-{n}: {n} events per batch, negative-binomial(mean 120, k=1) tracks in "
              "[10, 600], otherwise min-bias-like",
    "stress": "stress-{n}: {n} events per batch, negative-binomial(mean 240, k=1) tracks in "
              "[20, 3000], 5% inefficiency, 20% noise hits",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def seed_kernel_bytes(b, n_seeds: int) -> int:
    """Algorithmic HBM bytes of one launch of the seeding kernel (main form):
    hit x, z and id (12 B/hit), per item its order record (64 B: the item and
    its 13 zone offsets) and its seed count and pool offset (8 B), per seed
    its 96 B record written to the pool."""
    return 12 * b.n_hits + (64 + 8) * 2 * b.n_events + 96 * n_seeds


def match_kernel_bytes(b, n_seeds: int, n_longs: int) -> int:
    """Algorithmic HBM bytes of one launch of the matching kernel: per event
    the two items' seed counts and pool offsets, two VELO offsets and its
    long-track count and pool offset (32 B), the VELO states (x, y, z, tx, ty,
    id: 24 B each), five fields of each seed (20 B), and per long track its
    40 B record."""
    return 32 * b.n_events + 24 * b.n_velo + 20 * n_seeds + 40 * n_longs


def cpu_baseline(batch, seconds: float):
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    O.run(batch.subset(range(min(10, batch.n_events))), threads=cores)   # warm
    t0 = time.perf_counter()
    reps = 0
    while True:
        O.run(batch, threads=cores)
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    n1 = min(200, batch.n_events)
    t1 = time.perf_counter()
    O.run(batch.subset(range(n1)), threads=1)
    d1 = time.perf_counter() - t1
    return {"value": round(reps * batch.n_events / dt, 1), "unit": "events/s", "cores": cores,
            "kind": "oracle",
            "sample": f"the benchmark batch ({batch.n_events} events) run {reps}x on {cores} "
                      f"threads ({dt:.1f} s wall); single thread on {n1} events: "
                      f"{n1 / d1:.1f} events/s"}


def serve_stream(ctx, sm, host, capacity, n_req, load):
    """Requests of 1..N events (N = the batch size) drawn from the benchmark
    batch, Poisson arrivals at `load` x the batched capacity in events/s,
    continuous batching over the library's serving slots; then the same
    stream one request at a time through the plain form."""
    import numpy as np
    from paper_2606_14480_amd import serving
    rng = np.random.default_rng(11)
    sizes = rng.integers(1, host.n_events + 1, n_req)
    starts = [int(rng.integers(0, host.n_events - k + 1)) for k in sizes]
    mean_ev = float(np.mean(sizes))
    rate = load * capacity / mean_ev
    arr = serving.poisson_arrivals(rate, n_req, seed=12)
    reqs = []
    for i, (s, k) in enumerate(zip(starts, sizes)):
        sub = host.subset(range(s, s + int(k)))
        reqs.append(serving.Request(i, sub, float(arr[i]), serving.pin(sub)))
    me = max(r.batch.n_events for r in reqs)
    mh = max(r.batch.n_hits for r in reqs)
    mv = max(r.batch.n_velo for r in reqs)
    srv = serving.Server(ctx, SERVE_SLOTS, me, mh, mv)
    # warm the slots, scratch and captured graphs with the largest request first
    big = max(reqs, key=lambda r: r.batch.n_hits)
    srv.serve([dataclasses.replace(big, arrival=0.0)] + [dataclasses.replace(r, arrival=0.0) for r in reqs[:3]])
    t0 = time.perf_counter()
    res = srv.serve(reqs, keep=False)
    wall = time.perf_counter() - t0
    s = serving.summarize(res, wall)
    out = {"requests": n_req, "events_per_request": "uniform 1-%d" % host.n_events,
           "offered_events_per_s": round(rate * mean_ev, 1),
           "events_per_s": round(s["events_per_s"], 1),
           "latency_ms_p50": round(s["latency_ms_p50"], 3),
           "latency_ms_p99": round(s["latency_ms_p99"], 3),
           "what": "arrival to results in pinned host memory, incl. H2D of the request and D2H of results"}
    n_plain = min(n_req, 12)
    t0 = time.perf_counter()
    pres = serving.serve_plain(ctx, reqs[:n_plain], me, mh, mv)
    wall_p = time.perf_counter() - t0
    p = serving.summarize(pres, wall_p)
    out["plain_stream"] = {"requests": n_plain, "events_per_s": round(p["events_per_s"], 1),
                           "latency_ms_p50": round(p["latency_ms_p50"], 3),
                           "latency_ms_p99": round(p["latency_ms_p99"], 3)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--events", type=int, default=0,
                    help="events per batch (default: the workload's own size)")
    ap.add_argument("--workload", default="minbias", choices=("minbias", "uneven", "stress"))
    ap.add_argument("--p-min", type=float, default=0.0,
                    help="minimum momentum the windows are opened for, MeV/c (0: the default 3 GeV)")
    ap.add_argument("--parity-events", type=int, default=2000,
                    help="events of the batch checked against the oracle")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=2.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=60,
                    help="requests in the served-stream measurement (0: skip)")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="offered load as a fraction of the measured batched capacity")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain copy of this many MiB (rocprof counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: events are independent, so more GPUs would "
              "each run their own batches (no collective); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_14480_amd import events as ev
    from paper_2606_14480_amd import sm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = {"minbias": 2, "uneven": 3, "stress": 4}[args.workload]
    cfg = ev.config(wl, n_events=args.events or None)
    t0 = time.perf_counter()
    host = ev.generate(cfg)
    log(f"[bench] generated {host.n_events} events, {host.n_hits} hits, {host.n_velo} VELO "
        f"states in {time.perf_counter() - t0:.1f} s")
    over = {"p_min": args.p_min} if args.p_min > 0 else {}
    ctx = sm.Context(params=sm.default_params(**over), n_slots=SERVE_SLOTS)
    db = sm.DeviceBatch(host)
    out = sm.DeviceOut(host.n_events, host.n_hits // 4 + 1024, host.n_velo + 1024)
    stream = torch.cuda.current_stream()

    ctx.run(db, out, stream)                          # sizes scratch
    gpu = out.to_host()
    n_seeds, n_longs = out.n_seeds, out.n_longs
    parity = None
    if not args.no_parity:
        from oracle import oracle as O
        import parity as PT
        npar = min(host.n_events, args.parity_events)
        sub = host if npar == host.n_events else host.subset(range(npar))
        g_sub = (gpu[0][:npar + 1], gpu[1][:gpu[0][npar]], gpu[2][:npar + 1], gpu[3][:gpu[2][npar]])
        o = O.run(sub, O.default_params(**over), threads=os.cpu_count())
        st = PT.compare(o, g_sub, npar)
        if st["mismatches"]:
            st = PT.compare(o, g_sub, npar, band=(
                O.run(sub, PT.eps_params(O, 1e-4, **over), threads=os.cpu_count()),
                O.run(sub, PT.eps_params(O, -1e-4, **over), threads=os.cpu_count())))
        parity = {"events_checked": npar, "seed_jaccard": round(st["seed_jaccard"], 6),
                  "long_jaccard": round(st["long_jaccard"], 6),
                  "mismatches": st["mismatches"], "unexplained": len(st["unexplained"]),
                  "param_failures": len(st["param_fail"])}
        log(f"[bench] parity vs oracle: {parity}")

    # ---- batched form: the timed region
    for _ in range(args.warmup):
        ctx.run(db, out, stream)
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        ctx.run(db, out, stream)
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    value = args.steps * host.n_events / elapsed
    lat_ms = np.array(lat) * 1e3
    log(f"[bench] batched: {value:.0f} events/s, {elapsed / args.steps * 1e3:.3f} ms/step")

    # ---- per-kernel device time from HIP events on the launch stream
    kt = [ctx.profile(db, out, stream) for _ in range(max(5, args.steps // 5))]
    kern = {k: float(np.mean([t[k] for t in kt])) for k in kt[0]}
    log(f"[bench] kernel ms: {json.dumps({k: round(v, 4) for k, v in kern.items()})}")

    # ---- plain form: one kernel sequence per event
    plain = None
    if args.plain_steps > 0:
        ctx.run(db, out, stream, plain=True)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(args.plain_steps):
            ctx.run(db, out, stream, plain=True)
        torch.cuda.synchronize()
        plain = args.plain_steps * host.n_events / (time.perf_counter() - tp)
        log(f"[bench] plain: {plain:.0f} events/s")

    serve = None
    if args.serve_requests > 0 and args.workload == "minbias":
        serve = serve_stream(ctx, sm, host, value, args.serve_requests, args.serve_load)
        log(f"[bench] served: {serve}")
    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {n * 4} bytes read, {n * 4} bytes written")

    alg_bytes = seed_kernel_bytes(host, n_seeds)
    # the main-form instantiation that ran (the other returns at once)
    fused = kern["seed_fused"] > kern["seed"]
    seed_ms = kern["seed_fused"] if fused else kern["seed"]
    achieved = alg_bytes / (seed_ms * 1e-3) / 1e9
    m_bytes = match_kernel_bytes(host, n_seeds, n_longs)
    m_achieved = m_bytes / (kern["match"] * 1e-3) / 1e9 if kern["match"] > 0 else None
    res = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload].format(n=host.n_events),
                   "events_per_batch": host.n_events, "hits": host.n_hits,
                   "velo_states": host.n_velo, "seeds": n_seeds, "long_tracks": n_longs,
                   "form": "batched: captured graph, persistent kernels, LPT work queue",
                   "search_dtype": "f32", "fit_dtype": "f64",
                   "p_min_mev": float(args.p_min) if args.p_min > 0 else 3000.0},
        "plain_events_per_s": round(plain, 1) if plain else None,
        "batched_over_plain": round(value / plain, 2) if plain else None,
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4),
                       "what": "per-batch latency of the batched form, call to results"},
        "kernel_ms": {k: round(v, 4) for k, v in kern.items()},
        "served": serve,
        "gpu_events_per_s": round(host.n_events / (kern["total"] * 1e-3), 1),
        "parity": parity,
        "roofline": {"bound": "hbm",
                     "kernel": "k_seed<0, 256, %s> (seeding, main form%s)"
                               % (("true", ", matching inside") if fused else ("false", "")),
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None if fused else measured_traffic(),
                     "alg_bytes_per_launch": alg_bytes},
        "roofline_match": {"bound": "hbm", "kernel": "k_match",
                           "achieved": round(m_achieved, 2) if m_achieved else None,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(m_achieved / HBM_PEAK_GBS, 5) if m_achieved else None,
                           "alg_bytes_per_launch": m_bytes},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(host, args.cpu_seconds)
    ctx.close()
    print(json.dumps(res), flush=True)


def measured_traffic():
    """HBM bytes of one k_seed launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None
    when the kernel sources differ from the ones the counters were taken on."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_seed_minbias1000_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    for name in ("sm_device.hip", "sm_device.h"):
        src = os.path.join(ROOT, "paper_2606_14480_amd", "csrc", name)
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if not re.search(re.escape(name) + r"` sha256\s*`" + digest + "`", text):
            return None
    f = re.search(r"^fetch_bytes_per_launch: (\d+)$", text, re.M)
    w = re.search(r"^write_bytes_per_launch: (\d+)$", text, re.M)
    return int(f.group(1)) + int(w.group(1)) if f and w else None


if __name__ == "__main__":
    main()
