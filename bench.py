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
    "ghost": "minbias-{n} with the network form of the final selection (Sec. 4.4: ghost "
             "probability < 0.8, clone gap 0.05; weights trained on the generator's truth)",
    "third": "minbias-{n} with the third x-z iteration after the clean-up (Sec. 3; windows "
             "opened for 1.5 GeV/c on the hits the first two iterations left)",
    "ut": "minbias-{n} with the UT hit search (Sec. 4.3; a synthetic four-layer UT, about 500 "
          "UT hits per event; more than two UT hits per long track)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def seed_kernel_bytes(b, n_seeds: int) -> int:
    """Algorithmic HBM bytes of one launch of the seeding kernel (main form):
    hit x, z and id (12 B/hit), per item its order record (64 B: the item and
    its 13 zone offsets) and its seed count and pool offset (8 B), per seed
    its 96 B record written to the pool."""
    return 12 * b.n_hits + (64 + 8) * 2 * b.n_events + 96 * n_seeds


# batches of up to this many events have their seeds written to the outputs by
# the matching kernel (the copy kernel then moves only the long tracks)
MATCH_SEEDS_EVENTS = 4096


def match_kernel_bytes(b, n_seeds: int, n_longs: int) -> int:
    """Algorithmic HBM bytes of one launch of the matching kernel: per event
    the two items' seed counts and pool offsets, two VELO offsets and its
    long-track count and pool offset (32 B), the VELO states (x, y, z, tx, ty,
    id: 24 B each), per long track its 64 B record, and per seed five fields
    (20 B), or, when the kernel also writes the seeds to the outputs, its
    96 B record read and written."""
    per_seed = 2 * 96 if b.n_events <= MATCH_SEEDS_EVENTS else 20
    return 32 * b.n_events + 24 * b.n_velo + per_seed * n_seeds + 64 * n_longs


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(batch, seconds: float):
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = min(cores, 16)   # the host share of one GPU
    O.run(batch.subset(range(min(10, batch.n_events))), threads=cores, margins=False)   # warm
    t0 = time.perf_counter()
    reps = 0
    while True:
        O.run(batch, threads=cores, margins=False)
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    n1 = min(200, batch.n_events)
    t1 = time.perf_counter()
    O.run(batch.subset(range(n1)), threads=1, margins=False)
    d1 = time.perf_counter() - t1
    return {"value": round(reps * batch.n_events / dt, 1), "unit": "events/s", "cores": cores,
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"the benchmark batch ({batch.n_events} events) run {reps}x on {cores} "
                      f"threads ({dt:.1f} s wall), the oracle's margin log off; single "
                      f"thread on {n1} events: {n1 / d1:.1f} events/s"}


def copy_bandwidth(mib: int = 256):
    """Host<->device copy rate of pinned memory (GB/s), timed with events on
    one stream: the link the serving leg moves requests and results over."""
    import torch
    n = mib << 20
    h = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(n, dtype=torch.uint8, device="cuda")
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    for _ in range(2):
        e0.record(); d.copy_(h, non_blocking=True); e1.record(); h.copy_(d, non_blocking=True)
        e2.record(); torch.cuda.synchronize()
    return {"h2d_GBps": round(n / (e0.elapsed_time(e1) * 1e-3) / 1e9, 2),
            "d2h_GBps": round(n / (e1.elapsed_time(e2) * 1e-3) / 1e9, 2),
            "bytes": n}


def serve_stream(ctx, sm, pool_batch, n_req, loads, n_plain):
    """Serving leg: requests of 1..N consecutive events of a pinned pool of
    N min-bias events, continuous batching over the library's serving slots.
    The served capacity (every request queued at t = 0, copies included) is
    measured first; then Poisson arrivals at each offered load (a fraction of
    that capacity), and the first requests of the 0.8 stream one at a time
    through the plain form."""
    import numpy as np
    import torch
    from paper_2606_14480_amd import serving
    pool = serving.EventPool(pool_batch)
    N = pool.n_events
    rng = np.random.default_rng(11)
    sizes = rng.integers(1, N + 1, n_req)
    firsts = [int(rng.integers(0, N - int(k) + 1)) for k in sizes]
    mean_ev = float(np.mean(sizes))

    def stream(arr):
        return [serving.Request(i, None, float(arr[i]), pool=pool, first=firsts[i],
                                count=int(sizes[i])) for i in range(n_req)]

    free, _ = torch.cuda.mem_get_info()
    srv = serving.Server(ctx, SERVE_SLOTS, N, pool_batch.n_hits, pool_batch.n_velo,
                         mem_budget=int(free * 0.8))
    srv.serve(stream(np.zeros(n_req))[:2 * SERVE_SLOTS], keep=False)   # warm slots and graphs
    t0 = time.perf_counter()
    res = srv.serve(stream(np.zeros(n_req)), keep=False)
    wall = time.perf_counter() - t0
    cap = sum(r.n_events for r in res) / wall
    out = {"requests_per_load": n_req, "events_per_request": "uniform 1-%d" % N,
           "pool": "%d min-bias events packed once in pinned memory; a request is a run of "
                   "consecutive pool events" % N,
           "capacity_events_per_s": round(cap, 1),
           "capacity_what": "every request queued at t=0; H2D of each request and D2H of its "
                            "results included",
           "what": "latency = arrival to results in pinned host memory", "loads": {}}
    for k, load in enumerate(loads):
        rate = load * cap / mean_ev
        arr = serving.poisson_arrivals(rate, n_req, seed=12 + k)
        t0 = time.perf_counter()
        res = srv.serve(stream(arr), keep=False)
        wall = time.perf_counter() - t0
        st = serving.summarize(res, wall)
        out["loads"][str(load)] = {"offered_events_per_s": round(rate * mean_ev, 1),
                                   "events_per_s": round(st["events_per_s"], 1),
                                   "latency_ms_p50": round(st["latency_ms_p50"], 3),
                                   "latency_ms_p99": round(st["latency_ms_p99"], 3)}
        log(f"[bench] served at {load}: {out['loads'][str(load)]}")
    if n_plain > 0:
        rate = 0.8 * cap / mean_ev
        arr = serving.poisson_arrivals(rate, n_req, seed=13)
        reqs = stream(arr)[:n_plain]
        t0 = time.perf_counter()
        pres = serving.serve_plain(ctx, reqs, N, pool_batch.n_hits, pool_batch.n_velo)
        p = serving.summarize(pres, time.perf_counter() - t0)
        out["plain_stream"] = {"requests": n_plain, "what": "the first requests of the 0.8 "
                               "stream, one kernel sequence per event",
                               "events_per_s": round(p["events_per_s"], 1),
                               "latency_ms_p50": round(p["latency_ms_p50"], 3),
                               "latency_ms_p99": round(p["latency_ms_p99"], 3)}
    out["copy_bandwidth"] = copy_bandwidth()
    return out


def run_in_flight(ctx, sm, db, outs, n):
    """n resident batches through the context's submit/poll slots with
    len(outs) of them in flight (each slot its own stream and graph; a new
    batch takes the output buffers of the one that just completed).  Returns
    the wall time and each batch's latency from submit to its results."""
    k = len(outs)
    pending, lat = [], []
    nxt = 0
    t0 = time.perf_counter()
    while len(lat) < n:
        while nxt < n and len(pending) < k:
            st, t = ctx.submit(db, outs[nxt % k])
            if st != sm.OK:
                raise sm.SmError(st, "sm_submit")
            pending.append((t, time.perf_counter()))
            nxt += 1
        t, ts = pending.pop(0)
        st = ctx.poll(t, True)
        if st != sm.OK:
            raise sm.SmError(st, "sm_poll")
        lat.append(time.perf_counter() - ts)
    return time.perf_counter() - t0, lat


def run_sized(ctx, sm, db, host, stream):
    """One run with outputs sized from the first guess, or from the sizes the
    library reports if they do not fit."""
    out = sm.DeviceOut(host.n_events, host.n_hits // 8 + 1024, host.n_velo + 1024)
    if ctx.run(db, out, stream, check=False) == sm.ERR_CAPACITY:
        out = sm.DeviceOut(host.n_events, out.n_seeds + 1024, out.n_longs + 1024)
        ctx.run(db, out, stream)
    return out


def oracle_parity(host, gpu, n_events, over):
    """Seeds and long tracks of the first n_events events against the oracle."""
    from oracle import oracle as O
    import parity as PT
    npar = min(host.n_events, n_events)
    sub = host if npar == host.n_events else host.subset(range(npar))
    g_sub = (gpu[0][:npar + 1], gpu[1][:gpu[0][npar]], gpu[2][:npar + 1], gpu[3][:gpu[2][npar]])
    th = min(os.cpu_count() or 1, 16)
    o = O.run(sub, O.default_params(**over), threads=th)
    st = PT.compare(o, g_sub, npar)
    if st["mismatches"]:
        st = PT.compare(o, g_sub, npar, band=(
            O.run(sub, PT.eps_params(O, 1e-4, **over), threads=th),
            O.run(sub, PT.eps_params(O, -1e-4, **over), threads=th)))
    return {"events_checked": npar, "seed_jaccard": round(st["seed_jaccard"], 6),
            "long_jaccard": round(st["long_jaccard"], 6),
            "mismatches": st["mismatches"], "unexplained": len(st["unexplained"]),
            "param_failures": len(st["param_fail"])}


def extra_leg(ctx, sm, name, host, steps, warmup, parity_events, over):
    """Batched events/s of one more workload at its stated size (same
    context, same captured-graph form), with oracle parity on its first
    events."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()
    db = sm.DeviceBatch(host)
    out = run_sized(ctx, sm, db, host, stream)
    gpu = out.to_host()
    par = oracle_parity(host, gpu, parity_events, over) if parity_events > 0 else None
    for _ in range(warmup):
        ctx.run(db, out, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run(db, out, stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kern = ctx.profile(db, out, stream)
    ev_hits = host.event_hits()
    res = {"workload": WORKLOADS[name].format(n=host.n_events), "events": host.n_events,
           "hits": host.n_hits, "hits_per_event": {"min": int(ev_hits.min()),
                                                   "mean": round(float(ev_hits.mean()), 1),
                                                   "max": int(ev_hits.max())},
           "events_per_s": round(host.n_events / dt, 1), "ms_per_batch": round(dt * 1e3, 3),
           "steps": steps, "seeds": out.n_seeds, "long_tracks": out.n_longs,
           "launch": dict(ctx.launch_shape(host), source=ctx.shape_source),
           "kernel_ms": {k: round(v, 4) for k, v in kern.items()}, "parity": par}
    log(f"[bench] {name}: {res['events_per_s']:.0f} events/s, {res['ms_per_batch']} ms/batch, "
        f"parity {par}")
    del db, out
    torch.cuda.empty_cache()
    return res


class TiledBatch:
    """A device batch holding the events of another r times over (hit and
    VELO offsets shifted per copy): batches far larger than the host can
    generate, of the same events."""

    def __init__(self, sm, db, r):
        import torch
        nh, nv = db.n_hits, db.n_velo
        assert r * nh < 2 ** 31 and r * nv < 2 ** 31, "offsets are int32"
        self.n_events, self.n_hits, self.n_velo = r * db.n_events, r * nh, r * nv

        def offs(o, n):
            o = o.to(torch.int64)
            return torch.cat([o[:-1] + k * n for k in range(r)] + [o[-1:] + (r - 1) * n]) \
                .to(torch.int32)

        self.zone_off = offs(db.zone_off, nh)
        self.velo_off = offs(db.velo_off, nv)
        rep = lambda a: a.repeat(r)
        self.hit_x, self.hit_z, self.hit_id = rep(db.hit_x), rep(db.hit_z), rep(db.hit_id)
        self.velo = [rep(getattr(db, "velo_" + k)) for k in ("x", "y", "z", "tx", "ty", "id")]
        v = [a.data_ptr() for a in self.velo]
        self.c = sm.Batch(n_events=self.n_events, pad=0, n_hits=self.n_hits, n_velo=self.n_velo,
                          zone_off=self.zone_off.data_ptr(), hit_x=self.hit_x.data_ptr(),
                          hit_z=self.hit_z.data_ptr(), hit_id=self.hit_id.data_ptr(),
                          velo_off=self.velo_off.data_ptr(), velo_x=v[0], velo_y=v[1],
                          velo_z=v[2], velo_tx=v[3], velo_ty=v[4], velo_id=v[5], n_ut=0,
                          ut_off=None, ut_x=None, ut_id=None)


def stress_sweep(sm, params, host, reps, steps):
    """Batch-size sweep of the stress workload: its events tiled r times in
    one batch, for each r while the device holds it; every copy's outputs
    must equal the single batch's, byte for byte.  It runs on a context of
    its own, closed at the end, so that the largest batch's scratch does not
    stay with the bench's context."""
    import torch
    ctx = sm.Context(params=params)
    try:
        return _stress_sweep(ctx, sm, host, reps, steps)
    finally:
        ctx.close()
        torch.cuda.empty_cache()


def _stress_sweep(ctx, sm, host, reps, steps):
    import torch
    stream = torch.cuda.current_stream()
    db = sm.DeviceBatch(host)
    base = run_sized(ctx, sm, db, host, stream)
    bs, bl = base.n_seeds, base.n_longs
    seed_rec = base.seeds[: bs * sm.SEED_DTYPE.itemsize]
    long_rec = base.longs[: bl * sm.LONG_DTYPE.itemsize]
    total = torch.cuda.mem_get_info()[1]
    rows, per_event = [], None
    for r in reps:
        if r * db.n_hits >= 2 ** 31:
            rows.append({"copies": r, "events": r * host.n_events, "skipped": "more than 2^31 hits "
                         "(int32 hit offsets)"})
            continue
        if per_event is not None and per_event * r * host.n_events > 0.8 * total:
            rows.append({"copies": r, "events": r * host.n_events,
                         "skipped": "projected device memory above 80 % of the device"})
            continue
        tb = TiledBatch(sm, db, r)
        out = sm.DeviceOut(tb.n_events, r * bs + 1024, r * bl + 1024)
        if ctx.run(tb, out, stream, check=False) == sm.ERR_CAPACITY:
            raise RuntimeError("tiled stress batch: outputs sized from the single batch overflowed")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run(tb, out, stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        used = total - torch.cuda.mem_get_info()[0]
        same = out.n_seeds == r * bs and out.n_longs == r * bl and all(
            torch.equal(out.seeds[k * seed_rec.numel():(k + 1) * seed_rec.numel()], seed_rec) and
            torch.equal(out.longs[k * long_rec.numel():(k + 1) * long_rec.numel()], long_rec)
            for k in range(r))
        per_event = used / tb.n_events
        rows.append({"copies": r, "events": tb.n_events, "hits": tb.n_hits,
                     "events_per_s": round(tb.n_events / dt, 1), "ms_per_batch": round(dt * 1e3, 2),
                     "device_bytes_in_use": int(used), "copies_identical": bool(same)})
        log(f"[bench] stress sweep: {rows[-1]}")
        del tb, out
        torch.cuda.empty_cache()
    del db, base
    torch.cuda.empty_cache()
    hit_bytes = 12 * host.n_hits / host.n_events
    return {"what": "the stress batch's events tiled r times in one batch; each copy's outputs "
                    "compared byte for byte with the single batch's (itself checked against the "
                    "oracle on events 0-499)",
            "device_bytes": int(total),
            "limit": "int32 hit offsets: at most 2^31 hits per batch (about %d stress events); "
                     "device memory would hold about %d at the largest run's bytes per event"
                     % (2 ** 31 / (host.n_hits / host.n_events),
                        0.8 * total / per_event if per_event else 0),
            "hit_bytes_per_event": round(hit_bytes, 1), "batches": rows}


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
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per offered load in the serving leg (0: skip)")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95",
                    help="offered loads, as fractions of the measured served capacity")
    ap.add_argument("--serve-pool", type=int, default=4000,
                    help="min-bias events in the serving pool (requests are 1..this many)")
    ap.add_argument("--serve-plain", type=int, default=20,
                    help="requests of the 0.8 stream also run through the plain form")
    ap.add_argument("--legs", default="uneven,stress,ghost,ut,third",
                    help="further workloads at their stated sizes, timed beside the headline "
                         "(comma list of uneven, stress, ghost, ut, third; empty: none)")
    ap.add_argument("--leg-steps", type=int, default=5)
    ap.add_argument("--stress-sweep", default="1,2,4,8,12",
                    help="batch-size sweep of the stress leg: copies of its events per batch "
                         "(empty: none)")
    ap.add_argument("--in-flight", type=int, default=2,
                    help="resident batches on the device at once in the timed region "
                         "(continuous batching over the context's slots)")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes generating the synthetic events")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain copy of this many MiB (rocprof counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: events are independent, so more GPUs would "
              "each run their own batches (no collective); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_2606_14480_amd import events as ev

    # every synthetic input first, in worker processes started before this
    # process touches the GPU
    wl = {"minbias": 2, "uneven": 3, "stress": 4}[args.workload]
    gen = lambda cfg: ev.generate_parallel(cfg, args.gen_workers)
    t0 = time.perf_counter()
    host = gen(ev.config(wl, n_events=args.events or None))
    legs = [x for x in args.legs.split(",") if x and x != args.workload]
    leg_hosts = {x: gen(ev.config({"uneven": 3, "stress": 4}[x])) for x in legs
                 if x not in ("ghost", "ut", "third")}
    pool = gen(ev.config(5, n_events=args.serve_pool)) \
        if args.serve_requests > 0 and args.workload == "minbias" else None
    log(f"[bench] generated {host.n_events} events, {host.n_hits} hits, {host.n_velo} VELO "
        f"states (+ {', '.join(f'{k} {v.n_events}' for k, v in leg_hosts.items()) or 'no legs'}"
        f"{', serving pool %d' % pool.n_events if pool is not None else ''}) in "
        f"{time.perf_counter() - t0:.1f} s")

    import torch
    from paper_2606_14480_amd import sm
    assert torch.cuda.is_available(), "bench.py needs a GPU"
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
        parity = oracle_parity(host, gpu, args.parity_events, over)
        log(f"[bench] parity vs oracle: {parity}")

    # ---- batched form, one batch at a time (blocking call per batch)
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
    seq_elapsed = time.perf_counter() - t_start
    seq_value = args.steps * host.n_events / seq_elapsed
    seq_lat_ms = np.array(lat) * 1e3
    log(f"[bench] batched, one at a time: {seq_value:.0f} events/s, "
        f"{seq_elapsed / args.steps * 1e3:.3f} ms/step")

    # ---- the timed region: a continuous stream of resident batches, each a
    # full pass of the path, args.in_flight of them on the device at once
    # (continuous batching on the context's slots)
    k_in = max(1, min(args.in_flight, SERVE_SLOTS - 1))
    outs = [out] + [sm.DeviceOut(host.n_events, host.n_hits // 4 + 1024, host.n_velo + 1024)
                    for _ in range(k_in - 1)]
    run_in_flight(ctx, sm, db, outs, max(args.warmup, 2 * k_in))
    torch.cuda.synchronize()
    elapsed, lat = run_in_flight(ctx, sm, db, outs, args.steps)
    torch.cuda.synchronize()
    value = args.steps * host.n_events / elapsed
    lat_ms = np.array(lat) * 1e3
    # every slot's last outputs equal the first run's
    same = True
    for o in outs:
        same = same and all(a.tobytes() == b.tobytes() for a, b in zip(o.to_host(), gpu))
    log(f"[bench] batched, {k_in} in flight: {value:.0f} events/s, "
        f"{elapsed / args.steps * 1e3:.3f} ms/step, outputs identical: {same}")
    del outs

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

    # serving before the large legs: after the stress batch-size sweep has
    # taken and released most of the device's memory, the served capacity
    # measured lower (1.2-1.3 M against 1.74 M events/s)
    serve = None
    if pool is not None:
        loads = [float(x) for x in args.serve_loads.split(",") if x]
        serve = serve_stream(ctx, sm, pool, args.serve_requests, loads, args.serve_plain)
        log(f"[bench] served: capacity {serve['capacity_events_per_s']:.0f} events/s, "
            f"copies {serve['copy_bandwidth']}")

    # further workloads at their stated sizes (uneven: all events against the
    # oracle; stress: events 0-499)
    leg_res = {}
    # the headline batch again, through a context with the network form of
    # the final selection, and one with the UT search
    for name, g_over in (("ghost", dict(over, final_sel=1)), ("ut", dict(over, ut_mode=1)),
                         ("third", dict(over, third_iter=1))):
        if name not in legs or args.workload != "minbias":
            continue
        gctx = sm.Context(params=sm.default_params(**g_over))
        o_over = dict(g_over, ghost_nn=sm.ghost_nn_weights()) if name == "ghost" else g_over
        try:
            leg_res[name] = extra_leg(gctx, sm, name, host, args.leg_steps, 1,
                                      0 if args.no_parity else host.n_events, o_over)
        finally:
            gctx.close()
    for name, lh in leg_hosts.items():
        leg_res[name] = extra_leg(ctx, sm, name, lh, args.leg_steps, 1,
                                  0 if args.no_parity else (lh.n_events if name == "uneven" else 500),
                                  over)
        reps = [int(x) for x in args.stress_sweep.split(",") if x]
        if name == "stress" and reps:
            leg_res[name]["batch_size_sweep"] = stress_sweep(sm, sm.default_params(**over), lh,
                                                             reps, 2)
        del lh
    leg_hosts.clear()

    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {n * 4} bytes read, {n * 4} bytes written")

    alg_bytes = seed_kernel_bytes(host, n_seeds)
    # the main-form instantiation that ran (only the one that fits is launched)
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
                   "form": "batched: captured graph, persistent kernels, LPT work queue; "
                           "%d batches in flight" % k_in,
                   "search_dtype": "f32", "fit_dtype": "f64",
                   "p_min_mev": float(args.p_min) if args.p_min > 0 else 3000.0},
        "plain_events_per_s": round(plain, 1) if plain else None,
        "batched_over_plain": round(value / plain, 2) if plain else None,
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4),
                       "what": "per-batch latency with %d batches in flight, submit to results"
                               % k_in},
        "in_flight": {"batches": k_in, "outputs_identical": bool(same),
                      "what": "a continuous stream of resident batches on the context's "
                              "slots (each its own stream and captured graph); a batch "
                              "starts when an earlier one completes"},
        "one_at_a_time": {"events_per_s": round(seq_value, 1),
                          "ms_per_batch": round(seq_elapsed / args.steps * 1e3, 4),
                          "latency_ms": {"p50": round(float(np.percentile(seq_lat_ms, 50)), 4),
                                         "p99": round(float(np.percentile(seq_lat_ms, 99)), 4)},
                          "what": "one blocking call per batch, call to results"},
        "kernel_ms": {k: round(v, 4) for k, v in kern.items()},
        "launch": dict(ctx.launch_shape(host), source=ctx.shape_source),
        "served": serve,
        "workloads": leg_res,
        "gpu_events_per_s": round(host.n_events / (kern["total"] * 1e-3), 1),
        "parity": parity,
        "roofline": {"bound": "hbm",
                     "kernel": "k_seed<0, 256, %s, 0> (seeding, main form%s)"
                               % (("true", ", matching inside") if fused else ("false", "")),
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None if fused else measured_traffic(),
                     "alg_bytes_per_launch": alg_bytes,
                     "counters": None if fused else measured_sq()},
        "roofline_match": {"bound": "hbm", "kernel": "k_match<0>",
                           "achieved": round(m_achieved, 2) if m_achieved else None,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(m_achieved / HBM_PEAK_GBS, 5) if m_achieved else None,
                           "alg_bytes_per_launch": m_bytes},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(host, args.cpu_seconds)
    ctx.close()
    print(json.dumps(res), flush=True)


def _profile_lines(name):
    """The key: value lines of a committed rocprofv3 summary, or None when
    the kernel sources differ from the ones it was taken on."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    for src_name in ("sm_device.hip", "sm_device.h"):
        src = os.path.join(ROOT, "paper_2606_14480_amd", "csrc", src_name)
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if not re.search(re.escape(src_name) + r"` sha256\s*`" + digest + "`", text):
            return None
    return dict(re.findall(r"^([a-z_]+): ([0-9.]+)$", text, re.M))


def measured_sq():
    """VALU busy, active lanes, waves per CU and LDS use of the seeding
    kernel from the committed SQ counter summary (None if stale)."""
    kv = _profile_lines("k_seed_minbias1000_sq_counters.md")
    if not kv:
        return None
    keys = ("valu_busy", "valu_active_lanes", "waves_per_cu", "lds_utilisation", "lds_bank_conflict")
    out = {k: float(kv[k]) for k in keys if k in kv}
    out["source"] = "profiles/k_seed_minbias1000_sq_counters.md"
    return out


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
