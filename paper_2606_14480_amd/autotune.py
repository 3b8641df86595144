"""Launch-shape autotuner for the batched form.

For a representative batch of one class (mean (event, half) hit count and
event count, each rounded up to a power of two) it times every combination
of the persistent seeding grid (workgroups per CU) and the per-workgroup LDS
hit budget (which decides which items are staged in LDS and how many
workgroups fit per CU), with HIP events around the kernels, and keeps the
fastest.  The results form the context's table of launch shapes
(sm_set_shapes), cached in JSON per device name, so every batched call takes
the measured shape of its class.  The cache committed beside this module was
measured on one MI355X.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
WGS_PER_CU = (2, 3, 4)
# LDS hit budgets: round sizes, and the largest ones that still fit 4, 3 and
# 2 workgroups per CU (160 KB of LDS each, about 24.9 KB of shared state per
# workgroup besides the hits)
LDS_HITS = (1024, 1280, 1536, 2048, 2304, 3072, 4096, 4608, 6144)


def _pow2(x: float) -> int:
    return 2 ** int(math.ceil(math.log2(max(x, 1.0))))


def batch_class(batch) -> tuple:
    """(max_mean_item_hits, max_events) of the class that holds this batch."""
    ne = batch.n_events
    mean = batch.n_hits / (2.0 * ne) if ne else 0.0
    return _pow2(mean), _pow2(ne)


def load(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def shapes_for(device_name: str, path: str = CACHE) -> list:
    """The device's tuned launch shapes, tightest class first (the order in
    which the library tries them)."""
    rows = load(path).get(device_name, [])
    rows = sorted(rows, key=lambda r: (r["max_mean_item_hits"], r["max_events"]))
    return [{k: int(r[k]) for k in ("max_mean_item_hits", "max_events", "seed_wgs", "lds_hits")}
            for r in rows]


def lookup(device_name: str, batch, path: str = CACHE):
    """The tuned entry whose class holds this batch, or None."""
    mh, me = batch_class(batch)
    mean = batch.n_hits / (2.0 * batch.n_events) if batch.n_events else 0.0
    for r in shapes_for(device_name, path):
        if mean <= r["max_mean_item_hits"] and batch.n_events <= r["max_events"]:
            return r
    return None


def tune(batch, reps: int = 5, path: str = CACHE, wgs_per_cu=WGS_PER_CU, lds_hits=LDS_HITS,
         workload: str = "", log=print) -> dict:
    """Times every shape on `batch` and stores the fastest for its class."""
    import torch

    from . import sm
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    mh, me = batch_class(batch)
    db = sm.DeviceBatch(batch)
    out = sm.DeviceOut(batch.n_events, batch.n_hits // 8 + 1024, batch.n_velo + 1024)
    ctx = sm.Context(shapes=[])
    trials = []
    ref = None
    try:
        if ctx.run(db, out, check=False) == sm.ERR_CAPACITY:
            out = sm.DeviceOut(batch.n_events, out.n_seeds + 1024, out.n_longs + 1024)
        for w in wgs_per_cu:
            for h in lds_hits:
                shape = {"max_mean_item_hits": mh, "max_events": me, "seed_wgs": w * cus,
                         "lds_hits": h}
                if ctx.set_shapes([shape], check=False) != sm.OK:
                    log(f"[tune] {w} wg/CU, lds_hits {h}: not available on this device")
                    continue
                ctx.run(db, out)                      # sizes scratch, builds the graph
                got = out.to_host()
                if ref is None:
                    ref = got
                # every shape gives the same bytes
                assert all(a.tobytes() == b.tobytes() for a, b in zip(ref, got)), shape
                t = [ctx.profile(db, out)["total"] for _ in range(reps)]
                ms = float(np.median(t))
                trials.append({"wgs_per_cu": w, "seed_wgs": w * cus, "lds_hits": h, "ms": ms})
                log(f"[tune] {props.name} class ({mh}, {me}): {w} wg/CU, lds_hits {h}: "
                    f"{ms:.4f} ms")
    finally:
        ctx.close()
    best = min(trials, key=lambda r: r["ms"])
    cache = load(path)
    rows = [r for r in cache.get(props.name, [])
            if (r["max_mean_item_hits"], r["max_events"]) != (mh, me)]
    entry = {"max_mean_item_hits": mh, "max_events": me, "seed_wgs": best["seed_wgs"],
             "lds_hits": best["lds_hits"], "ms": best["ms"], "workload": workload,
             "n_events": batch.n_events, "n_hits": int(batch.n_hits), "trials": trials}
    rows.append(entry)
    cache[props.name] = sorted(rows, key=lambda r: (r["max_mean_item_hits"], r["max_events"]))
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return entry


# the batch classes the committed cache covers: (workload id, events)
CLASSES = ((2, 64), (2, 512), (2, 1000), (2, 4000), (3, 10000), (4, 5000), (4, 50000))


if __name__ == "__main__":
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2606_14480_amd import events as ev
    ap = argparse.ArgumentParser(description="tune the launch shapes of the batched form")
    ap.add_argument("--path", default=CACHE)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--only", type=int, default=0, help="tune only the classes of this workload id")
    a = ap.parse_args()
    names = {2: "minbias", 3: "uneven", 4: "stress"}
    todo = [c for c in CLASSES if not a.only or c[0] == a.only]
    batches = [(w, ev.generate_parallel(ev.config(w, n_events=n), 16)) for w, n in todo]
    for w, b in batches:
        e = tune(b, reps=a.reps, path=a.path, workload=f"{names[w]}-{b.n_events}",
                 log=lambda *x: print(*x, file=sys.stderr, flush=True))
        print(json.dumps({k: v for k, v in e.items() if k != "trials"}), flush=True)
