"""Launch-shape autotuner for the batched form.

For a representative batch it times every combination of the persistent
seeding grid (workgroups per CU) and the per-workgroup LDS hit budget (which
decides which (event, half) items are staged in LDS and how many workgroups
fit per CU), with HIP events around the kernels, and keeps the fastest.
Results are cached in JSON keyed by device name and the batch's mean and
maximum (event, half) hit counts (bucketed to powers of two), so a batch of
a new shape is tuned once.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
WGS_PER_CU = (2, 3, 4, 6, 8)
LDS_HITS = (1024, 1536, 2048, 3072, 4096)


def shape_key(device_name: str, batch) -> str:
    h = batch.event_hits().astype(np.float64) / 2.0
    mean = float(h.mean()) if len(h) else 0.0
    mx = float(h.max()) if len(h) else 0.0
    b = lambda x: 2 ** int(math.ceil(math.log2(max(x, 1.0))))
    return f"{device_name}|mean<={b(mean)}|max<={b(mx)}"


def load(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(device_name: str, batch, path: str = CACHE):
    """(seed_wgs, lds_hits) for this device and batch shape, or None."""
    e = load(path).get(shape_key(device_name, batch))
    return (e["seed_wgs"], e["lds_hits"]) if e else None


def tune(batch, reps: int = 5, path: str = CACHE, wgs_per_cu=WGS_PER_CU, lds_hits=LDS_HITS,
         log=print) -> dict:
    import torch

    from . import sm
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    key = shape_key(props.name, batch)
    db = sm.DeviceBatch(batch)
    out = sm.DeviceOut(batch.n_events, batch.n_hits // 4 + 1024, batch.n_velo + 1024)
    trials = []
    for w in wgs_per_cu:
        for h in lds_hits:
            ctx = sm.Context(seed_wgs=w * cus, lds_hits=h)
            try:
                ctx.run(db, out)                      # sizes scratch, builds the graph
                t = [ctx.profile(db, out)["total"] for _ in range(reps)]
            finally:
                ctx.close()
            ms = float(np.median(t))
            trials.append({"wgs_per_cu": w, "seed_wgs": w * cus, "lds_hits": h, "ms": ms})
            log(f"[tune] {key}: {w} wg/CU, lds_hits {h}: {ms:.4f} ms")
    best = min(trials, key=lambda r: r["ms"])
    cache = load(path)
    cache[key] = {"seed_wgs": best["seed_wgs"], "lds_hits": best["lds_hits"], "ms": best["ms"],
                  "n_events": batch.n_events, "trials": trials}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return cache[key]


if __name__ == "__main__":
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2606_14480_amd import events as ev
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, action="append", default=None)
    ap.add_argument("--events", type=int, default=1000)
    a = ap.parse_args()
    for c in a.config or [2]:
        best = tune(ev.generate(ev.config(c, n_events=a.events)))
        print(json.dumps({k: v for k, v in best.items() if k != "trials"}), flush=True)
