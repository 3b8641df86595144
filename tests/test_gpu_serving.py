"""Serving (continuous batching) and autotuning on the GPU, through the C-ABI."""
import sys

import numpy as np
import pytest

import parity as PT
from paper_2606_14480_amd import events as ev

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_14480_amd import sm as S
    return S


def make_requests(n, max_events, seed=3, rate=50000.0):
    from paper_2606_14480_amd import serving
    rng = np.random.default_rng(seed)
    pool = ev.generate(ev.config(5, n_events=max_events * 2))
    arr = serving.poisson_arrivals(rate, n, seed=seed)
    reqs = []
    for i in range(n):
        k = int(rng.integers(1, max_events + 1))
        s = int(rng.integers(0, pool.n_events - k + 1))
        reqs.append(serving.Request(i, pool.subset(range(s, s + k)), float(arr[i])))
    return reqs


def test_served_results_equal_alone(sm, orc):
    """Requests admitted while others run give the same bytes as alone."""
    from paper_2606_14480_amd import serving
    reqs = make_requests(24, 120)
    me = max(r.batch.n_events for r in reqs)
    mh = max(r.batch.n_hits for r in reqs)
    mv = max(r.batch.n_velo for r in reqs)
    say(f"[gpu] serving {len(reqs)} requests, up to {me} events")
    ctx = sm.Context(n_slots=3)
    try:
        srv = serving.Server(ctx, 3, me, mh, mv)
        res = srv.serve(reqs)
        assert sorted(r.rid for r in res) == list(range(len(reqs)))
        overlapped = sum(1 for r in res if any(o.admitted < r.done and o.done > r.admitted and
                                               o.rid != r.rid for o in res))
        say(f"[gpu] serving: {overlapped} requests overlapped another; {serving.summarize(res)}")
        by = {r.rid: r for r in res}
        for q in reqs:
            alone = sm.reconstruct(ctx, q.batch)
            r = by[q.rid]
            for a, b in zip(alone, (r.seed_off, r.seeds, r.long_off, r.longs)):
                assert a.tobytes() == b.tobytes(), q.rid
        # and a served result against the oracle
        q = max(reqs, key=lambda x: x.batch.n_events)
        o = orc.run(q.batch, threads=8)
        r = by[q.rid]
        PT.assert_parity(PT.compare(o, (r.seed_off, r.seeds, r.long_off, r.longs), q.batch.n_events))
        assert overlapped > 0
    finally:
        ctx.close()


def test_admission_by_memory_budget(sm):
    """A budget that fits one batch serialises admissions; results unchanged."""
    from paper_2606_14480_amd import serving
    reqs = make_requests(6, 60, seed=5)
    me = max(r.batch.n_events for r in reqs)
    mh = max(r.batch.n_hits for r in reqs)
    mv = max(r.batch.n_velo for r in reqs)
    say("[gpu] admission by memory")
    ctx = sm.Context(n_slots=2)
    try:
        one = max(ctx.batch_bytes(r.batch.n_events, r.batch.n_hits, r.batch.n_velo) for r in reqs)
        srv = serving.Server(ctx, 2, me, mh, mv, mem_budget=one)
        res = srv.serve(reqs)
        assert srv.peak_in_use <= one
        by = {r.rid: r for r in res}
        for q in reqs:
            alone = sm.reconstruct(ctx, q.batch)
            assert alone[1].tobytes() == by[q.rid].seeds.tobytes()
    finally:
        ctx.close()


def test_submit_busy_and_poll(sm):
    b = ev.generate(ev.config(2, n_events=20))
    say("[gpu] busy / poll")
    ctx = sm.Context(n_slots=1)
    try:
        db = sm.DeviceBatch(b)
        o1 = sm.DeviceOut(b.n_events, b.n_hits // 4 + 64, b.n_velo + 64)
        o2 = sm.DeviceOut(b.n_events, b.n_hits // 4 + 64, b.n_velo + 64)
        st, t1 = ctx.submit(db, o1)
        assert st == sm.OK
        st2, _ = ctx.submit(db, o2)
        assert st2 == sm.ERR_BUSY
        assert ctx.poll(t1, wait=True) == sm.OK
        assert ctx.poll(t1, wait=False) == sm.ERR_INVALID      # reported once
        ref = sm.reconstruct(ctx, b)
        assert o1.to_host()[1].tobytes() == ref[1].tobytes()
    finally:
        ctx.close()


def test_autotune_roundtrip(sm, tmp_path):
    """The tuner's best shape comes back from its cache as the class's entry,
    a context given the table takes it, and the bytes equal the built-in
    shape's."""
    from paper_2606_14480_amd import autotune
    import torch
    b = ev.generate(ev.config(2, n_events=100))
    say("[gpu] autotune")
    path = str(tmp_path / "tune.json")
    best = autotune.tune(b, reps=2, path=path, wgs_per_cu=(2, 4), lds_hits=(1024, 2048), log=say)
    name = torch.cuda.get_device_properties(0).name
    e = autotune.lookup(name, b, path)
    assert (e["seed_wgs"], e["lds_hits"]) == (best["seed_wgs"], best["lds_hits"])
    c = sm.Context(shapes=autotune.shapes_for(name, path))
    try:
        got = c.launch_shape(b)
        assert (got["seed_wgs"], got["lds_hits"]) == (best["seed_wgs"], best["lds_hits"])
        g = sm.reconstruct(c, b)
    finally:
        c.close()
    c2 = sm.Context(shapes=[])
    try:
        assert c2.launch_shape(b)["max_events"] == 0          # the built-in choice
        g2 = sm.reconstruct(c2, b)
    finally:
        c2.close()
    for x, y in zip(g, g2):
        assert x.tobytes() == y.tobytes()


def test_shape_table_classes(sm):
    """Batches take the first table entry whose class holds them (a batch
    beyond every class of its item size the largest of the smallest item
    size); a grid larger than the context's grows its scratch; entries out of
    range are refused; outputs do not depend on the shape."""
    small = ev.generate(ev.config(2, n_events=30))
    big = ev.generate(ev.config(4, n_events=30))
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    table = [{"max_mean_item_hits": 1024, "max_events": 64, "seed_wgs": 5 * cus, "lds_hits": 1536},
             {"max_mean_item_hits": 1 << 20, "max_events": 1 << 20, "seed_wgs": 2 * cus,
              "lds_hits": 3072}]
    say("[gpu] shape table")
    c = sm.Context(shapes=table)
    ref = sm.Context(shapes=[])
    try:
        assert c.launch_shape(small)["seed_wgs"] == 5 * cus       # min-bias items: first class
        assert c.launch_shape(big)["lds_hits"] == 3072            # dense items: second class
        for b in (small, big):
            for x, y in zip(sm.reconstruct(c, b), sm.reconstruct(ref, b)):
                assert x.tobytes() == y.tobytes()
        # a batch with more events than every class of its item size: the
        # class of the smallest item size that holds it, with the most events
        from types import SimpleNamespace as NS
        far = [{"max_mean_item_hits": 1024, "max_events": 64, "seed_wgs": 5 * cus, "lds_hits": 1536},
               {"max_mean_item_hits": 1024, "max_events": 512, "seed_wgs": 4 * cus,
                "lds_hits": 1280},
               {"max_mean_item_hits": 2048, "max_events": 128, "seed_wgs": 3 * cus,
                "lds_hits": 2048}]
        c.set_shapes(far)
        assert c.launch_shape(NS(n_events=1000, n_hits=1000 * 1000))["seed_wgs"] == 4 * cus
        assert c.launch_shape(NS(n_events=100, n_hits=100 * 1000))["seed_wgs"] == 4 * cus
        assert c.launch_shape(NS(n_events=50, n_hits=50 * 1000))["seed_wgs"] == 5 * cus
        assert c.launch_shape(NS(n_events=1000, n_hits=1000 * 3000))["seed_wgs"] == 3 * cus
        assert c.launch_shape(NS(n_events=1000, n_hits=1000 * 5000))["max_events"] == 0
        for bad in ({"max_mean_item_hits": 1, "max_events": 1, "seed_wgs": 1, "lds_hits": 1024},
                    {"max_mean_item_hits": 1, "max_events": 1, "seed_wgs": 64, "lds_hits": 1000},
                    {"max_mean_item_hits": 1, "max_events": 1, "seed_wgs": 64, "lds_hits": 8192}):
            assert c.set_shapes([bad], check=False) == sm.ERR_INVALID
    finally:
        c.close()
        ref.close()


def test_pool_slice_requests_equal_alone(sm):
    """Requests that are runs of consecutive events of one pinned pool (the
    serving leg's form: hits copied straight from the pool, offsets rebased)
    give the same bytes as the same events run alone."""
    from paper_2606_14480_amd import serving
    host = ev.generate(ev.config(5, n_events=300))
    pool = serving.EventPool(host)
    rng = np.random.default_rng(9)
    sizes = rng.integers(1, 200, 16)
    firsts = [int(rng.integers(0, host.n_events - int(k) + 1)) for k in sizes]
    arr = serving.poisson_arrivals(20000.0, len(sizes), seed=4)
    reqs = [serving.Request(i, None, float(arr[i]), pool=pool, first=firsts[i], count=int(k))
            for i, k in enumerate(sizes)]
    say(f"[gpu] pool-slice serving: {len(reqs)} requests")
    ctx = sm.Context(n_slots=3)
    try:
        srv = serving.Server(ctx, 3, host.n_events, host.n_hits, host.n_velo)
        res = srv.serve(reqs)
        by = {r.rid: r for r in res}
        assert sorted(by) == list(range(len(reqs)))
        for q in reqs:
            alone = sm.reconstruct(ctx, host.subset(range(q.first, q.first + q.count)))
            r = by[q.rid]
            for a, b in zip(alone, (r.seed_off, r.seeds, r.long_off, r.longs)):
                assert a.tobytes() == b.tobytes(), q.rid
    finally:
        ctx.close()
