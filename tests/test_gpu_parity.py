"""HIP library vs FP64 oracle, through the C-ABI (needs an MI355X).

Sizes: the tiny workload, 100..1000 min-bias events, uneven and stress
subsets — big enough to span many workgroups, LDS tiles and a ragged tail,
small enough for the oracle to finish in seconds.
"""
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


@pytest.fixture(scope="module")
def ctx(sm):
    c = sm.Context()
    yield c
    c.close()


def gpu_run(sm, ctx, b, plain=False, seed_cap=None, long_cap=None):
    return sm.reconstruct(ctx, b, plain=plain, seed_cap=seed_cap, long_cap=long_cap)


def check(orc, sm, ctx, b, tag, params_over=None, ctx_params=None):
    params_over = params_over or {}
    say(f"[gpu] {tag}: {b.n_events} events, {b.n_hits} hits, {b.n_velo} velo")
    g = gpu_run(sm, ctx, b)
    o = orc.run(b, orc.default_params(**params_over), threads=8)
    st = PT.compare(o, g, b.n_events)
    if st["mismatches"]:
        loose = orc.run(b, PT.eps_params(orc, 1e-4, **params_over), threads=8)
        tight = orc.run(b, PT.eps_params(orc, -1e-4, **params_over), threads=8)
        st = PT.compare(o, g, b.n_events, band=(loose, tight))
    say(f"[gpu] {tag}: seeds {st['seeds_o']}/{st['seeds_g']} jaccard {st['seed_jaccard']:.6f} "
        f"longs {st['longs_o']}/{st['longs_g']} jaccard {st['long_jaccard']:.6f} "
        f"mismatches {st['mismatches']}")
    PT.assert_parity(st)
    return g, o, st


def test_tiny_config(orc, sm, ctx):
    b = ev.generate(ev.config(1, n_events=10))
    g, o, st = check(orc, sm, ctx, b, "tiny")
    assert st["mismatches"] == 0


def test_tiny_config_low_pmin(orc, sm):
    b = ev.generate(ev.config(1, n_events=10))
    c = sm.Context(params=sm.default_params(p_min=1800.0))
    try:
        g, o, st = check(orc, sm, c, b, "tiny p_min 1.8 GeV", params_over=dict(p_min=1800.0))
        assert st["seeds_g"] >= 190
    finally:
        c.close()


def test_minbias_parity(orc, sm, ctx):
    b = ev.generate(ev.config(2, n_events=200))
    check(orc, sm, ctx, b, "minbias 200")


def test_minbias_full_size(orc, sm, ctx):
    """The benchmarked workload itself: 1000 min-bias events, one batch."""
    b = ev.generate(ev.config(2, n_events=1000))
    check(orc, sm, ctx, b, "minbias 1000")


def test_global_hit_path_parity(orc, sm):
    """An LDS hit capacity of 256, below every min-bias item: each item reads
    its hits from global memory (and its candidate-side arrays from global
    scratch where they outgrow LDS), against the oracle."""
    b = ev.generate(ev.config(2, n_events=100))
    say("[gpu] global hit path, minbias 100, lds_hits 256, smallest item",
        int(np.diff(b.zone_off[::12].astype(np.int64)).min()))
    c = sm.Context(lds_hits=256)
    try:
        check(orc, sm, c, b, "minbias 100, lds_hits 256")
    finally:
        c.close()


def test_uneven_subset(orc, sm, ctx):
    b = ev.generate(ev.config(3, n_events=300))
    check(orc, sm, ctx, b, "uneven 300")


def test_stress_subset(orc, sm, ctx):
    b = ev.generate(ev.config(4, n_events=60))
    say("[gpu] stress hits/event max", int(b.event_hits().max()))
    check(orc, sm, ctx, b, "stress 60")


def test_batched_equals_plain(sm, ctx):
    b = ev.generate(ev.config(2, n_events=40))
    say("[gpu] batched vs plain, 40 events")
    g1 = gpu_run(sm, ctx, b)
    g2 = gpu_run(sm, ctx, b, plain=True)
    for x, y in zip(g1, g2):
        assert x.tobytes() == y.tobytes()


def test_grid_shape_and_batch_composition(sm, ctx):
    """Deterministic for any grid shape, and an event's result does not depend
    on the other events of its batch."""
    b = ev.generate(ev.config(3, n_events=50))
    say("[gpu] grid shapes, 50 events")
    g1 = gpu_run(sm, ctx, b)
    c2 = sm.Context(seed_wgs=7, lds_hits=1024)
    try:
        g2 = gpu_run(sm, c2, b)
    finally:
        c2.close()
    for x, y in zip(g1, g2):
        assert x.tobytes() == y.tobytes()
    sub = [3, 17, 42]
    g3 = gpu_run(sm, ctx, b.subset(sub))
    for i, e in enumerate(sub):
        s1 = g1[1][g1[0][e]:g1[0][e + 1]]
        s3 = g3[1][g3[0][i]:g3[0][i + 1]]
        assert s1.tobytes() == s3.tobytes()
        l1 = g1[3][g1[2][e]:g1[2][e + 1]]
        l3 = g3[3][g3[2][i]:g3[2][i + 1]]
        assert l1.tobytes() == l3.tobytes()


def test_edge_cases(orc, sm, ctx):
    say("[gpu] edge cases")
    empty = ev.empty_event()
    # a batch of no events
    g = gpu_run(sm, ctx, ev.concat([]))
    assert list(g[0]) == [0] and list(g[2]) == [0]
    # empty events around a real one, an event with no VELO states
    one = ev.generate(ev.config(1)).event(0)
    novelo = ev.generate(ev.config(1, first_event=1)).event(0)
    novelo.velo_off = np.array([0, 0], np.int32)
    for k in ("velo_x", "velo_y", "velo_z", "velo_tx", "velo_ty"):
        setattr(novelo, k, np.zeros(0, np.float32))
    novelo.velo_id = np.zeros(0, np.int32)
    b = ev.concat([empty, one, empty, novelo, empty])
    g = gpu_run(sm, ctx, b)
    o = orc.run(b)
    st = PT.compare(o, g, b.n_events)
    PT.assert_parity(st)
    assert st["seeds_g"] > 0 and g[2][-1] == o.long_off[-1]
    # only one half populated
    oneh = ev.generate(ev.config(2, n_events=1)).event(0)
    x = oneh.zone_off.copy()
    x[12:] = x[12]
    oneh.zone_off = x
    n = int(x[-1])
    oneh.hit_x, oneh.hit_z, oneh.hit_id = oneh.hit_x[:n], oneh.hit_z[:n], oneh.hit_id[:n]
    g = gpu_run(sm, ctx, oneh)
    o = orc.run(oneh)
    PT.assert_parity(PT.compare(o, g, 1))


def test_capacity_error_and_retry(sm, ctx):
    b = ev.generate(ev.config(2, n_events=5))
    say("[gpu] capacity errors")
    db = sm.DeviceBatch(b)
    out = sm.DeviceOut(b.n_events, 3, 2)
    st = ctx.run(db, out, check=False)
    assert st == sm.ERR_CAPACITY
    ns, nl = out.n_seeds, out.n_longs
    assert ns > 3 and nl > 2
    out2 = sm.DeviceOut(b.n_events, ns, nl)
    assert ctx.run(db, out2, check=False) == sm.OK
    assert out2.n_seeds == ns and out2.n_longs == nl
    g = out2.to_host()
    g2 = gpu_run(sm, ctx, b)
    for x, y in zip(g, g2):
        assert x.tobytes() == y.tobytes()


def test_scratch_growth(orc, sm):
    """A context with tiny scratch grows it and re-runs; results unchanged."""
    b = ev.generate(ev.config(4, n_events=8))
    say("[gpu] scratch growth")
    c = sm.Context(seed_wgs=16)
    try:
        g = gpu_run(sm, c, b)
    finally:
        c.close()
    o = orc.run(b, threads=8)
    PT.assert_parity(PT.compare(o, g, b.n_events, band=(
        orc.run(b, PT.eps_params(orc, 1e-4), threads=8),
        orc.run(b, PT.eps_params(orc, -1e-4), threads=8))))


def test_uneven_full_size(orc, sm, ctx):
    """The uneven workload at its own size: 10,000 events in one batch."""
    b = ev.generate(ev.config(3))
    say("[gpu] uneven hits/event range", int(b.event_hits().min()), int(b.event_hits().max()))
    check(orc, sm, ctx, b, "uneven 10000")


def test_stress_batch_with_oracle_subset(orc, sm, ctx):
    """A 5000-event stress batch on the GPU; the oracle checks events 0..499
    (events are independent, so a subset of the batch's outputs is the
    subset's result)."""
    b = ev.generate(ev.config(4, n_events=5000))
    say("[gpu] stress 5000, hits/event max", int(b.event_hits().max()))
    g = gpu_run(sm, ctx, b)
    n = 500
    sub = b.subset(range(n))
    gs = (g[0][:n + 1], g[1][:g[0][n]], g[2][:n + 1], g[3][:g[2][n]])
    o = orc.run(sub, threads=8)
    st = PT.compare(o, gs, n)
    if st["mismatches"]:
        st = PT.compare(o, gs, n, band=(orc.run(sub, PT.eps_params(orc, 1e-4), threads=8),
                                        orc.run(sub, PT.eps_params(orc, -1e-4), threads=8)))
    say(f"[gpu] stress subset: seeds {st['seeds_o']}/{st['seeds_g']} mismatches {st['mismatches']}")
    PT.assert_parity(st)


def test_stress_full_size_and_tiled(orc, sm, ctx):
    """The stress workload at its stated size: 50,000 events in one batch,
    the oracle on events 0..499; then the same events twice over in one
    100,000-event batch (offsets shifted on the device), whose two copies
    must each equal the single batch's outputs byte for byte."""
    import torch
    b = ev.generate_parallel(ev.config(4), 16)
    assert b.n_events == 50000
    say("[gpu] stress 50000, hits", b.n_hits, "max per event", int(b.event_hits().max()))
    db = sm.DeviceBatch(b)
    out = sm.DeviceOut(b.n_events, b.n_hits // 8 + 1024, b.n_velo + 1024)
    assert ctx.run(db, out) == sm.OK
    g = out.to_host()
    n = 500
    sub = b.subset(range(n))
    gs = (g[0][:n + 1], g[1][:g[0][n]], g[2][:n + 1], g[3][:g[2][n]])
    o = orc.run(sub, threads=8)
    st = PT.compare(o, gs, n)
    if st["mismatches"]:
        st = PT.compare(o, gs, n, band=(orc.run(sub, PT.eps_params(orc, 1e-4), threads=8),
                                        orc.run(sub, PT.eps_params(orc, -1e-4), threads=8)))
    say(f"[gpu] stress 50000 subset: seeds {st['seeds_o']}/{st['seeds_g']} "
        f"mismatches {st['mismatches']}")
    PT.assert_parity(st)
    # two copies of the batch in one
    nh, nv = db.n_hits, db.n_velo

    def twice(a):
        return torch.cat([a, a])

    def offs(a, step):
        a = a.to(torch.int64)
        return torch.cat([a[:-1], a + step]).to(torch.int32)

    t = dict(zone_off=offs(db.zone_off, nh), velo_off=offs(db.velo_off, nv),
             hit_x=twice(db.hit_x), hit_z=twice(db.hit_z), hit_id=twice(db.hit_id),
             **{"velo_" + k: twice(getattr(db, "velo_" + k)) for k in ("x", "y", "z", "tx", "ty", "id")})
    tb = sm.Batch(n_events=2 * b.n_events, pad=0, n_hits=2 * nh, n_velo=2 * nv, n_ut=0,
                  ut_off=None, ut_x=None, ut_id=None, **{k: v.data_ptr() for k, v in t.items()})
    out2 = sm.DeviceOut(2 * b.n_events, 2 * out.n_seeds + 1024, 2 * out.n_longs + 1024)
    ctx.run_c(tb, out2.c)
    say(f"[gpu] stress 100000 (two copies): seeds {out2.n_seeds} longs {out2.n_longs}")
    assert out2.n_seeds == 2 * out.n_seeds and out2.n_longs == 2 * out.n_longs
    g2 = out2.to_host()
    for k in range(2):
        for a, a2, cnt in ((g[1], g2[1], out.n_seeds), (g[3], g2[3], out.n_longs)):
            assert a2[k * cnt:(k + 1) * cnt].tobytes() == a.tobytes()
        for off, off2 in ((g[0], g2[0]), (g[2], g2[2])):
            seg = off2[k * b.n_events:(k + 1) * b.n_events + 1].astype(np.int64)
            assert np.array_equal(seg - seg[0], off.astype(np.int64))
    del db, out, out2, t
    torch.cuda.empty_cache()


def test_tied_hit_positions(orc, sm, ctx):
    """Hits with identical x in a zone: window and closest-hit choices follow
    the lower position, as in the oracle."""
    base = ev.generate(ev.config(1, n_events=3))
    evs = []
    for e in range(3):
        E = base.event(e)
        x = E.hit_x.copy()
        # duplicate every hit of every other zone (same x, new id), keep sorting
        hx, hz, hid, off = [], [], [], [0]
        nid = E.n_hits
        for k in range(24):
            lo, hi = E.zone_off[k], E.zone_off[k + 1]
            for i in range(lo, hi):
                hx.append(x[i]); hz.append(E.hit_z[i]); hid.append(E.hit_id[i])
                if k % 2 == 0:
                    hx.append(x[i]); hz.append(E.hit_z[i]); hid.append(nid); nid += 1
            off.append(len(hx))
        E.zone_off = np.array(off, np.int32)
        E.hit_x = np.array(hx, np.float32)
        E.hit_z = np.array(hz, np.float32)
        E.hit_id = np.array(hid, np.int32)
        evs.append(E)
    b = ev.concat(evs)
    say("[gpu] tied hits")
    g = gpu_run(sm, ctx, b)
    o = orc.run(b)
    st = PT.compare(o, g, b.n_events)
    PT.assert_parity(st)
    assert st["mismatches"] == 0 and st["seeds_g"] > 0


def test_noise_only_event(orc, sm, ctx):
    cfg = ev.GenConfig(n_events=4, config_id=301, mult="fixed", mean_tracks=1, noise=400.0)
    b = ev.generate(cfg)
    say("[gpu] noise-dominated events", b.n_hits)
    g = gpu_run(sm, ctx, b)
    o = orc.run(b)
    PT.assert_parity(PT.compare(o, g, b.n_events))


def test_item_hit_limit(sm, ctx):
    """An (event, half) with 2^21 hits is refused with SM_ERR_LIMIT."""
    n = 1 << 21
    off = np.zeros(25, np.int32)
    off[1:] = n                      # every hit in zone 0 (half 0, layer 0)
    b = ev.Batch(zone_off=off, hit_x=np.sort(np.random.default_rng(0).uniform(-3000, 3000, n)).astype(np.float32),
                 hit_z=np.full(n, 7826.0, np.float32), hit_id=np.arange(n, dtype=np.int32),
                 velo_off=np.array([0, 0], np.int32), velo_x=np.zeros(0, np.float32),
                 velo_y=np.zeros(0, np.float32), velo_z=np.zeros(0, np.float32),
                 velo_tx=np.zeros(0, np.float32), velo_ty=np.zeros(0, np.float32),
                 velo_id=np.zeros(0, np.int32))
    say("[gpu] hit limit")
    db = sm.DeviceBatch(b)
    out = sm.DeviceOut(1, 1024, 1024)
    assert ctx.run(db, out, check=False) == sm.ERR_LIMIT
    # the context still works afterwards
    b2 = ev.generate(ev.config(1))
    g = gpu_run(sm, ctx, b2)
    assert g[0][-1] > 0


HOUGH_OFF = ("the Hough-cluster UV kernel is switched off in sm_create: one run of "
             "test_hough_uv_deterministic (5-workgroup context) ended in a GPU memory "
             "aperture fault whose cause is not found yet")


@pytest.mark.skip(reason=HOUGH_OFF)
@pytest.mark.parametrize("cfgn,n", [(2, 300), (3, 200), (4, 40)])
def test_hough_uv_parity(orc, sm, cfgn, n):
    """The Hough-cluster UV variant (Sec. 3.4) against the oracle's."""
    b = ev.generate(ev.config(cfgn, n_events=n))
    c = sm.Context(params=sm.default_params(uv_mode=1))
    try:
        check(orc, sm, c, b, f"hough uv config {cfgn} x {n}", params_over=dict(uv_mode=1))
    finally:
        c.close()


@pytest.mark.skip(reason=HOUGH_OFF)
def test_hough_uv_deterministic(sm):
    """Fixed-point fine-bin sums: the same bytes for any grid shape and in the
    per-event (plain) form."""
    b = ev.generate(ev.config(3, n_events=60))
    say("[gpu] hough determinism")
    p = sm.default_params(uv_mode=1)
    c1, c2 = sm.Context(params=p), sm.Context(params=p, seed_wgs=5, lds_hits=1024)
    try:
        g1 = gpu_run(sm, c1, b)
        g2 = gpu_run(sm, c2, b)
        g3 = gpu_run(sm, c1, b, plain=True)
    finally:
        c1.close()
        c2.close()
    for x, y, z in zip(g1, g2, g3):
        assert x.tobytes() == y.tobytes() == z.tobytes()


def test_hough_uv_refused(sm):
    """While its kernel is switched off, uv_mode 1 is refused up front."""
    with pytest.raises(sm.SmError) as e:
        sm.Context(params=sm.default_params(uv_mode=1))
    assert e.value.status == sm.ERR_INVALID


def big_item_batch():
    """40 min-bias events around the largest event of the first 200 stress
    events, so that one item would outlast the rest of the batch."""
    stress = ev.generate(ev.config(4, n_events=200))
    sizes = np.diff(stress.zone_off[::12].astype(np.int64))
    e = int(np.argmax(sizes)) // 2
    mb = ev.generate(ev.config(2, n_events=40))
    return ev.concat([mb.event(i) for i in range(20)] + [stress.event(e)] +
                     [mb.event(i) for i in range(20, 40)])


def test_big_items_batched_equals_plain(sm, ctx):
    """A dominating item runs in the big-item form (1024-thread workgroup,
    own scratch) in the batched call and in the 256-thread form in the
    per-event call; both give the same bytes, and the oracle agrees."""
    b = big_item_batch()
    sizes = np.diff(b.zone_off[::12].astype(np.int64))
    say("[gpu] big items: largest item", int(sizes.max()), "hits")
    assert sizes.max() >= 8191
    g1 = gpu_run(sm, ctx, b)
    g2 = gpu_run(sm, ctx, b, plain=True)
    for x, y in zip(g1, g2):
        assert x.tobytes() == y.tobytes()


def test_big_items_parity(orc, sm, ctx):
    b = big_item_batch()
    check(orc, sm, ctx, b, "batch with a dominating item")


@pytest.mark.parametrize("batch", ["minbias", "big"])
def test_matching_kernel_equals_fused(sm, ctx, batch):
    """Matching in a kernel of its own after all seeding, and matching inside
    the seeding kernel by the workgroup that completes an event, give the
    same bytes: on min-bias (automatic choice: the matching kernel) and on a
    batch with a big item (automatic choice: inside), each forced both ways,
    also with one matching workgroup and with fewer workgroups than events."""
    b = ev.generate(ev.config(2, n_events=300)) if batch == "minbias" else big_item_batch()
    say(f"[gpu] matching kernel vs fused, {batch}: {b.n_events} events")
    g0 = gpu_run(sm, ctx, b)
    for mw in (-1, 1, 37, 4096):
        c = sm.Context(match_wgs=mw)
        try:
            g = gpu_run(sm, c, b)
        finally:
            c.close()
        for x, y in zip(g0, g):
            assert x.tobytes() == y.tobytes(), mw


@pytest.mark.parametrize("p_min", [1500.0, 2000.0, 5000.0])
def test_p_min_scan(orc, sm, p_min):
    """The window constants follow the minimum momentum (eq. tolHp, eq.
    alphacorr): parity at several p_min on min-bias events, and fewer seeds
    as p_min rises."""
    b = ev.generate(ev.config(2, n_events=100))
    c = sm.Context(params=sm.default_params(p_min=p_min))
    try:
        g, o, st = check(orc, sm, c, b, f"p_min {p_min / 1000:.1f} GeV", params_over=dict(p_min=p_min))
    finally:
        c.close()
    ref = orc.run(b, orc.default_params(), threads=8)
    if p_min < 3000.0:
        assert st["seeds_g"] >= len(ref.seeds)
    else:
        assert st["seeds_g"] <= len(ref.seeds)


def test_validating_sequence_equals_default(sm, ctx):
    """With input validation on, the batch runs k_prepare, k_validate and the
    big form as separate launches (the default prepares inside the big-form
    launch); both give the same bytes, and validation rejects an unsorted
    zone."""
    b = ev.generate(ev.config(2, n_events=60))
    say("[gpu] validating sequence vs default, 60 events")
    g0 = gpu_run(sm, ctx, b)
    c = sm.Context(validate=True)
    try:
        g1 = gpu_run(sm, c, b)
        for x, y in zip(g0, g1):
            assert x.tobytes() == y.tobytes()
        bad = b.subset(range(3))
        zo = bad.zone_off
        L = next(k for k in range(12) if zo[k + 1] - zo[k] >= 2)
        i = int(zo[L])
        bad.hit_x[i], bad.hit_x[i + 1] = bad.hit_x[i + 1] + 1.0, bad.hit_x[i]
        with pytest.raises(sm.SmError) as e:
            gpu_run(sm, c, bad)
        assert e.value.status == sm.ERR_UNSORTED
        g2 = gpu_run(sm, c, b)   # the context stays usable
        for x, y in zip(g0, g2):
            assert x.tobytes() == y.tobytes()
    finally:
        c.close()


def _ghost_random_net(orc, b, loose):
    """A random network standardised by the surviving pairs' own spread (from
    the oracle), with small output weights: probabilities fall on both sides
    of the cut and close to each other, so that many cut and clone decisions
    occur."""
    p = orc.default_params(**loose)
    r0 = orc.run(b, params=p, threads=8)
    F = []
    for e in range(b.n_events):
        v0, v1 = int(b.velo_off[e]), int(b.velo_off[e + 1])
        velo = {"x": b.velo_x[v0:v1], "y": b.velo_y[v0:v1], "z": b.velo_z[v0:v1],
                "tx": b.velo_tx[v0:v1], "ty": b.velo_ty[v0:v1]}
        F.append(orc.match_pairs(r0.event_seeds(e), velo, params=p)["f"])
    F = np.concatenate(F)
    rng = np.random.default_rng(11)
    return {"mean": F.mean(0).tolist(), "scale": F.std(0).tolist(),
            "w1": rng.normal(0, 1, (32, 8)).tolist(), "b1": rng.normal(0, 0.5, 32).tolist(),
            "w2": rng.normal(0, 0.125, 32).tolist(), "b2": 0.5}


@pytest.mark.parametrize("net", ["shipped", "random"])
def test_ghost_network_selection(orc, sm, ctx, net):
    """The network form of the final selection (Sec. 4.4) against the oracle:
    the shipped weights on 300 min-bias events, and a random network under
    loose matching cuts (thousands of cut and clone decisions) on 100 events.
    Long tracks and their ghost probabilities agree; the batched and the
    per-event forms give the same bytes."""
    if net == "shipped":
        b = ev.generate(ev.config(2, n_events=300))
        over = dict(final_sel=1, ghost_nn=sm.ghost_nn_weights())
    else:
        b = ev.generate(ev.config(2, n_events=100))
        loose = dict(chi2m_max=500.0, max_dx=200.0, max_dy=600.0, max_dty=0.08)
        over = dict(final_sel=1, ghost_nn=_ghost_random_net(orc, b, loose), **loose)
    c = sm.Context(params=sm.default_params(**over))
    try:
        g, o, st = check(orc, sm, c, b, f"ghost network ({net})", params_over=over)
        assert st["longs_common"] > 10000 if net == "shipped" else st["longs_common"] > 1000
        dmax = 0.0
        for e in range(b.n_events):
            osd, old = PT.event_sets(o.seed_off, o.seeds, o.long_off, o.longs, e, "id")
            gsd, gld = PT.event_sets(g[0], g[1], g[2], g[3], e, "hits")
            for k in old.keys() & gld.keys():
                dmax = max(dmax, abs(float(old[k]["gp"]) - float(gld[k]["ghost_prob"])))
        say(f"[gpu] ghost network ({net}): largest ghost-probability difference {dmax:.3g}")
        gp = g[3]["ghost_prob"]
        assert np.all((gp >= 0) & (gp < 0.8))
        gpl = gpu_run(sm, c, b, plain=True)
        for x, y in zip(g, gpl):
            assert x.tobytes() == y.tobytes()
    finally:
        c.close()
    if net == "shipped":
        # the chi2 form keeps at most one track per VELO state and seed; the
        # network form may keep near-equal pairs on one segment
        ref = gpu_run(sm, ctx, b)
        assert np.all(ref[3]["ghost_prob"] == -1.0)


@pytest.mark.parametrize("variant", ["ut", "ut+ghost"])
def test_ut_search_parity(orc, sm, ctx, variant):
    """The UT hit search (Sec. 4.3) against the oracle on 300 min-bias events
    with UT hits: long tracks, their UT hit ids and counts; alone and with the
    network form of the final selection.  Matching in its own kernel and
    inside the seeding kernel, and the per-event form, give the same bytes.
    Without UT hits in the batch the call is refused."""
    b = ev.generate(ev.config(2, n_events=300))
    over = dict(ut_mode=1)
    if variant == "ut+ghost":
        over.update(final_sel=1, ghost_nn=sm.ghost_nn_weights())
    c = sm.Context(params=sm.default_params(**over))
    try:
        g, o, st = check(orc, sm, c, b, f"UT search ({variant})", params_over=over)
        assert st["longs_common"] > 10000
        assert np.all(g[3]["n_ut"] >= 3)
        assert np.all((g[3]["ut_hits"] >= 0).sum(axis=1) == g[3]["n_ut"])
        gpl = gpu_run(sm, c, b, plain=True)
        for x, y in zip(g, gpl):
            assert x.tobytes() == y.tobytes()
        with pytest.raises(sm.SmError):
            gpu_run(sm, c, b.without_ut())
    finally:
        c.close()
    cf = sm.Context(params=sm.default_params(**over), match_wgs=-1)
    try:
        gf = gpu_run(sm, cf, b)
        for x, y in zip(g, gf):
            assert x.tobytes() == y.tobytes()
    finally:
        cf.close()
    # the default context ignores the UT hits
    ref = gpu_run(sm, ctx, b)
    assert np.all(ref[3]["n_ut"] == 0) and np.all(ref[3]["ut_hits"] == -1)
    assert len(ref[3]) > len(g[3])


def test_large_batch_matching_kernel(orc, sm):
    """Batches of up to 4096 events have their seeds written by the matching
    kernel, larger ones by the copy kernel: 4200 min-bias events forced
    through the matching kernel against the oracle, and the same bytes with
    matching inside the seeding kernel."""
    b = ev.generate(ev.config(2, n_events=4200))
    c = sm.Context(match_wgs=1024)
    try:
        g, _, _ = check(orc, sm, c, b, "4200 events, matching kernel")
    finally:
        c.close()
    c = sm.Context(match_wgs=-1)
    try:
        g2 = gpu_run(sm, c, b)
    finally:
        c.close()
    for x, y in zip(g, g2):
        assert x.tobytes() == y.tobytes()


def test_third_iteration_parity(orc, sm):
    """The third x-z iteration with clean-up against the oracle on 300
    min-bias events: the first two iterations' seeds, the third's (iteration
    2, on the hits they left), and the long tracks over all of them; the same
    bytes on another grid and LDS budget; the per-event form refuses it."""
    b = ev.generate(ev.config(2, n_events=300))
    over = dict(third_iter=1)
    c = sm.Context(params=sm.default_params(**over))
    try:
        g, o, st = check(orc, sm, c, b, "third iteration", params_over=over)
        assert (g[1]["iter"] == 2).sum() > 1000
        with pytest.raises(sm.SmError):
            gpu_run(sm, c, b, plain=True)
    finally:
        c.close()
    c2 = sm.Context(params=sm.default_params(**over), seed_wgs=300, lds_hits=1024)
    try:
        g2 = gpu_run(sm, c2, b)
        for x, y in zip(g, g2):
            assert x.tobytes() == y.tobytes()
    finally:
        c2.close()
