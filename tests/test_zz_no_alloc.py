"""The allocation-free entry point (sm_run_noalloc) against sm_run, through
the C-ABI (needs an MI355X).

Two calls in a row on the device's static scratch, the second with a smaller
batch, each byte-identical to sm_run on the same batch; the second also
against the FP64 oracle.  A batch above the call's event limit is refused
before any launch.
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


def run_both(sm, ctx, b):
    db = sm.DeviceBatch(b)
    ref = sm.DeviceOut(b.n_events, max(b.n_hits // 4, 16), max(b.n_velo * 2, 16))
    ctx.run(db, ref)
    out = sm.DeviceOut(b.n_events, max(b.n_hits // 4, 16), max(b.n_velo * 2, 16))
    # poison the outputs so that stale or unwritten bytes cannot pass
    out.seeds.fill_(0xA5)
    out.longs.fill_(0x5A)
    out.seed_off.fill_(-7)
    out.long_off.fill_(-7)
    ctx.run_noalloc(db, out)
    return ref, out


def assert_same(ref, out):
    assert out.n_seeds == ref.n_seeds and out.n_longs == ref.n_longs
    ro, rs, rlo, rl = ref.to_host()
    oo, os_, olo, ol = out.to_host()
    np.testing.assert_array_equal(oo, ro)
    np.testing.assert_array_equal(olo, rlo)
    assert os_.tobytes() == rs.tobytes()
    assert ol.tobytes() == rl.tobytes()


def test_noalloc_equals_run_twice(orc, sm):
    ctx = sm.Context()
    try:
        b1 = ev.generate(ev.config(3, n_events=400))     # uneven: items on both hit paths
        say(f"[gpu] noalloc call 1: uneven {b1.n_events} events, {b1.n_hits} hits")
        ref1, out1 = run_both(sm, ctx, b1)
        assert_same(ref1, out1)
        assert out1.n_seeds > 0 and out1.n_longs > 0
        b2 = ev.generate(ev.config(2, n_events=150))     # smaller, after the first
        say(f"[gpu] noalloc call 2: min-bias {b2.n_events} events, {b2.n_hits} hits")
        ref2, out2 = run_both(sm, ctx, b2)
        assert_same(ref2, out2)
        o = orc.run(b2, orc.default_params(), threads=8)
        st = PT.compare(o, out2.to_host(), b2.n_events)
        say(f"[gpu] noalloc call 2 vs oracle: {st}")
        PT.assert_parity(st)
        assert st["mismatches"] == 0
    finally:
        ctx.close()


def test_noalloc_limits(sm):
    ctx = sm.Context()
    try:
        n = sm.NOALLOC_MAX_EVENTS + 1
        b = ev.concat([ev.empty_event() for _ in range(n)])
        say(f"[gpu] noalloc limit: {n} empty events")
        db = sm.DeviceBatch(b)
        out = sm.DeviceOut(n, 16, 16)
        assert ctx.run_noalloc(db, out, check=False) == sm.ERR_LIMIT
        # the same batch runs through sm_run, and the call after the refusal works
        assert ctx.run(db, out, check=False) == sm.OK
        b2 = ev.generate(ev.config(2, n_events=20))
        ref2, out2 = run_both(sm, ctx, b2)
        assert_same(ref2, out2)
    finally:
        ctx.close()
