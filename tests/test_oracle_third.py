"""Pins of the oracle's third x-z iteration with clean-up (Sec. 3: the HLT2
form reconstructs high momenta first, cleans the environment and searches
again with wider windows for lower momenta).

- The third iteration's window constants equal the values worked by hand at
  its 1.5 GeV/c floor (tests/golden/window_constants_third_iteration.txt).
- The clean-up: no third-iteration seed shares a hit with a seed of the first
  two iterations of its event half.
- An independent route: the event rebuilt in Python without the hits of the
  first two iterations' seeds, then the oracle's own x-z stage for iteration
  2 on it; every third-iteration seed's x hits form one of that stage's
  candidates.
- Generator truth: the third iteration finds tracks below the 3 GeV/c floor
  of the first two (their efficiency rises a lot) and leaves the first two
  iterations' seeds unchanged.
"""
import os

import numpy as np
import pytest

from paper_2606_14480_amd import events as ev

HERE = os.path.dirname(os.path.abspath(__file__))


def test_window_constants_worked_values(orc):
    row = [l.split() for l in open(os.path.join(HERE, "golden", "window_constants_third_iteration.txt"))
           if l.strip() and not l.startswith("#")][0]
    p_min3, x0, dx3, alpha = (float(x) for x in row)
    p = orc.default_params(third_iter=1, p_min3=p_min3)
    got = orc.window_constants(2, p)
    assert got[0] == pytest.approx(dx3, abs=0.01)
    assert got[1] == pytest.approx(alpha, abs=0.01)
    assert got[0] == pytest.approx((9229.0 - 7826.0) / 7826.0 * x0, rel=1e-4)
    # iterations 0 and 1 keep the 3 GeV/c constants
    assert orc.window_constants(0, p)[0] == pytest.approx(392.5675, abs=1e-3)


@pytest.fixture(scope="module")
def runs(orc):
    b = ev.generate(ev.config(2, n_events=60))
    r0 = orc.run(b, threads=8)
    r1 = orc.run(b, orc.default_params(third_iter=1), threads=8)
    return b, r0, r1


def _ids(sd):
    return {int(h) for h in sd["id"] if h >= 0}


def test_first_two_iterations_unchanged_and_clean_up_holds(runs):
    b, r0, r1 = runs
    n3 = 0
    for e in range(b.n_events):
        s0, s1 = r0.event_seeds(e), r1.event_seeds(e)
        first = s1[s1["it"] < 2]
        assert sorted(map(tuple, first["id"])) == sorted(map(tuple, s0["id"]))
        for sd in s1[s1["it"] == 2]:
            n3 += 1
            mine = _ids(sd)
            for other in first[first["half"] == sd["half"]]:
                assert not (mine & _ids(other)), e
    assert n3 > 300


def test_third_iteration_equals_stage_on_cleaned_event(orc, runs):
    b, r0, r1 = runs
    p = orc.default_params(third_iter=1)
    n = 0
    for e in range(0, b.n_events, 3):
        E = b.event(e)
        s1 = r1.event_seeds(e)
        used = set()
        for sd in s1[s1["it"] < 2]:
            used |= _ids(sd)
        keep = np.array([int(h) not in used for h in E.hit_id])
        zo = np.concatenate([[0], np.cumsum([keep[E.zone_off[z]:E.zone_off[z + 1]].sum()
                                             for z in range(24)])]).astype(np.int32)
        C = ev.Batch(zone_off=zo, hit_x=E.hit_x[keep], hit_z=E.hit_z[keep], hit_id=E.hit_id[keep],
                     velo_off=E.velo_off, velo_x=E.velo_x, velo_y=E.velo_y, velo_z=E.velo_z,
                     velo_tx=E.velo_tx, velo_ty=E.velo_ty, velo_id=E.velo_id)
        for half in (0, 1):
            cands = orc.xz_candidates(C, half, 2, params=p)
            ok = cands[cands["status"] == 0]
            sets = {frozenset(int(C.hit_id[q]) for q in c["pos"] if q >= 0) for c in ok}
            for sd in s1[(s1["it"] == 2) & (s1["half"] == half)]:
                xs = frozenset(int(sd["id"][l]) for l in (0, 3, 4, 7, 8, 11) if sd["id"][l] >= 0)
                assert xs in sets, (e, half)
                n += 1
    assert n > 80


def test_truth_low_momentum_tracks_recovered(orc, runs):
    b, r0, r1 = runs
    t = b.truth

    def found(r):
        lo = hi = lo_all = hi_all = 0
        for e in range(b.n_events):
            t0, t1 = int(t["track_off"][e]), int(t["track_off"][e + 1])
            sets = [_ids(sd) for sd in r.event_seeds(e)]
            for k in range(t0, t1):
                own = {int(h) for h in t["hits"][k] if h >= 0}
                if len(own) < 10:
                    continue
                hit = any(len(s & own) >= 0.7 * len(s) and len(s & own) >= 8 for s in sets)
                if t["p"][k] < 3000.0:
                    lo_all += 1
                    lo += hit
                else:
                    hi_all += 1
                    hi += hit
        return lo / lo_all, hi / hi_all
    lo0, hi0 = found(r0)
    lo1, hi1 = found(r1)
    assert lo1 > lo0 + 0.2, (lo0, lo1)
    assert hi1 >= hi0
