"""Comparison of the HIP library's outputs with the FP64 oracle's.

Tracks are matched by identity, not by position in the lists: a seed by its
12 hit ids, a long track by (VELO index, seed hit ids).  The bar:
  - |O & G| / |O | G| >= 0.999 for seeds and for long tracks;
  - every track in the symmetric difference lies within 1e-4 of a decision:
    the oracle's margin log puts an oracle-only track's closest decision
    within MARGIN of going the other way, or lists a GPU-only track (or its
    x-z part, or the seed or the VELO state of a GPU-only long track) as a
    near miss or next to an oracle track within MARGIN; failing that, its
    membership changes when the oracle's thresholds are scaled by 1 +- 1e-4;
  - parameters of matched tracks within 1e-4 relative, with an absolute floor
    where FP32 storage makes a relative bound meaningless (stated per field).
"""
from __future__ import annotations

import numpy as np

# (field in oracle seed, field in GPU seed, rel tol, abs floor)
SEED_FIELDS = [("a", "ax", 1e-4, 1e-3), ("b", "bx", 1e-4, 1e-7), ("c", "cx", 1e-4, 5e-10),
               ("y0", "y0", 1e-4, 1e-3), ("ty", "ty", 1e-4, 1e-7),
               ("chi2x", "chi2_x", 1e-4, 1e-3), ("chi2y", "chi2_y", 1e-4, 1e-3)]
LONG_FIELDS = [("qop", "qop", 1e-4, 1e-10), ("chi2", "chi2", 1e-4, 1e-3),
               ("zm", "z_match", 1e-4, 1e-2), ("dx", "dx", 1e-4, 2e-3),
               ("dy", "dy", 1e-4, 2e-2), ("dtx", "dtx", 1e-4, 1e-6), ("dty", "dty", 1e-4, 1e-6),
               ("gp", "ghost_prob", 1e-4, 1e-4)]

MARGIN = 1e-4

THRESHOLDS = ["t2_tol0", "t2_tol1", "ext_tol", "chi2x_max", "uv_tol", "y_max", "chi2y_max",
              "max_dx", "max_dy", "max_dtx", "max_dty", "chi2m_max"]


def eps_params(orc, eps, **over):
    """Oracle params with every threshold scaled by (1 + eps) and the momentum
    window opened by the same relative amount."""
    p = orc.default_params(**over)
    for k in THRESHOLDS:
        setattr(p, k, getattr(p, k) * (1.0 + eps))
    p.p_min = p.p_min * (1.0 - eps)
    return p


def _seed_key(ids):
    return tuple(int(i) for i in ids)


def event_sets(seed_off, seeds, long_off, longs, e, id_field):
    S = seeds[seed_off[e]:seed_off[e + 1]]
    L = longs[long_off[e]:long_off[e + 1]]
    skeys = [_seed_key(s[id_field]) for s in S]
    sd = {k: s for k, s in zip(skeys, S)}
    ld = {}
    for l in L:
        ld[(int(l["velo_idx"]), skeys[int(l["seed_idx"])])] = l
    return sd, ld


INIT_LAYERS = ((0, 4, 8), (3, 7, 11))


def _origin(key, it):
    """The three-hit combination a seed descends from: its x-z iteration and
    its hits on that iteration's initial layers."""
    return (int(it),) + tuple(key[l] for l in INIT_LAYERS[int(it)])


def _seed_explained(orc_res, e, osd, gsd, k):
    if k in osd:
        return float(osd[k]["margin"]) < MARGIN
    org = _origin(k, gsd[k]["iter"])
    for r in orc_res.event_near(e):
        if r["margin"] >= MARGIN:
            continue
        ids = tuple(int(i) for i in r["id"])
        if (r["kind"] == 3 and ids == k) or \
                (r["kind"] in (1, 2, 3) and _origin(ids, r["it"]) == org):
            return True
    # the oracle's descendant of the same three-hit combination was decided
    # near a threshold (a different extension hit, stereo choice or cut)
    return any(_origin(o, s["it"]) == org and float(s["margin"]) < MARGIN for o, s in osd.items())


def margin_explains(orc_res, e, osd, old, gsd, gld, k, what):
    """True if the oracle's margin log explains mismatch k of event e."""
    if what == "seed":
        return _seed_explained(orc_res, e, osd, gsd, k)
    v, sk = k
    if k in old:
        return float(old[k]["margin"]) < MARGIN
    for r in orc_res.event_near(e):
        if r["kind"] == 4 and r["margin"] < MARGIN and int(r["velo_idx"]) == v and \
                tuple(int(i) for i in r["id"]) == sk:
            return True
    # its seed is itself a mismatch explained by the log, or an oracle long
    # track on its VELO state or on the same seed lineage was decided near a cut
    if sk not in osd and _seed_explained(orc_res, e, osd, gsd, sk):
        return True
    org = _origin(sk, gsd[sk]["iter"])
    return any((ov == v or _origin(os_, osd[os_]["it"]) == org) and float(l["margin"]) < MARGIN
               for (ov, os_), l in old.items())


def _close(x, y, rel, floor):
    return abs(float(x) - float(y)) <= max(rel * max(abs(float(x)), abs(float(y))), floor)


def compare(orc_res, gpu, n_events, band=None, events=None):
    """gpu = (seed_off, seeds, long_off, longs) from the library; band =
    (loose, tight) oracle results for the near-cut test, or None; events:
    the event indices to compare (default: all n_events)."""
    so, sg, lo, lg = gpu
    st = dict(seeds_o=0, seeds_g=0, seeds_common=0, longs_o=0, longs_g=0, longs_common=0,
              param_fail=[], unexplained=[], mismatches=0)
    for e in (range(n_events) if events is None else events):
        osd, old = event_sets(orc_res.seed_off, orc_res.seeds, orc_res.long_off, orc_res.longs,
                              e, "id")
        gsd, gld = event_sets(so, sg, lo, lg, e, "hits")
        st["seeds_o"] += len(osd)
        st["seeds_g"] += len(gsd)
        st["longs_o"] += len(old)
        st["longs_g"] += len(gld)
        common = osd.keys() & gsd.keys()
        st["seeds_common"] += len(common)
        for k in common:
            for fo, fg, rel, fl in SEED_FIELDS:
                if not _close(osd[k][fo], gsd[k][fg], rel, fl):
                    st["param_fail"].append(("seed", e, fo, float(osd[k][fo]), float(gsd[k][fg])))
            if int(osd[k]["nx"]) != int(gsd[k]["n_x"]) or int(osd[k]["nuv"]) != int(gsd[k]["n_uv"]):
                st["param_fail"].append(("seed", e, "n", int(osd[k]["nx"]), int(gsd[k]["n_x"])))
        lcommon = old.keys() & gld.keys()
        st["longs_common"] += len(lcommon)
        for k in lcommon:
            for fo, fg, rel, fl in LONG_FIELDS:
                if not _close(old[k][fo], gld[k][fg], rel, fl):
                    st["param_fail"].append(("long", e, fo, float(old[k][fo]), float(gld[k][fg])))
            if int(old[k]["velo_id"]) != int(gld[k]["velo_id"]):
                st["param_fail"].append(("long", e, "velo_id", 0, 0))
            # UT hits (ut_mode 1): the same hits, unless a UT choice of the
            # track was within MARGIN of going the other way
            if "ut_hits" in gld[k].dtype.names:
                same = int(old[k]["n_ut"]) == int(gld[k]["n_ut"]) and \
                    list(old[k]["ut_id"]) == list(gld[k]["ut_hits"])
                if not same and not float(old[k]["margin"]) < MARGIN:
                    st["param_fail"].append(("long", e, "ut_hits", list(old[k]["ut_id"]),
                                             list(gld[k]["ut_hits"])))
        diff_s = (osd.keys() ^ gsd.keys())
        diff_l = (old.keys() ^ gld.keys())
        st["mismatches"] += len(diff_s) + len(diff_l)
        if diff_s or diff_l:
            if hasattr(orc_res, "near"):
                ms = {k for k in diff_s if margin_explains(orc_res, e, osd, old, gsd, gld, k, "seed")}
                # the third iteration runs on the hits the first two left in
                # the half: a change among their seeds there carries over
                it_half = lambda k: ((int(osd[k]["it"]), int(osd[k]["half"])) if k in osd
                                     else (int(gsd[k]["iter"]), int(gsd[k]["half"])))
                moved = {it_half(k)[1] for k in ms if it_half(k)[0] < 2}
                ms |= {k for k in diff_s - ms if it_half(k)[0] == 2 and it_half(k)[1] in moved}
                ml = {k for k in diff_l
                      if k[1] in ms or margin_explains(orc_res, e, osd, old, gsd, gld, k, "long")}
                st["explained_by_margin"] = st.get("explained_by_margin", 0) + len(ms) + len(ml)
                diff_s, diff_l = diff_s - ms, diff_l - ml
            if not (diff_s or diff_l):
                continue
            if band is None:
                st["unexplained"] += [("seed", e, k) for k in diff_s] + [("long", e, k) for k in diff_l]
                continue
            loose, tight = band
            lsd, lld = event_sets(loose.seed_off, loose.seeds, loose.long_off, loose.longs, e, "id")
            tsd, tld = event_sets(tight.seed_off, tight.seeds, tight.long_off, tight.longs, e, "id")
            for k in diff_s:
                flips = len({k in osd, k in lsd, k in tsd}) > 1
                if not flips:
                    st["unexplained"].append(("seed", e, k))
            for k in diff_l:
                flips = len({k in old, k in lld, k in tld}) > 1
                if not flips:
                    st["unexplained"].append(("long", e, k))
    us = st["seeds_o"] + st["seeds_g"] - st["seeds_common"]
    ul = st["longs_o"] + st["longs_g"] - st["longs_common"]
    st["seed_jaccard"] = st["seeds_common"] / us if us else 1.0
    st["long_jaccard"] = st["longs_common"] / ul if ul else 1.0
    return st


def assert_parity(st, min_jaccard=0.999):
    assert st["seed_jaccard"] >= min_jaccard, st
    assert st["long_jaccard"] >= min_jaccard, st
    assert not st["unexplained"], st["unexplained"][:10]
    assert not st["param_fail"], st["param_fail"][:10]
