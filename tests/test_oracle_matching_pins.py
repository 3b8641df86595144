"""Pins of the oracle's Matching (Sec. 4) with hand-built inputs.

Seeds are built from the generator's exact truth parameters and VELO states
from the truth line, then shifted by known amounts.  Straight-line geometry
fixes every residual: shifting the VELO state by dx0 in x moves Delta x at the
kink plane by -dx0 (z_match does not depend on the VELO position), by dy0 in
y moves Delta y at the y plane by -dy0, and tilting t_y by d (about the y
matching plane) moves only Delta t_y by -d.  That tests each cut from both
sides and each term of chi2_match separately, and the final selection on
hand-built conflicts.
"""
import numpy as np
import pytest

from paper_2606_14480_amd import events as ev


def truth_tracks(n=30, p=(1300.0, 2000.0), cid=401):
    cfg = ev.GenConfig(n_events=1, config_id=cid, mult="fixed", mean_tracks=n, p_range=p, sigma=0.0)
    return ev.generate(cfg)


def seeds_from_truth(orc, T, idx):
    from oracle.oracle import SEED_DTYPE
    s = np.zeros(len(idx), SEED_DTYPE)
    for k, t in enumerate(idx):
        s[k]["a"], s[k]["b"], s[k]["c"] = T["a"][t], T["b"][t], T["c"][t]
        s[k]["y0"], s[k]["ty"] = T["y0"][t], T["ty"][t]
        s[k]["id"] = -1
        s[k]["pos"] = -1
    return s


def velo(b, t, dx=0.0, dy=0.0, dty_at_ym=0.0, P=None):
    """VELO state of truth track t (the batch's own float32 state, mapped
    back to the track), shifted in x and y and with t_y tilted about the y
    matching plane."""
    T = b.truth
    v = int(T["velo"][t])
    x, y, z = float(b.velo_x[v]), float(b.velo_y[v]), float(b.velo_z[v])
    tx, ty = float(b.velo_tx[v]), float(b.velo_ty[v])
    zy = P.z_ymatch
    y_at = y + ty * (zy - z)
    ty2 = ty + dty_at_ym
    y2 = y_at - ty2 * (zy - z)
    return dict(x=[x + dx], y=[y2 + dy], z=[z], tx=[tx], ty=[ty2], id=[v])


def one(orc, seeds, vel, P):
    return orc.match(seeds, {k: np.array(v) for k, v in vel.items()}, P)


def test_residuals_follow_the_shifts(orc):
    b = truth_tracks(p=(4000.0, 6000.0), cid=406)
    P = orc.default_params()
    T = b.truth
    t = 0
    s = seeds_from_truth(orc, T, [t])
    base = one(orc, s, velo(b, t, P=P), P)
    assert len(base) == 1
    for dx in (-5.0, 4.0):
        r = one(orc, s, velo(b, t, dx=dx, P=P), P)[0]
        assert r["dx"] == pytest.approx(base[0]["dx"] - dx, abs=1e-4)
        assert r["dy"] == pytest.approx(base[0]["dy"], abs=1e-9)
        assert r["zm"] == pytest.approx(base[0]["zm"], abs=1e-9)
    for dy in (-1.0, 0.8):
        r = one(orc, s, velo(b, t, dy=dy, P=P), P)[0]
        assert r["dy"] == pytest.approx(base[0]["dy"] - dy, abs=1e-4)
        assert r["dx"] == pytest.approx(base[0]["dx"], abs=1e-9)
    r = one(orc, s, velo(b, t, dty_at_ym=0.003, P=P), P)[0]
    assert r["dty"] == pytest.approx(base[0]["dty"] - 0.003, abs=1e-7)
    assert r["dy"] == pytest.approx(base[0]["dy"], abs=1e-3)


def test_chi2_terms_and_cut(orc):
    """chi2_match = dx^2/tol_x + dy^2/tol_y + dtx^2/tol_tx + dty^2/tol_ty
    (Sec. 4.2): each term, added by its own shift, adds its own amount; the
    cut at 2 is strict."""
    b = truth_tracks(p=(3000.0, 6000.0), cid=402)
    P = orc.default_params()
    T = b.truth
    t = 0
    s = seeds_from_truth(orc, T, [t])
    r0 = one(orc, s, velo(b, t, P=P), P)[0]
    tx, ty = float(b.velo_tx[T["velo"][t]]), float(b.velo_ty[T["velo"][t]])
    dtx = r0["dtx"]
    tol_x = 0.8 * (10.12 ** 2 + 101.0 ** 2 * dtx ** 2)
    tol_ty = 1.0 / 937.5
    base = r0["chi2"]
    assert base == pytest.approx(dtx ** 2 / 0.5, rel=1e-6, abs=1e-6)
    rx = one(orc, s, velo(b, t, dx=3.0, P=P), P)[0]
    assert rx["chi2"] - base == pytest.approx((r0["dx"] - 3.0) ** 2 / tol_x - r0["dx"] ** 2 / tol_x, rel=1e-6)
    # t_y tilt changes rho, so compare the Delta t_y term with tol_y re-evaluated
    d = 0.01
    rt = one(orc, s, velo(b, t, dty_at_ym=d, P=P), P)[0]
    rho2 = tx * tx + (ty + d) ** 2
    tol_y2 = 0.2 * (1.59 ** 2 + 212.1 ** 2 * rho2)
    want = r0["dx"] ** 2 / tol_x + rt["dy"] ** 2 / tol_y2 + dtx ** 2 / 0.5 + rt["dty"] ** 2 / tol_ty
    assert rt["chi2"] == pytest.approx(want, rel=1e-6)
    assert rt["chi2"] - base > 0.08          # the Delta t_y term is there (~937.5 * 1e-4)
    # walk y until the pair is lost: |dy| < 150 mm never binds first, so the
    # edge is where chi2 reaches 2 (accepted strictly below)
    lo, hi = 0.0, 100.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if len(one(orc, s, velo(b, t, dy=mid, P=P), P)):
            lo = mid
        else:
            hi = mid
    edge = one(orc, s, velo(b, t, dy=lo, P=P), P)[0]
    assert abs(edge["dy"]) < 50.0
    assert 2.0 - 1e-4 < edge["chi2"] < 2.0


def test_preselection_edges(orc):
    """|dx| < 20 mm binds at large slope differences (low p); |dty| < 0.02
    binds before chi2 does (chi2 alone would allow |dty| up to 0.046)."""
    b = truth_tracks(p=(1300.0, 1400.0), cid=403)
    P = orc.default_params()
    T = b.truth
    t = 0
    s = seeds_from_truth(orc, T, [t])
    r0 = one(orc, s, velo(b, t, P=P), P)[0]
    assert abs(r0["dtx"]) > 0.8
    # Delta x = r0.dx - shift: place it just inside and just outside 20 mm
    for target, kept in ((19.99, True), (-19.99, True), (20.01, False), (-20.01, False)):
        r = one(orc, s, velo(b, t, dx=r0["dx"] - target, P=P), P)
        assert (len(r) == 1) == kept, target
        if kept:
            assert r[0]["dx"] == pytest.approx(target, abs=1e-4)
    b2 = truth_tracks(p=(20000.0, 30000.0), cid=404)
    T2 = b2.truth
    s2 = seeds_from_truth(orc, T2, [0])
    r1 = one(orc, s2, velo(b2, 0, P=P), P)[0]
    for target, kept in ((0.0199, True), (-0.0199, True), (0.0201, False), (-0.0201, False)):
        r = one(orc, s2, velo(b2, 0, dty_at_ym=r1["dty"] - target, P=P), P)
        assert (len(r) == 1) == kept, target


def test_final_selection_is_mutual_best(orc):
    """Sec. 4.4 reading: among the pairs that pass the cuts, a pair is kept
    only if its chi2 is the lowest of its seed's pairs and of its VELO
    track's pairs.  Every pair is scored alone (1 seed x 1 VELO state, no
    competition) and the rule applied here, pairwise, to the scores."""
    b = truth_tracks(n=6, p=(20000.0, 30000.0), cid=405)
    P = orc.default_params()
    T = b.truth
    rng = np.random.default_rng(9)
    # three copies of each of two tracks' seeds, shifted, against shifted VELO states
    seeds = seeds_from_truth(orc, T, [0, 0, 0, 1, 1, 1])
    seeds["a"] += rng.uniform(-3.0, 3.0, len(seeds))
    vels = [velo(b, t, dx=float(rng.uniform(-3, 3)), dy=float(rng.uniform(-0.5, 0.5)), P=P)
            for t in (0, 0, 1, 1, 0)]
    V = {k: np.array(sum((v[k] for v in vels), [])) for k in vels[0]}
    chi = {}
    for vi in range(len(vels)):
        for si in range(len(seeds)):
            r = orc.match(seeds[si:si + 1], {k: V[k][vi:vi + 1] for k in V}, P)
            if len(r):
                chi[(vi, si)] = float(r[0]["chi2"])
    assert len(chi) >= 10
    want = sorted(k for k, c in chi.items()
                  if c == min(x for kk, x in chi.items() if kk[0] == k[0])
                  and c == min(x for kk, x in chi.items() if kk[1] == k[1]))
    got = sorted((int(x["velo_idx"]), int(x["seed_idx"])) for x in orc.match(seeds, V, P))
    assert got == want and len(want) >= 2
