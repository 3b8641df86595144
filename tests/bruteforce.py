"""Brute-force re-statements of the windowed searches, for tiny events only.

Every window is evaluated by scanning the WHOLE layer zone with the window
predicate, every "closest hit" by a full scan with an explicit tie rule, and
the clone vote by comparing every pair of tracks directly (O(n^2)).  These are
the pins for the oracle's binary-search windows and its O(n) vote table.
"""
from __future__ import annotations

import math

import numpy as np

X_LAYERS = (0, 3, 4, 7, 8, 11)
UV_LAYERS = (1, 2, 5, 6, 9, 10)
INIT = ((0, 4, 8), (3, 7, 11))
EXT = ((3, 7, 11), (0, 4, 8))


def g(u, d):
    return u * u * (1.0 + d * u)


def xmodel(p, z, zr, d):
    u = z - zr
    return p[0] + p[1] * u + p[2] * g(u, d)


def zone(ev, half, layer):
    return int(ev.zone_off[half * 12 + layer]), int(ev.zone_off[half * 12 + layer + 1])


def lstsq_xz(z, x, zr, d):
    u = np.asarray(z, float) - zr
    A = np.stack([np.ones_like(u), u, g(u, d)], axis=1)
    sol, *_ = np.linalg.lstsq(A, np.asarray(x, float), rcond=None)
    return sol


def closest_full_scan(X, lo, hi, pred, tol):
    best, bestd = -1, math.inf
    for i in range(lo, hi):
        x = float(X[i])
        if pred - tol <= x <= pred + tol:
            dd = abs(x - pred)
            if dd < bestd - 1e-6:   # closer by more than 1 nm, else the lower position stays
                best, bestd = i, dd
    return best


def triplets(ev, half, it, P, G, wc):
    """All (i1, i2, i3) passing the two-hit and three-hit predicates."""
    L1, L2, L3 = INIT[it]
    z2, zr, d = G.z[L2], G.z_ref, P.d_ratio
    dx3max, alpha = wc[0], wc[1]
    X, Z = ev.hit_x.astype(float), ev.hit_z.astype(float)
    out = []
    b1, e1 = zone(ev, half, L1)
    b2, e2 = zone(ev, half, L2)
    b3, e3 = zone(ev, half, L3)
    for i1 in range(b1, e1):
        x1, zh1 = X[i1], Z[i1]
        centre = (G.z[L3] + alpha) / zh1 * x1
        for i3 in range(b3, e3):
            if not (centre - dx3max <= X[i3] <= centre + dx3max):
                continue
            x3, zh3 = X[i3], Z[i3]
            t13 = (x3 - x1) / (zh3 - zh1)
            x0 = x1 - zh1 * t13
            ip = P.invp_a * abs(x0) + P.invp_b * x0 * x0
            cp = -(1.0 if x0 >= 0 else -1.0) * P.kappa_c * ip
            k3 = g(z2 - zr, d) - g(zh1 - zr, d) - (z2 - zh1) / (zh3 - zh1) * (g(zh3 - zr, d) - g(zh1 - zr, d))
            pred = x1 + (z2 - zh1) * t13 + k3 * cp
            tol = P.t2_tol0 + P.t2_tol1 * abs(k3 * cp)
            for i2 in range(b2, e2):
                if pred - tol <= X[i2] <= pred + tol:
                    out.append((i1, i2, i3))
    return out


def extend_and_fit(ev, half, it, trip, P, G):
    """Extension by full scans + lstsq fit. Returns (pos[12], n, status, a, b, c, chi2)."""
    L1, L2, L3 = INIT[it]
    X, Z = ev.hit_x.astype(float), ev.hit_z.astype(float)
    zr, d = G.z_ref, P.d_ratio
    pos = [-1] * 12
    for L, i in zip((L1, L2, L3), trip):
        pos[L] = i
    p3 = lstsq_xz([Z[i] for i in trip], [X[i] for i in trip], zr, d)
    n = 3
    for L in EXT[it]:
        lo, hi = zone(ev, half, L)
        h = closest_full_scan(X, lo, hi, xmodel(p3, G.z[L], zr, d), P.ext_tol)
        if h >= 0:
            pos[L] = h
            n += 1
    if n < P.min_x_hits:
        return pos, n, 1, None
    hs = [pos[L] for L in X_LAYERS if pos[L] >= 0]
    z, x = Z[hs], X[hs]
    p = lstsq_xz(z, x, zr, d)
    chi2 = float(np.sum(((x - xmodel(p, z, zr, d)) / P.sigma_x) ** 2) / (len(hs) - 3))
    return pos, n, (0 if chi2 < P.chi2x_max else 2), (p, chi2)


def vote_pairwise(cands):
    """Clone vote stated pairwise: track i owns hit h iff no other track using h
    has a strictly lower score; keep rule of Sec. 3.3.4; then drop the second
    iteration's copy of an identical x-hit set."""
    n = len(cands)
    sets = [set(int(h) for h in c["pos"] if h >= 0) for c in cands]
    keep = np.zeros(n, bool)
    for i in range(n):
        own = 0
        for h in sets[i]:
            if not any(cands[j]["score"] < cands[i]["score"] for j in range(n) if j != i and h in sets[j]):
                own += 1
        keep[i] = own >= 3 or (own >= 2 and cands[i]["n"] == 6)
    for i in range(n):
        if keep[i] and cands[i]["it"] == 1:
            for j in range(n):
                if keep[j] and cands[j]["it"] == 0 and list(cands[j]["pos"]) == list(cands[i]["pos"]):
                    keep[i] = False
                    break
    return keep


def uv_full_scan(ev, cand, P, G):
    """UV seeding of one x-z track with full-zone scans. Returns
    (pos[12] of stereo hits, n, y0, ty, chi2) of the best combination, or None."""
    X, Z = ev.hit_x.astype(float), ev.hit_z.astype(float)
    zr, d = G.z_ref, P.d_ratio
    prm = (cand["a"], cand["b"], cand["c"])
    half = int(cand["half"])
    ylo, yhi = (0.0, P.y_max) if half == 0 else (-P.y_max, 0.0)
    best = None
    for L0 in (1, 2):
        t0 = G.tan_a[L0]
        xp = xmodel(prm, G.z[L0], zr, d)
        e1, e2 = xp - yhi * t0, xp - ylo * t0
        lo_x, hi_x = min(e1, e2), max(e1, e2)
        b0, en0 = zone(ev, half, L0)
        for h0 in range(b0, en0):
            if not (lo_x <= X[h0] <= hi_x):
                continue
            pos = [-1] * 12
            pos[L0] = h0
            y = (xmodel(prm, Z[h0], zr, d) - X[h0]) / t0
            ty = y / Z[h0]
            pts = [(Z[h0], y, t0)]
            for L in UV_LAYERS:
                if L == L0:
                    continue
                tl = G.tan_a[L]
                pred = xmodel(prm, G.z[L], zr, d) - ty * G.z[L] * tl
                lo, hi = zone(ev, half, L)
                h = closest_full_scan(X, lo, hi, pred, P.uv_tol)
                if h < 0:
                    continue
                yl = (xmodel(prm, Z[h], zr, d) - X[h]) / tl
                ty = 0.5 * (ty + yl / Z[h])
                pos[L] = h
                pts.append((Z[h], yl, tl))
            n = len(pts)
            if n < P.min_uv_hits:
                continue
            zz = np.array([p[0] for p in pts]) - zr
            yy = np.array([p[1] for p in pts])
            w = np.array([(p[2] / P.sigma_x) ** 2 for p in pts])
            A = np.stack([np.ones_like(zz), zz], 1) * np.sqrt(w)[:, None]
            sol, *_ = np.linalg.lstsq(A, yy * np.sqrt(w), rcond=None)
            chi2 = float(np.sum(w * (yy - sol[0] - sol[1] * zz) ** 2) / (n - 2))
            if not chi2 < P.chi2y_max:
                continue
            if best is None or n > best[1] or (n == best[1] and chi2 < best[4]):
                best = (pos, n, sol[0], sol[1], chi2)
    return best


def uv_hough_full_scan(ev, cand, P, G):
    """Hough-cluster UV search with full-zone scans: coarse t_y histogram over
    the half's range, the most populated bins (ties to the lower bin), fine
    bins inside each, the mean t_y of a fine bin as the hypothesis, the
    closest hit within uv_tol per stereo layer, the weighted line fit.
    Returns (pos[12], n, y0, ty, chi2) of the best combination or None."""
    X, Z = ev.hit_x.astype(float), ev.hit_z.astype(float)
    zr, d = G.z_ref, P.d_ratio
    prm = (cand["a"], cand["b"], cand["c"])
    half = int(cand["half"])
    zmin = min(G.z[L] for L in UV_LAYERS)
    lo, hi = (0.0, P.y_max / zmin) if half == 0 else (-P.y_max / zmin, 0.0)
    ylo, yhi = (0.0, P.y_max) if half == 0 else (-P.y_max, 0.0)
    NB, NF = P.hough_bins, P.hough_fine
    w = (hi - lo) / NB
    tys = []
    for L in UV_LAYERS:
        a, bz = zone(ev, half, L)
        for h in range(a, bz):
            y = (xmodel(prm, Z[h], zr, d) - X[h]) / G.tan_a[L]
            if ylo <= y <= yhi:
                tys.append(y / Z[h])
    bins = [min(max(int(math.floor((t - lo) / w)), 0), NB - 1) for t in tys]
    counts = np.bincount(bins, minlength=NB) if bins else np.zeros(NB, int)
    order = sorted(range(NB), key=lambda b: (-counts[b], b))
    kept = [b for b in order if counts[b] >= P.hough_min][:P.hough_best]
    best = None
    for bb in kept:
        blo = lo + bb * w
        fw = w / NF
        for f in range(NF):
            sel = [t for t, b in zip(tys, bins)
                   if b == bb and min(max(int(math.floor((t - blo) / fw)), 0), NF - 1) == f]
            if not sel:
                continue
            ty = sum(sel) / len(sel)
            pos = [-1] * 12
            pts = []
            for L in UV_LAYERS:
                a, bz = zone(ev, half, L)
                pred = xmodel(prm, G.z[L], zr, d) - ty * G.z[L] * G.tan_a[L]
                h = closest_full_scan(X, a, bz, pred, P.uv_tol)
                if h >= 0:
                    pos[L] = h
                    pts.append((Z[h], (xmodel(prm, Z[h], zr, d) - X[h]) / G.tan_a[L], G.tan_a[L]))
            n = len(pts)
            if n < P.min_uv_hits:
                continue
            zz = np.array([p[0] for p in pts]) - zr
            yy = np.array([p[1] for p in pts])
            ww = np.array([(p[2] / P.sigma_x) ** 2 for p in pts])
            A = np.stack([np.ones_like(zz), zz], 1) * np.sqrt(ww)[:, None]
            sol, *_ = np.linalg.lstsq(A, yy * np.sqrt(ww), rcond=None)
            chi2 = float(np.sum(ww * (yy - sol[0] - sol[1] * zz) ** 2) / (n - 2))
            if not chi2 < P.chi2y_max:
                continue
            if best is None or n > best[1] or (n == best[1] and chi2 < best[4]):
                best = (pos, n, sol[0], sol[1], chi2)
    return best
