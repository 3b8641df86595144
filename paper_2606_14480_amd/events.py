"""Seeded synthetic SciFi + VELO events (input generator only).

This module simulates the detector, it does not reconstruct anything: it
draws charged tracks, bends them at a magnet kink, propagates them through the
twelve SciFi layers (Sec. 1: three stations of x-u-v-x layers, stereo angle
+-5 deg, vertical field bending in x-z) and emits the hit SoA and VELO states
that both the CPU oracle and the HIP library consume.  Neither side imports
anything else from here.

Forward model of one track (truth -> hits), all in mm and MeV:

* origin (x_o, y_o, z_o), slopes tx, ty ~ U(-0.25, 0.25), momentum p
  log-uniform, charge q = +-1;
* the magnet is a single kink at z_k.  The kink size follows the inverse
  momentum parametrisation of Sec. 3.3.1 (eq. invp) read backwards:
  |x0| solves a|x0| + b x0^2 = 1/p, and the slope change is
  dtx = q * pol * |x0| / z_k, so the straight SciFi line meets z = 0 at
  x0 = -q pol |x0| relative to the VELO line;
* z_k is placed where the kink-position parametrisation of Sec. 4.1
  (eq. z_match, Table 1) puts it for this very track, found by fixed-point
  iteration (the parametrisation depends on the SciFi state, which depends on
  z_k);
* inside the SciFi the x trajectory is the tangent line at the last layer
  plus the residual-field term of eq. trackequation,
  c * [g(zb) - g(zb_s) - g'(zb_s) (z - z_s)], g(u) = u^2 (1 + d_ratio u),
  with c = q * pol * kappa_c / p, so x(z) = a + b zb + c g(zb) exactly;
* y is a straight line (Sec. 4: no bending in y-z).

Hits: x-layers measure x(z) + N(0, sigma); stereo layers measure
x(z) - y(z) tan(alpha) + N(0, sigma).  Each hit is dropped with probability
`ineff`; `noise` * n_signal uniformly placed noise hits are added.  Hits are
grouped in zones ``zone = (event*2 + half)*12 + layer`` (half 0: y > 0,
half 1: y < 0), sorted by x inside each zone.  Hit ids are a seeded
permutation of 0..n-1 inside each event, so an id never equals a position by
accident.

UT (Sec. 4.3; a synthetic layer model, the paper gives none): four planar
layers UTaX, UTaU, UTbV, UTbX at z = 2327.5, 2372.5, 2597.5, 2642.5 mm, with
stereo angles 0, +5, -5, 0 deg, measuring x - y tan(alpha) + N(0, 0.055 mm)
(a 190 um pitch).  Between the VELO end-state and the UT a track follows the
parabola of eq. velo_ut_extrapolation with gamma_x = A_gamma + B_gamma q/p
(eq. gamma_parametrisation, Table 1), read forwards.  |x| <= 860 mm and
|y| <= 700 mm at each layer; the same inefficiency and noise fraction as the
SciFi.  UT hits are grouped by (event, layer), x-sorted, ids a permutation
inside the event.  They come from a second random stream of the event, so
every SciFi and VELO array is the same with or without them.

Every event has its own PCG64 stream seeded with
``1_000_000 * config + event_index``, so any subset regenerates identically.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------- detector --
N_LAYERS = 12
N_HALVES = 2
ZONES_PER_EVENT = N_LAYERS * N_HALVES
# 3 stations x (x, u, v, x); 70 mm layer pitch inside a station (Sec. 1: the
# layers of a station are 50 mm apart through air), spanning 7826-9439 mm.
LAYER_Z = np.array([7826.0, 7896.0, 7966.0, 8036.0,
                    8527.5, 8597.5, 8667.5, 8737.5,
                    9229.0, 9299.0, 9369.0, 9439.0])
_T5 = math.tan(math.radians(5.0))
LAYER_TAN = np.array([0.0, _T5, -_T5, 0.0] * 3)
Z_REF = 8525.0           # eq. trackequation reference point
X_ACC = 3200.0           # |x| acceptance at every layer
Y_ACC_MIN = 2.5          # |y| acceptance (beam hole)
Y_ACC_MAX = 2500.0
Z_VELO = 770.0           # z of the VELO end-state
# UT: UTaX, UTaU, UTbV, UTbX
N_UT = 4
UT_Z = np.array([2327.5, 2372.5, 2597.5, 2642.5])
UT_TAN = np.array([0.0, _T5, -_T5, 0.0])
UT_SIGMA = 0.055
UT_X_ACC = 860.0
UT_Y_ACC = 700.0
A_GAMMA = 7.707063e-11   # Table 1
B_GAMMA = -7.817364e-3

# physics constants of the forward model (Sec. 3.3.1 eq. invp, Table 1)
INVP_A = 1.6322e-7
INVP_B = -5.0217e-12
ZM = (5287.6, -7.98878, 317.683, 0.0119379, -1418.42)
D_RATIO = -3.0e-4        # residual-field cubic term, mm^-1
KAPPA_C = 3.0e-3         # curvature scale c = q pol kappa_c / p, MeV / mm
POLARITY = 1.0


@dataclasses.dataclass
class GenConfig:
    n_events: int
    config_id: int
    mult: str = "poisson"          # "fixed" | "poisson" | "negbin"
    mean_tracks: float = 120.0
    nb_k: float = 1.0
    clip: tuple = (0, 10 ** 9)
    p_range: tuple = (1500.0, 100000.0)
    sigma: float = 0.07
    ineff: float = 0.0
    noise: float = 0.0
    ghost_velo: float = 0.0
    velo_sigma_x: float = 0.0
    velo_sigma_t: float = 0.0
    first_event: int = 0


def config(n: int, n_events: int | None = None, first_event: int = 0) -> GenConfig:
    """The five workloads: 1 tiny, 2 min-bias, 3 uneven, 4 stress, 5 serving."""
    if n == 1:
        return GenConfig(n_events=n_events or 1, config_id=1, mult="fixed",
                         mean_tracks=20, p_range=(2000.0, 100000.0),
                         first_event=first_event)
    if n in (2, 5):
        return GenConfig(n_events=n_events or 1000, config_id=n, mult="poisson",
                         mean_tracks=120, ineff=0.02, noise=0.10,
                         ghost_velo=0.05, velo_sigma_x=0.01, velo_sigma_t=2e-4,
                         first_event=first_event)
    if n == 3:
        return GenConfig(n_events=n_events or 10000, config_id=3, mult="negbin",
                         mean_tracks=120, clip=(10, 600), ineff=0.02,
                         noise=0.10, ghost_velo=0.05, velo_sigma_x=0.01,
                         velo_sigma_t=2e-4, first_event=first_event)
    if n == 4:
        return GenConfig(n_events=n_events or 50000, config_id=4, mult="negbin",
                         mean_tracks=240, clip=(20, 3000), ineff=0.05,
                         noise=0.20, ghost_velo=0.05, velo_sigma_x=0.01,
                         velo_sigma_t=2e-4, first_event=first_event)
    raise ValueError(f"unknown config {n}")


@dataclasses.dataclass
class Batch:
    """Host-side batch in the layout of the C-ABI (all numpy)."""
    zone_off: np.ndarray     # int32 [n_events*24 + 1]
    hit_x: np.ndarray        # float32 [n_hits]
    hit_z: np.ndarray        # float32 [n_hits]
    hit_id: np.ndarray       # int32 [n_hits]
    velo_off: np.ndarray     # int32 [n_events + 1]
    velo_x: np.ndarray       # float32 [n_velo]
    velo_y: np.ndarray
    velo_z: np.ndarray
    velo_tx: np.ndarray
    velo_ty: np.ndarray
    velo_id: np.ndarray      # int32 [n_velo]
    truth: dict | None = None
    # UT hits, grouped by (event, layer) and x-sorted; None: no UT
    ut_off: np.ndarray | None = None    # int32 [n_events*4 + 1]
    ut_x: np.ndarray | None = None      # float32 [n_ut]
    ut_id: np.ndarray | None = None     # int32 [n_ut]

    @property
    def n_events(self) -> int:
        return (len(self.zone_off) - 1) // ZONES_PER_EVENT

    @property
    def n_hits(self) -> int:
        return int(self.zone_off[-1])

    @property
    def n_velo(self) -> int:
        return int(self.velo_off[-1])

    @property
    def n_ut(self) -> int:
        return int(self.ut_off[-1]) if self.ut_off is not None else 0

    @property
    def has_ut(self) -> bool:
        return self.ut_off is not None

    def event_hits(self) -> np.ndarray:
        o = self.zone_off[::ZONES_PER_EVENT]
        return np.diff(o)

    def subset(self, idx) -> "Batch":
        return concat([self.event(int(i)) for i in idx])

    def event(self, e: int) -> "Batch":
        z0 = e * ZONES_PER_EVENT
        h0, h1 = int(self.zone_off[z0]), int(self.zone_off[z0 + ZONES_PER_EVENT])
        v0, v1 = int(self.velo_off[e]), int(self.velo_off[e + 1])
        truth = None
        if self.truth is not None:
            t0, t1 = self.truth["track_off"][e], self.truth["track_off"][e + 1]
            truth = {k: (v[t0:t1] if k != "track_off" else np.array([0, t1 - t0]))
                     for k, v in self.truth.items()}
        ut = {}
        if self.ut_off is not None:
            u0, u1 = int(self.ut_off[e * N_UT]), int(self.ut_off[(e + 1) * N_UT])
            ut = dict(ut_off=(self.ut_off[e * N_UT:(e + 1) * N_UT + 1] - u0).astype(np.int32),
                      ut_x=self.ut_x[u0:u1], ut_id=self.ut_id[u0:u1])
        return Batch(
            zone_off=(self.zone_off[z0:z0 + ZONES_PER_EVENT + 1] - h0).astype(np.int32),
            hit_x=self.hit_x[h0:h1], hit_z=self.hit_z[h0:h1], hit_id=self.hit_id[h0:h1],
            velo_off=np.array([0, v1 - v0], np.int32),
            velo_x=self.velo_x[v0:v1], velo_y=self.velo_y[v0:v1],
            velo_z=self.velo_z[v0:v1], velo_tx=self.velo_tx[v0:v1],
            velo_ty=self.velo_ty[v0:v1], velo_id=self.velo_id[v0:v1], truth=truth, **ut)

    def without_ut(self) -> "Batch":
        return dataclasses.replace(self, ut_off=None, ut_x=None, ut_id=None)


def concat(events: list) -> Batch:
    """Concatenate single- or multi-event batches (offsets are rebased)."""
    zo, vo = [np.zeros(1, np.int32)], [np.zeros(1, np.int32)]
    hbase = vbase = 0
    for b in events:
        zo.append(b.zone_off[1:] + hbase)
        vo.append(b.velo_off[1:] + vbase)
        hbase += b.n_hits
        vbase += b.n_velo
    cat = lambda name, dt: (np.concatenate([getattr(b, name) for b in events]).astype(dt)
                            if events else np.zeros(0, dt))
    truth = None
    if events and all(b.truth is not None for b in events):
        keys = [k for k in events[0].truth if k != "track_off"]
        truth = {k: np.concatenate([b.truth[k] for b in events]) for k in keys}
        # per-event track offsets of every part, rebased (a part may hold several events)
        offs, tbase = [np.zeros(1, np.int64)], 0
        for b in events:
            offs.append(np.asarray(b.truth["track_off"][1:], np.int64) + tbase)
            tbase += len(b.truth["p"])
        truth["track_off"] = np.concatenate(offs)
    ut = {}
    if events and all(b.ut_off is not None for b in events):
        uo, ubase = [np.zeros(1, np.int64)], 0
        for b in events:
            uo.append(b.ut_off[1:].astype(np.int64) + ubase)
            ubase += b.n_ut
        ut = dict(ut_off=np.concatenate(uo).astype(np.int32), ut_x=cat("ut_x", np.float32),
                  ut_id=cat("ut_id", np.int32))
    return Batch(zone_off=np.concatenate(zo).astype(np.int32),
                 hit_x=cat("hit_x", np.float32), hit_z=cat("hit_z", np.float32),
                 hit_id=cat("hit_id", np.int32),
                 velo_off=np.concatenate(vo).astype(np.int32),
                 velo_x=cat("velo_x", np.float32), velo_y=cat("velo_y", np.float32),
                 velo_z=cat("velo_z", np.float32), velo_tx=cat("velo_tx", np.float32),
                 velo_ty=cat("velo_ty", np.float32), velo_id=cat("velo_id", np.int32),
                 truth=truth, **ut)


# ------------------------------------------------------------- the physics --
def _g(u):
    return u * u * (1.0 + D_RATIO * u)


def _dg(u):
    return 2.0 * u + 3.0 * D_RATIO * u * u


def _draw_tracks(rng, n, p_range, pol):
    """Draw n candidate tracks; returns a dict of per-track arrays."""
    lp = rng.uniform(math.log(p_range[0]), math.log(p_range[1]), n)
    p = np.exp(lp)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    xo = rng.normal(0.0, 0.03, n)
    yo = rng.normal(0.0, 0.03, n)
    zo = rng.normal(0.0, 50.0, n)
    tx = rng.uniform(-0.25, 0.25, n)
    ty = rng.uniform(-0.25, 0.25, n)
    # |x0| from 1/p = a|x0| + b x0^2 (smaller positive root)
    ax0 = (-INVP_A + np.sqrt(INVP_A ** 2 + 4.0 * INVP_B / p)) / (2.0 * INVP_B)
    zs = LAYER_Z[-1]
    xv = lambda z: xo + tx * (z - zo)
    zk = np.full(n, ZM[0])
    for _ in range(30):
        dtx = q * pol * ax0 / zk
        xs = xv(zk) + (tx + dtx) * (zs - zk)
        znew = (ZM[0] + ZM[1] * np.abs(dtx) + ZM[2] * dtx * dtx
                + ZM[3] * np.abs(xs) + ZM[4] * tx * tx)
        done = np.max(np.abs(znew - zk)) < 1e-10
        zk = znew
        if done:
            break
    dtx = q * pol * ax0 / zk
    txs = tx + dtx
    xs = xv(zk) + txs * (zs - zk)
    c = q * pol * KAPPA_C / p
    ubs = zs - Z_REF
    b = txs - c * _dg(ubs)
    a = xs - b * ubs - c * _g(ubs)
    y0 = yo + ty * (Z_REF - zo)
    return dict(p=p, q=q, xo=xo, yo=yo, zo=zo, tx=tx, ty=ty, zk=zk, dtx=dtx,
                a=a, b=b, c=c, y0=y0)


def _track_xy(t, z):
    u = z[None, :] - Z_REF
    x = t["a"][:, None] + t["b"][:, None] * u + t["c"][:, None] * _g(u)
    y = t["y0"][:, None] + t["ty"][:, None] * u
    return x, y


def _accepted(t):
    x, y = _track_xy(t, LAYER_Z)
    ok = np.all(np.abs(x) <= X_ACC, axis=1)
    ok &= np.all((np.abs(y) >= Y_ACC_MIN) & (np.abs(y) <= Y_ACC_MAX), axis=1)
    ok &= np.all(np.sign(y) == np.sign(y[:, :1]), axis=1)
    return ok


def _n_tracks(rng, cfg: GenConfig) -> int:
    if cfg.mult == "fixed":
        n = int(cfg.mean_tracks)
    elif cfg.mult == "poisson":
        n = int(rng.poisson(cfg.mean_tracks))
    elif cfg.mult == "negbin":
        k = cfg.nb_k
        n = int(rng.negative_binomial(k, k / (k + cfg.mean_tracks)))
    else:
        raise ValueError(cfg.mult)
    return int(min(max(n, cfg.clip[0]), cfg.clip[1]))


def generate_event(cfg: GenConfig, e: int, pol: float = POLARITY) -> Batch:
    """One event of workload `cfg` (event index `e` within the workload)."""
    rng = np.random.Generator(np.random.PCG64(1_000_000 * cfg.config_id + e))
    n = _n_tracks(rng, cfg)
    parts, have = [], 0
    while have < n:
        t = _draw_tracks(rng, max(2 * (n - have), 8), cfg.p_range, pol)
        ok = _accepted(t)
        t = {k: v[ok] for k, v in t.items()}
        parts.append(t)
        have += len(t["p"])
    t = {k: np.concatenate([pp[k] for pp in parts])[:n] for k in parts[0]}

    x, y = _track_xy(t, LAYER_Z)                          # [n, 12]
    meas = x - y * LAYER_TAN[None, :]
    meas = meas + rng.normal(0.0, cfg.sigma, meas.shape) if cfg.sigma > 0 else meas
    keep = rng.random(meas.shape) >= cfg.ineff if cfg.ineff > 0 else np.ones(meas.shape, bool)
    half = np.where(y > 0, 0, 1)
    trk = np.repeat(np.arange(n), N_LAYERS).reshape(n, N_LAYERS)
    lay = np.tile(np.arange(N_LAYERS), (n, 1))
    hx, hl, hh, ht = meas[keep], lay[keep], half[keep], trk[keep]
    n_sig = len(hx)
    n_noise = int(round(cfg.noise * n_sig))
    if n_noise:
        hx = np.concatenate([hx, rng.uniform(-X_ACC, X_ACC, n_noise)])
        hl = np.concatenate([hl, rng.integers(0, N_LAYERS, n_noise)])
        hh = np.concatenate([hh, rng.integers(0, N_HALVES, n_noise)])
        ht = np.concatenate([ht, np.full(n_noise, -1)])
    hx32 = hx.astype(np.float32)
    zone = hh * N_LAYERS + hl
    order = np.lexsort((np.arange(len(hx32)), hx32, zone))
    hx32, zone, hl, ht = hx32[order], zone[order], hl[order], ht[order]
    counts = np.bincount(zone, minlength=ZONES_PER_EVENT)
    zone_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    nh = len(hx32)
    hit_id = rng.permutation(nh).astype(np.int32)
    hit_z = LAYER_Z[hl].astype(np.float32)

    # truth: hit ids of each track by layer (-1 where inefficient)
    thits = np.full((n, N_LAYERS), -1, np.int32)
    sig = ht >= 0
    thits[ht[sig], hl[sig]] = hit_id[sig]

    # VELO end-states: one per track (+ ghosts), in a seeded random order
    vx = t["xo"] + t["tx"] * (Z_VELO - t["zo"])
    vy = t["yo"] + t["ty"] * (Z_VELO - t["zo"])
    vtx, vty = t["tx"].copy(), t["ty"].copy()
    if cfg.velo_sigma_x > 0:
        vx = vx + rng.normal(0, cfg.velo_sigma_x, n)
        vy = vy + rng.normal(0, cfg.velo_sigma_x, n)
    if cfg.velo_sigma_t > 0:
        vtx = vtx + rng.normal(0, cfg.velo_sigma_t, n)
        vty = vty + rng.normal(0, cfg.velo_sigma_t, n)
    n_ghost = int(round(cfg.ghost_velo * n))
    vtrk = np.arange(n)
    if n_ghost:
        gtx = rng.uniform(-0.25, 0.25, n_ghost)
        gty = rng.uniform(-0.25, 0.25, n_ghost)
        gzo = rng.normal(0, 50.0, n_ghost)
        vx = np.concatenate([vx, rng.normal(0, 0.03, n_ghost) + gtx * (Z_VELO - gzo)])
        vy = np.concatenate([vy, rng.normal(0, 0.03, n_ghost) + gty * (Z_VELO - gzo)])
        vtx = np.concatenate([vtx, gtx])
        vty = np.concatenate([vty, gty])
        vtrk = np.concatenate([vtrk, np.full(n_ghost, -1)])
    vperm = rng.permutation(len(vx))
    nv = len(vx)
    velo_id = rng.permutation(nv).astype(np.int32)
    vx, vy, vtx, vty, vtrk = vx[vperm], vy[vperm], vtx[vperm], vty[vperm], vtrk[vperm]
    velo_of_track = np.full(n, -1, np.int64)
    velo_of_track[vtrk[vtrk >= 0]] = np.nonzero(vtrk >= 0)[0]

    ut_off, ut_x, ut_id, ut_hits = _ut_hits(cfg, e, t)
    truth = dict(p=t["p"], q=t["q"], a=t["a"], b=t["b"], c=t["c"], y0=t["y0"],
                 ty=t["ty"], tx=t["tx"], zk=t["zk"], dtx=t["dtx"], hits=thits,
                 velo=velo_of_track, ut_hits=ut_hits, track_off=np.array([0, n], np.int64))
    return Batch(zone_off=zone_off, hit_x=hx32, hit_z=hit_z, hit_id=hit_id,
                 velo_off=np.array([0, nv], np.int32),
                 velo_x=vx.astype(np.float32), velo_y=vy.astype(np.float32),
                 velo_z=np.full(nv, Z_VELO, np.float32),
                 velo_tx=vtx.astype(np.float32), velo_ty=vty.astype(np.float32),
                 velo_id=velo_id, truth=truth, ut_off=ut_off, ut_x=ut_x, ut_id=ut_id)


def _ut_hits(cfg: GenConfig, e: int, t: dict):
    """UT hits of one event's tracks (second random stream of the event)."""
    rng = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(1_000_000 * cfg.config_id + e, spawn_key=(1,))))
    n = len(t["p"])
    dz = UT_Z[None, :] - Z_VELO
    xv = t["xo"] + t["tx"] * (Z_VELO - t["zo"])
    yv = t["yo"] + t["ty"] * (Z_VELO - t["zo"])
    gam = A_GAMMA + B_GAMMA * t["q"] / t["p"]
    x = xv[:, None] + t["tx"][:, None] * dz + gam[:, None] * dz * dz
    y = yv[:, None] + t["ty"][:, None] * dz
    meas = x - y * UT_TAN[None, :]
    meas = meas + rng.normal(0.0, UT_SIGMA, meas.shape)
    keep = (np.abs(x) <= UT_X_ACC) & (np.abs(y) <= UT_Y_ACC)
    if cfg.ineff > 0:
        keep &= rng.random(meas.shape) >= cfg.ineff
    trk = np.repeat(np.arange(n), N_UT).reshape(n, N_UT)
    lay = np.tile(np.arange(N_UT), (n, 1))
    hx, hl, ht = meas[keep], lay[keep], trk[keep]
    n_noise = int(round(cfg.noise * len(hx)))
    if n_noise:
        hx = np.concatenate([hx, rng.uniform(-UT_X_ACC, UT_X_ACC, n_noise)])
        hl = np.concatenate([hl, rng.integers(0, N_UT, n_noise)])
        ht = np.concatenate([ht, np.full(n_noise, -1)])
    hx32 = hx.astype(np.float32)
    order = np.lexsort((np.arange(len(hx32)), hx32, hl))
    hx32, hl, ht = hx32[order], hl[order], ht[order]
    ut_off = np.concatenate([[0], np.cumsum(np.bincount(hl, minlength=N_UT))]).astype(np.int32)
    ut_id = rng.permutation(len(hx32)).astype(np.int32)
    ut_hits = np.full((n, N_UT), -1, np.int32)
    sig = ht >= 0
    ut_hits[ht[sig], hl[sig]] = ut_id[sig]
    return ut_off, hx32, ut_id, ut_hits


def generate(cfg: GenConfig, pol: float = POLARITY) -> Batch:
    return concat([generate_event(cfg, cfg.first_event + i, pol) for i in range(cfg.n_events)])


def _generate_range(cfg: GenConfig, first: int, n: int, pol: float) -> Batch:
    return generate(dataclasses.replace(cfg, n_events=n, first_event=first), pol)


def generate_parallel(cfg: GenConfig, workers: int = 16, pol: float = POLARITY) -> Batch:
    """generate() spread over worker processes.  Every event is drawn from its
    own seed, so the batch is identical to generate()'s.  The workers are
    started fresh (spawn), never forked from a process that may hold GPU
    state."""
    n = cfg.n_events
    workers = max(1, min(workers, n // 64))
    if workers <= 1:
        return generate(cfg, pol)
    import concurrent.futures as cf
    import multiprocessing as mp
    k = 4 * workers
    bounds = [n * i // k for i in range(k + 1)]
    jobs = [(cfg, cfg.first_event + bounds[i], bounds[i + 1] - bounds[i], pol)
            for i in range(k) if bounds[i + 1] > bounds[i]]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_generate_range, *zip(*jobs)))
    return concat(parts)


def tile(b: Batch, times: int) -> Batch:
    """The events of b repeated `times` times, one after the other (a larger
    batch of the same events, for batch-size sweeps beyond what is worth
    generating).  Truth is dropped."""
    nh, nv, ne = b.n_hits, b.n_velo, b.n_events
    zo = np.concatenate([np.zeros(1, np.int64)] +
                        [b.zone_off[1:].astype(np.int64) + k * nh for k in range(times)])
    vo = np.concatenate([np.zeros(1, np.int64)] +
                        [b.velo_off[1:].astype(np.int64) + k * nv for k in range(times)])
    if zo[-1] >= 2 ** 31 or vo[-1] >= 2 ** 31:
        raise ValueError("tiled batch exceeds the int32 offsets of the batch layout")
    rep = lambda a: np.tile(a, times)
    ut = {}
    if b.ut_off is not None:
        nu = b.n_ut
        uo = np.concatenate([np.zeros(1, np.int64)] +
                            [b.ut_off[1:].astype(np.int64) + k * nu for k in range(times)])
        ut = dict(ut_off=uo.astype(np.int32), ut_x=rep(b.ut_x), ut_id=rep(b.ut_id))
    return Batch(zone_off=zo.astype(np.int32), hit_x=rep(b.hit_x), hit_z=rep(b.hit_z),
                 hit_id=rep(b.hit_id), velo_off=vo.astype(np.int32), velo_x=rep(b.velo_x),
                 velo_y=rep(b.velo_y), velo_z=rep(b.velo_z), velo_tx=rep(b.velo_tx),
                 velo_ty=rep(b.velo_ty), velo_id=rep(b.velo_id), truth=None, **ut)


def empty_event() -> Batch:
    return Batch(zone_off=np.zeros(ZONES_PER_EVENT + 1, np.int32),
                 hit_x=np.zeros(0, np.float32), hit_z=np.zeros(0, np.float32),
                 hit_id=np.zeros(0, np.int32), velo_off=np.zeros(2, np.int32),
                 velo_x=np.zeros(0, np.float32), velo_y=np.zeros(0, np.float32),
                 velo_z=np.zeros(0, np.float32), velo_tx=np.zeros(0, np.float32),
                 velo_ty=np.zeros(0, np.float32), velo_id=np.zeros(0, np.int32),
                 truth={k: np.zeros((0, 12) if k == "hits" else ((0, 4) if k == "ut_hits" else 0))
                        for k in ("p", "q", "a", "b", "c", "y0", "ty", "tx", "zk",
                                  "dtx", "hits", "velo", "ut_hits")} | {"track_off": np.array([0, 0])},
                 ut_off=np.zeros(N_UT + 1, np.int32), ut_x=np.zeros(0, np.float32),
                 ut_id=np.zeros(0, np.int32))
