"""ctypes binding of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
NL = 12
NUT = 4


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain IEEE double, no fast-math)."""
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall",
                               "-fno-fast-math", "-ffp-contract=off", src, "-o", tmp,
                               "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Geom(C.Structure):
    _fields_ = [("z", C.c_double * NL), ("tan_a", C.c_double * NL), ("z_ref", C.c_double),
                ("ut_z", C.c_double * NUT), ("ut_tan", C.c_double * NUT)]


NN_IN, NN_HID = 8, 32


class GhostNN(C.Structure):
    _fields_ = [("mean", C.c_double * NN_IN), ("scale", C.c_double * NN_IN),
                ("w1", (C.c_double * NN_IN) * NN_HID), ("b1", C.c_double * NN_HID),
                ("w2", C.c_double * NN_HID), ("b2", C.c_double)]


def set_ghost_nn(nn: GhostNN, w: dict) -> None:
    """Fill the network from a dict (mean, scale [8]; w1 [32][8]; b1, w2 [32];
    b2), as stored in the package's ghost_nn.json."""
    for i in range(NN_IN):
        nn.mean[i] = float(w["mean"][i])
        nn.scale[i] = float(w["scale"][i])
    for j in range(NN_HID):
        for i in range(NN_IN):
            nn.w1[j][i] = float(w["w1"][j][i])
        nn.b1[j] = float(w["b1"][j])
        nn.w2[j] = float(w["w2"][j])
    nn.b2 = float(w["b2"])


class Params(C.Structure):
    _fields_ = [("p_min", C.c_double), ("invp_a", C.c_double), ("invp_b", C.c_double),
                ("alpha0", C.c_double), ("alpha1", C.c_double), ("d_ratio", C.c_double),
                ("kappa_c", C.c_double), ("t2_tol0", C.c_double), ("t2_tol1", C.c_double),
                ("ext_tol", C.c_double), ("min_x_hits", C.c_int32), ("pad0", C.c_int32),
                ("sigma_x", C.c_double), ("chi2x_max", C.c_double),
                ("uv_tol", C.c_double), ("y_max", C.c_double),
                ("min_uv_hits", C.c_int32), ("pad1", C.c_int32), ("chi2y_max", C.c_double),
                ("zm", C.c_double * 5), ("z_ymatch", C.c_double), ("z_state", C.c_double),
                ("max_dx", C.c_double), ("max_dy", C.c_double), ("max_dtx", C.c_double),
                ("max_dty", C.c_double),
                ("tolx_scale", C.c_double), ("tolx_a", C.c_double), ("tolx_b", C.c_double),
                ("toly_scale", C.c_double), ("toly_a", C.c_double), ("toly_b", C.c_double),
                ("tol_tx", C.c_double), ("tol_ty", C.c_double), ("chi2m_max", C.c_double),
                ("polarity", C.c_double), ("uv_mode", C.c_int32), ("hough_bins", C.c_int32),
                ("hough_best", C.c_int32), ("hough_fine", C.c_int32), ("hough_min", C.c_int32),
                ("pad2", C.c_int32), ("final_sel", C.c_int32), ("pad3", C.c_int32),
                ("ghost_cut", C.c_double), ("clone_gap", C.c_double), ("ghost_nn", GhostNN),
                ("ut_mode", C.c_int32), ("ut_min_hits", C.c_int32),
                ("a_gamma", C.c_double), ("b_gamma", C.c_double)] + \
               [(f"ut_{k}_{w}", C.c_double * NUT) for k in ("loose", "tight")
                for w in ("a", "b", "lo", "hi")] + \
               [("third_iter", C.c_int32), ("pad4", C.c_int32), ("p_min3", C.c_double)]

    ARRAYS = ("zm",) + tuple(f"ut_{k}_{w}" for k in ("loose", "tight") for w in ("a", "b", "lo", "hi"))

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            if name.startswith("pad") or name == "ghost_nn":
                continue
            v = getattr(self, name)
            out[name] = list(v) if name in self.ARRAYS else v
        return out


# margins: the relative distance of a track's closest decision from going
# the other way (oracle.h, ORC_NEAR); near misses: rejections within NEAR
NEAR = 1e-3
NEAR_XZ, NEAR_VOTE, NEAR_UV, NEAR_MATCH = 1, 2, 3, 4

CAND_DTYPE = np.dtype([("half", "i4"), ("it", "i4"), ("status", "i4"), ("n", "i4"),
                       ("pos", "i4", NL), ("a", "f8"), ("b", "f8"), ("c", "f8"),
                       ("chi2", "f8"), ("score", "f8"), ("margin", "f8")], align=True)
SEED_DTYPE = np.dtype([("a", "f8"), ("b", "f8"), ("c", "f8"), ("y0", "f8"), ("ty", "f8"),
                       ("chi2x", "f8"), ("chi2y", "f8"), ("score", "f8"),
                       ("nx", "i4"), ("nuv", "i4"), ("half", "i4"), ("it", "i4"),
                       ("pos", "i4", NL), ("id", "i4", NL), ("margin", "f8")], align=True)
LONG_DTYPE = np.dtype([("velo_idx", "i4"), ("velo_id", "i4"), ("seed_idx", "i4"),
                       ("n_ut", "i4"), ("ut_id", "i4", NUT), ("qop", "f8"), ("chi2", "f8"), ("zm", "f8"),
                       ("dx", "f8"), ("dy", "f8"), ("dtx", "f8"), ("dty", "f8"),
                       ("gp", "f8"), ("margin", "f8")], align=True)
PAIR_DTYPE = np.dtype([("velo_idx", "i4"), ("seed_idx", "i4"), ("f", "f8", NN_IN), ("gp", "f8")],
                      align=True)
NEAR_DTYPE = np.dtype([("event", "i4"), ("kind", "i4"), ("velo_idx", "i4"), ("it", "i4"),
                       ("id", "i4", NL), ("margin", "f8")], align=True)


class _Result(C.Structure):
    _fields_ = [("n_seeds", C.c_int64), ("n_longs", C.c_int64),
                ("seed_off", C.POINTER(C.c_int32)), ("seeds", C.c_void_p),
                ("long_off", C.POINTER(C.c_int32)), ("longs", C.c_void_p),
                ("n_near", C.c_int64), ("near", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.orc_default_geom.argtypes = [C.POINTER(Geom)]
        L.orc_default_params.argtypes = [C.POINTER(Params)]
        L.orc_xz_candidates.argtypes = [C.POINTER(Geom), C.POINTER(Params), vp, vp, vp,
                                        C.c_int, C.c_int, vp, C.c_int]
        L.orc_xz_candidates.restype = C.c_int
        L.orc_clone_vote.argtypes = [vp, C.c_int, C.c_int, vp]
        L.orc_uv.argtypes = [C.POINTER(Geom), C.POINTER(Params), vp, vp, vp, vp, vp, vp]
        L.orc_uv.restype = C.c_int
        L.orc_match.argtypes = [C.POINTER(Geom), C.POINTER(Params), vp, C.c_int, C.c_int,
                                vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]
        L.orc_match.restype = C.c_int
        L.orc_match_pairs.argtypes = [C.POINTER(Geom), C.POINTER(Params), vp, C.c_int, C.c_int,
                                      vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]
        L.orc_match_pairs.restype = C.c_int
        L.orc_ut_window.argtypes = [C.POINTER(Params), C.c_int, C.c_int, C.c_double]
        L.orc_ut_window.restype = C.c_double
        L.orc_ghost_prob.argtypes = [C.POINTER(Params), vp]
        L.orc_ghost_prob.restype = C.c_double
        L.orc_run.argtypes = [C.POINTER(Geom), C.POINTER(Params), C.c_int] + [vp] * 14 + \
                             [C.c_int, C.c_int, C.POINTER(_Result)]
        L.orc_run.restype = C.c_int
        L.orc_free.argtypes = [C.POINTER(_Result)]
        L.orc_window_constants.argtypes = [C.POINTER(Geom), C.POINTER(Params), C.c_int, vp]
        _lib = L
    return _lib


def default_geom() -> Geom:
    g = Geom()
    lib().orc_default_geom(C.byref(g))
    return g


def default_params(**over) -> Params:
    p = Params()
    lib().orc_default_params(C.byref(p))
    for k, v in over.items():
        if k in Params.ARRAYS:
            for i, x in enumerate(v):
                getattr(p, k)[i] = x
        elif k == "ghost_nn":
            set_ghost_nn(p.ghost_nn, v)
        else:
            setattr(p, k, v)
    return p


def window_constants(it: int, params: Params | None = None, geom: Geom | None = None):
    """(Delta x3^max, alpha_corr, K3) of iteration `it`."""
    out = np.zeros(3)
    lib().orc_window_constants(C.byref(geom or default_geom()), C.byref(params or default_params()),
                               it, out.ctypes.data_as(C.c_void_p))
    return tuple(out)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def xz_candidates(ev, half: int, it: int, params: Params | None = None,
                  geom: Geom | None = None) -> np.ndarray:
    """Every three-hit combination of one event-half-iteration (ev: 1-event Batch)."""
    params = params or default_params()
    geom = geom or default_geom()
    zo, x, z = _c(ev.zone_off, np.int32), _c(ev.hit_x, np.float32), _c(ev.hit_z, np.float32)
    n = lib().orc_xz_candidates(C.byref(geom), C.byref(params), _ptr(zo), _ptr(x), _ptr(z),
                                half, it, None, 0)
    out = np.zeros(n, CAND_DTYPE)
    lib().orc_xz_candidates(C.byref(geom), C.byref(params), _ptr(zo), _ptr(x), _ptr(z),
                            half, it, _ptr(out), n)
    return out


def clone_vote(cands: np.ndarray, n_pos: int) -> np.ndarray:
    c = _c(cands, CAND_DTYPE)
    keep = np.zeros(len(c), np.int32)
    lib().orc_clone_vote(_ptr(c), len(c), int(n_pos), _ptr(keep))
    return keep.astype(bool)


def uv(ev, cand, params: Params | None = None, geom: Geom | None = None):
    params = params or default_params()
    geom = geom or default_geom()
    c = _c(np.atleast_1d(cand), CAND_DTYPE)
    out = np.zeros(1, SEED_DTYPE)
    zo, x, z, i = (_c(ev.zone_off, np.int32), _c(ev.hit_x, np.float32),
                   _c(ev.hit_z, np.float32), _c(ev.hit_id, np.int32))
    ok = lib().orc_uv(C.byref(geom), C.byref(params), _ptr(zo), _ptr(x), _ptr(z), _ptr(i),
                      _ptr(c), _ptr(out))
    return out[0] if ok else None


def _ut_args(ut):
    """(off [5], x, id) of one event's UT hits as pointers, or three NULLs;
    the arrays are returned too, so that they outlive the call."""
    if ut is None:
        return [None, None, None], []
    a = [_c(ut["off"], np.int32), _c(ut["x"], np.float32), _c(ut["id"], np.int32)]
    assert len(a[0]) == NUT + 1
    return [_ptr(x) for x in a], a


def match(seeds: np.ndarray, velo: dict, params: Params | None = None,
          geom: Geom | None = None, ut: dict | None = None) -> np.ndarray:
    """Matching of one event; ut: its UT hits {off [5], x, id} or None."""
    params = params or default_params()
    geom = geom or default_geom()
    s = _c(seeds, SEED_DTYPE)
    arr = [_c(velo[k], np.float32) for k in ("x", "y", "z", "tx", "ty")]
    vid = _c(velo["id"], np.int32)
    nv = len(vid)
    up, keep = _ut_args(ut)
    args = [C.byref(geom), C.byref(params), _ptr(s), len(s), nv] + [_ptr(a) for a in arr] + \
        [_ptr(vid)] + up
    n = lib().orc_match(*args, None, 0)
    out = np.zeros(n, LONG_DTYPE)
    lib().orc_match(*args, _ptr(out), n)
    return out


def match_pairs(seeds: np.ndarray, velo: dict, params: Params | None = None,
                geom: Geom | None = None, ut: dict | None = None) -> np.ndarray:
    """The pairs that pass the preselection, the chi2_match cut and (ut_mode
    1) the UT hit count, with the network's eight inputs and (final_sel 1)
    their ghost probability."""
    params = params or default_params()
    geom = geom or default_geom()
    s = _c(seeds, SEED_DTYPE)
    arr = [_c(velo[k], np.float32) for k in ("x", "y", "z", "tx", "ty")]
    nv = len(arr[0])
    up, keep = _ut_args(ut)
    args = [C.byref(geom), C.byref(params), _ptr(s), len(s), nv] + [_ptr(a) for a in arr] + up
    n = lib().orc_match_pairs(*args, None, 0)
    out = np.zeros(n, PAIR_DTYPE)
    lib().orc_match_pairs(*args, _ptr(out), n)
    return out


def ut_window(layer: int, tight: bool, qop: float, params: Params | None = None) -> float:
    return float(lib().orc_ut_window(C.byref(params or default_params()), int(layer),
                                     int(bool(tight)), float(qop)))


def ghost_prob(params: Params, f) -> float:
    x = np.ascontiguousarray(f, np.float64)
    assert x.shape == (NN_IN,)
    return float(lib().orc_ghost_prob(C.byref(params), _ptr(x)))


class Result:
    def __init__(self, seed_off, seeds, long_off, longs, near=None):
        self.seed_off, self.seeds, self.long_off, self.longs = seed_off, seeds, long_off, longs
        self.near = near if near is not None else np.zeros(0, NEAR_DTYPE)

    def event_near(self, e):
        return self.near[self.near["event"] == e]

    def event_seeds(self, e):
        return self.seeds[self.seed_off[e]:self.seed_off[e + 1]]

    def event_longs(self, e):
        return self.longs[self.long_off[e]:self.long_off[e + 1]]


def run(batch, params: Params | None = None, geom: Geom | None = None,
        threads: int = 1, margins: bool = True) -> Result:
    """Seeding + Matching of every event of `batch` (an events.Batch).
    margins=False skips the margin log's own passes (same tracks; used to
    time the method alone)."""
    params = params or default_params()
    geom = geom or default_geom()
    arrs = [_c(batch.zone_off, np.int32), _c(batch.hit_x, np.float32),
            _c(batch.hit_z, np.float32), _c(batch.hit_id, np.int32),
            _c(batch.velo_off, np.int32), _c(batch.velo_x, np.float32),
            _c(batch.velo_y, np.float32), _c(batch.velo_z, np.float32),
            _c(batch.velo_tx, np.float32), _c(batch.velo_ty, np.float32),
            _c(batch.velo_id, np.int32)]
    has_ut = getattr(batch, "ut_off", None) is not None
    if params.ut_mode == 1 and not has_ut:
        raise ValueError("ut_mode 1 needs a batch with UT hits")
    ut = [_c(batch.ut_off, np.int32), _c(batch.ut_x, np.float32), _c(batch.ut_id, np.int32)] \
        if has_ut else None
    res = _Result()
    n_ev = batch.n_events
    rc = lib().orc_run(C.byref(geom), C.byref(params), n_ev, _ptr(arrs[0]), _ptr(arrs[1]),
                       _ptr(arrs[2]), _ptr(arrs[3]), _ptr(arrs[4]), _ptr(arrs[5]),
                       _ptr(arrs[6]), _ptr(arrs[7]), _ptr(arrs[8]), _ptr(arrs[9]),
                       _ptr(arrs[10]), *([_ptr(a) for a in ut] if ut else [None] * 3),
                       int(threads), int(bool(margins)), C.byref(res))
    if rc != 0:
        raise RuntimeError(f"orc_run failed: {rc}")
    try:
        seed_off = np.ctypeslib.as_array(res.seed_off, (n_ev + 1,)).copy()
        long_off = np.ctypeslib.as_array(res.long_off, (n_ev + 1,)).copy()
        ns, nl = res.n_seeds, res.n_longs
        seeds = np.frombuffer((C.c_char * (ns * SEED_DTYPE.itemsize)).from_address(res.seeds),
                              SEED_DTYPE).copy() if ns else np.zeros(0, SEED_DTYPE)
        longs = np.frombuffer((C.c_char * (nl * LONG_DTYPE.itemsize)).from_address(res.longs),
                              LONG_DTYPE).copy() if nl else np.zeros(0, LONG_DTYPE)
        nn = res.n_near
        near = np.frombuffer((C.c_char * (nn * NEAR_DTYPE.itemsize)).from_address(res.near),
                             NEAR_DTYPE).copy() if nn else np.zeros(0, NEAR_DTYPE)
    finally:
        lib().orc_free(C.byref(res))
    return Result(seed_off, seeds, long_off, longs, near)
