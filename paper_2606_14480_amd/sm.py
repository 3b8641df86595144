"""Python binding of libsm (include/sm.h): ctypes argument marshalling only.

Device memory and streams come from PyTorch; every step of Seeding and
Matching runs in the library's HIP kernels.  There is no fallback: if the
library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsm.so")
NL = 12
NUT = 4

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "or python paper_2606_14480_amd/build.py")

# PyTorch ships its own HIP runtime.  Loading it first makes libsm.so bind to
# that same runtime (the shared-object name matches), so device memory,
# streams and the GPU itself are shared by one runtime in this process; a
# second runtime loaded after torch's would not find the GPU.
import torch  # noqa: E402,F401

# limits of the allocation-free call (include/sm.h)
NOALLOC_MAX_EVENTS = 1024
NOALLOC_MAX_VELO = 262144
NOALLOC_WORKGROUPS = 128

OK, ERR_INVALID, ERR_UNSORTED, ERR_CAPACITY, ERR_OOM, ERR_DEVICE, ERR_BUSY, ERR_NOT_READY, \
    ERR_LIMIT = 0, -1, -2, -3, -4, -5, -6, -7, -8


class SmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


class Geometry(C.Structure):
    _fields_ = [("z", C.c_double * NL), ("tan_stereo", C.c_double * NL), ("z_ref", C.c_double),
                ("ut_z", C.c_double * NUT), ("ut_tan", C.c_double * NUT)]


NN_INPUTS, NN_HIDDEN = 8, 32
GHOST_NN_PATH = os.path.join(PKG, "ghost_nn.json")


class GhostNN(C.Structure):
    _fields_ = [("mean", C.c_double * NN_INPUTS), ("scale", C.c_double * NN_INPUTS),
                ("w1", (C.c_double * NN_INPUTS) * NN_HIDDEN), ("b1", C.c_double * NN_HIDDEN),
                ("w2", C.c_double * NN_HIDDEN), ("b2", C.c_double)]


def ghost_nn_weights(path: str = GHOST_NN_PATH) -> dict:
    """The ghost network's weights shipped with the package (trained on the
    synthetic generator's truth; the paper publishes none)."""
    import json
    with open(path) as f:
        return json.load(f)


def _set_ghost_nn(nn: GhostNN, w: dict) -> None:
    for i in range(NN_INPUTS):
        nn.mean[i] = float(w["mean"][i])
        nn.scale[i] = float(w["scale"][i])
    for j in range(NN_HIDDEN):
        for i in range(NN_INPUTS):
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


class Config(C.Structure):
    _fields_ = [("device", C.c_int32), ("n_slots", C.c_int32), ("seed_wgs", C.c_int32),
                ("match_wgs", C.c_int32), ("lds_hits", C.c_int32), ("validate", C.c_int32),
                ("mem_budget", C.c_int64)]


class Batch(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("pad", C.c_int32), ("n_hits", C.c_int64),
                ("n_velo", C.c_int64), ("zone_off", C.c_void_p), ("hit_x", C.c_void_p),
                ("hit_z", C.c_void_p), ("hit_id", C.c_void_p), ("velo_off", C.c_void_p),
                ("velo_x", C.c_void_p), ("velo_y", C.c_void_p), ("velo_z", C.c_void_p),
                ("velo_tx", C.c_void_p), ("velo_ty", C.c_void_p), ("velo_id", C.c_void_p),
                ("n_ut", C.c_int64), ("ut_off", C.c_void_p), ("ut_x", C.c_void_p),
                ("ut_id", C.c_void_p)]


class Shape(C.Structure):
    _fields_ = [("max_mean_item_hits", C.c_int32), ("max_events", C.c_int32),
                ("seed_wgs", C.c_int32), ("lds_hits", C.c_int32)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class KernelTimes(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("prepare", "seed_big", "seed", "seed_fused", "match", "copy",
                                         "total")]

    def as_dict(self):
        return {n: float(getattr(self, n)) for n, _ in self._fields_}


class Out(C.Structure):
    _fields_ = [("seed_cap", C.c_int64), ("long_cap", C.c_int64), ("seed_off", C.c_void_p),
                ("seeds", C.c_void_p), ("long_off", C.c_void_p), ("longs", C.c_void_p),
                ("n_seeds", C.c_int64), ("n_longs", C.c_int64)]


SEED_DTYPE = np.dtype([("ax", "f4"), ("bx", "f4"), ("cx", "f4"), ("y0", "f4"), ("ty", "f4"),
                       ("chi2_x", "f4"), ("chi2_y", "f4"), ("score", "f4"),
                       ("n_x", "i4"), ("n_uv", "i4"), ("half", "i4"), ("iter", "i4"),
                       ("hits", "i4", NL)])
LONG_DTYPE = np.dtype([("velo_idx", "i4"), ("seed_idx", "i4"), ("velo_id", "i4"),
                       ("qop", "f4"), ("chi2", "f4"), ("z_match", "f4"), ("dx", "f4"),
                       ("dy", "f4"), ("dtx", "f4"), ("dty", "f4"), ("ghost_prob", "f4"),
                       ("n_ut", "i4"), ("ut_hits", "i4", NUT)])
assert SEED_DTYPE.itemsize == 96 and LONG_DTYPE.itemsize == 64

_lib = C.CDLL(LIB_PATH)
_P = C.POINTER
_lib.sm_default_geometry.argtypes = [_P(Geometry)]
_lib.sm_default_params.argtypes = [_P(Params)]
_lib.sm_create.argtypes = [_P(Geometry), _P(Params), _P(Config), _P(C.c_void_p)]
_lib.sm_create.restype = C.c_int
_lib.sm_run.argtypes = [C.c_void_p, _P(Batch), _P(Out), C.c_void_p]
_lib.sm_run.restype = C.c_int
_lib.sm_run_plain.argtypes = [C.c_void_p, _P(Batch), _P(Out), C.c_void_p]
_lib.sm_run_plain.restype = C.c_int
_lib.sm_run_noalloc.argtypes = [C.c_void_p, _P(Batch), _P(Out), C.c_void_p]
_lib.sm_run_noalloc.restype = C.c_int
_lib.sm_submit.argtypes = [C.c_void_p, _P(Batch), _P(Out), _P(C.c_int64)]
_lib.sm_submit.restype = C.c_int
_lib.sm_poll.argtypes = [C.c_void_p, C.c_int64, C.c_int]
_lib.sm_poll.restype = C.c_int
_lib.sm_profile.argtypes = [C.c_void_p, _P(Batch), _P(Out), C.c_void_p, _P(KernelTimes)]
_lib.sm_profile.restype = C.c_int
_lib.sm_set_shapes.argtypes = [C.c_void_p, _P(Shape), C.c_int32]
_lib.sm_set_shapes.restype = C.c_int
_lib.sm_launch_shape.argtypes = [C.c_void_p, _P(Batch), _P(Shape)]
_lib.sm_launch_shape.restype = C.c_int
_lib.sm_batch_bytes.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64]
_lib.sm_batch_bytes.restype = C.c_int64
_lib.sm_destroy.argtypes = [C.c_void_p]
_lib.sm_destroy.restype = C.c_int
_lib.sm_status_str.argtypes = [C.c_int]
_lib.sm_status_str.restype = C.c_char_p

EXPORTS = ("sm_default_geometry", "sm_default_params", "sm_create", "sm_run", "sm_run_plain",
           "sm_run_noalloc", "sm_submit", "sm_poll", "sm_profile", "sm_set_shapes",
           "sm_launch_shape", "sm_batch_bytes", "sm_destroy", "sm_status_str")


def lib():
    return _lib


def status_str(s: int) -> str:
    return _lib.sm_status_str(int(s)).decode()


def default_geometry() -> Geometry:
    g = Geometry()
    _lib.sm_default_geometry(C.byref(g))
    return g


def default_params(**over) -> Params:
    """The library's defaults with fields replaced.  ghost_nn takes a dict of
    weights; final_sel=1 without ghost_nn takes the package's weights."""
    p = Params()
    _lib.sm_default_params(C.byref(p))
    for k, v in over.items():
        if k in Params.ARRAYS:
            for i, x in enumerate(v):
                getattr(p, k)[i] = x
        elif k == "ghost_nn":
            _set_ghost_nn(p.ghost_nn, v)
        else:
            setattr(p, k, v)
    if over.get("final_sel") == 1 and "ghost_nn" not in over:
        _set_ghost_nn(p.ghost_nn, ghost_nn_weights())
    return p


class DeviceBatch:
    """A batch resident in device memory (torch tensors) plus its sm_batch."""

    def __init__(self, host, device="cuda"):
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)
        self.n_events = host.n_events
        self.zone_off = t(host.zone_off, torch.int32)
        self.hit_x = t(host.hit_x, torch.float32)
        self.hit_z = t(host.hit_z, torch.float32)
        self.hit_id = t(host.hit_id, torch.int32)
        self.velo_off = t(host.velo_off, torch.int32)
        self.velo_x = t(host.velo_x, torch.float32)
        self.velo_y = t(host.velo_y, torch.float32)
        self.velo_z = t(host.velo_z, torch.float32)
        self.velo_tx = t(host.velo_tx, torch.float32)
        self.velo_ty = t(host.velo_ty, torch.float32)
        self.velo_id = t(host.velo_id, torch.int32)
        self.n_hits = int(host.n_hits)
        self.n_velo = int(host.n_velo)
        # UT hits, when the host batch has them (read only with ut_mode 1)
        has_ut = getattr(host, "ut_off", None) is not None
        self.ut_off = t(host.ut_off, torch.int32) if has_ut else None
        self.ut_x = t(host.ut_x, torch.float32) if has_ut else None
        self.ut_id = t(host.ut_id, torch.int32) if has_ut else None
        self.n_ut = int(host.ut_off[-1]) if has_ut else 0
        ptr = lambda a: a.data_ptr() if a is not None else None
        self.c = Batch(n_events=self.n_events, pad=0, n_hits=self.n_hits, n_velo=self.n_velo,
                       zone_off=self.zone_off.data_ptr(), hit_x=self.hit_x.data_ptr(),
                       hit_z=self.hit_z.data_ptr(), hit_id=self.hit_id.data_ptr(),
                       velo_off=self.velo_off.data_ptr(), velo_x=self.velo_x.data_ptr(),
                       velo_y=self.velo_y.data_ptr(), velo_z=self.velo_z.data_ptr(),
                       velo_tx=self.velo_tx.data_ptr(), velo_ty=self.velo_ty.data_ptr(),
                       velo_id=self.velo_id.data_ptr(), n_ut=self.n_ut, ut_off=ptr(self.ut_off),
                       ut_x=ptr(self.ut_x), ut_id=ptr(self.ut_id))


class DeviceOut:
    """Caller-allocated outputs (torch uint8 buffers viewed as the C structs)."""

    def __init__(self, n_events, seed_cap, long_cap, device="cuda"):
        import torch
        self.n_events = n_events
        self.seed_off = torch.zeros(n_events + 1, dtype=torch.int32, device=device)
        self.long_off = torch.zeros(n_events + 1, dtype=torch.int32, device=device)
        self.seeds = torch.empty(max(seed_cap, 1) * SEED_DTYPE.itemsize, dtype=torch.uint8, device=device)
        self.longs = torch.empty(max(long_cap, 1) * LONG_DTYPE.itemsize, dtype=torch.uint8, device=device)
        self.c = Out(seed_cap=seed_cap, long_cap=long_cap, seed_off=self.seed_off.data_ptr(),
                     seeds=self.seeds.data_ptr(), long_off=self.long_off.data_ptr(),
                     longs=self.longs.data_ptr(), n_seeds=0, n_longs=0)

    @property
    def n_seeds(self):
        return int(self.c.n_seeds)

    @property
    def n_longs(self):
        return int(self.c.n_longs)

    def to_host(self):
        """(seed_off, seeds, long_off, longs) as numpy arrays."""
        ns, nl = self.n_seeds, self.n_longs
        seeds = self.seeds[: ns * SEED_DTYPE.itemsize].cpu().numpy().view(SEED_DTYPE)
        longs = self.longs[: nl * LONG_DTYPE.itemsize].cpu().numpy().view(LONG_DTYPE)
        return self.seed_off.cpu().numpy(), seeds, self.long_off.cpu().numpy(), longs


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    """A library context.  shapes: the table of launch shapes by batch class
    (list of dicts with max_mean_item_hits, max_events, seed_wgs, lds_hits);
    "tuned" (the default) takes the autotuner's committed table for this
    device, unless seed_wgs or lds_hits are given, which then fix the
    launch shape of every batch; [] keeps the built-in choice."""

    def __init__(self, geometry: Geometry | None = None, params: Params | None = None,
                 device: int = 0, n_slots: int = 2, seed_wgs: int = 0, lds_hits: int = 0,
                 validate: bool = False, mem_budget: int = 0, match_wgs: int = 0,
                 shapes="tuned"):
        self.geometry = geometry or default_geometry()
        self.params = params or default_params()
        cfg = Config(device=device, n_slots=n_slots, seed_wgs=seed_wgs, match_wgs=match_wgs,
                     lds_hits=lds_hits, validate=int(validate), mem_budget=mem_budget)
        h = C.c_void_p()
        st = _lib.sm_create(C.byref(self.geometry), C.byref(self.params), C.byref(cfg), C.byref(h))
        if st != OK:
            raise SmError(st, "sm_create")
        self.h = h
        self.shape_source = "built-in"
        if shapes == "tuned":
            shapes = [] if (seed_wgs or lds_hits) else _tuned_shapes(device)
            if shapes:
                self.shape_source = "autotune"
        elif shapes:
            self.shape_source = "given"
        if shapes:
            self.set_shapes(shapes)

    def set_shapes(self, shapes, check: bool = True) -> int:
        arr = (Shape * max(len(shapes), 1))()
        for i, e in enumerate(shapes):
            arr[i] = Shape(**{k: int(e[k]) for k in ("max_mean_item_hits", "max_events",
                                                      "seed_wgs", "lds_hits")})
        st = _lib.sm_set_shapes(self.h, arr, len(shapes))
        if check and st != OK:
            raise SmError(st, "sm_set_shapes")
        return st

    def launch_shape(self, batch) -> dict:
        """The launch shape a batched call takes for `batch` (a DeviceBatch,
        or anything with n_events and n_hits)."""
        b = Batch(n_events=int(batch.n_events), n_hits=int(batch.n_hits))
        sh = Shape()
        st = _lib.sm_launch_shape(self.h, C.byref(b), C.byref(sh))
        if st != OK:
            raise SmError(st, "sm_launch_shape")
        return sh.as_dict()

    def close(self):
        if getattr(self, "h", None):
            _lib.sm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def run(self, batch: DeviceBatch, out: DeviceOut, stream=None, plain: bool = False,
            check: bool = True) -> int:
        fn = _lib.sm_run_plain if plain else _lib.sm_run
        st = fn(self.h, C.byref(batch.c), C.byref(out.c), _stream_ptr(stream))
        if check and st != OK:
            raise SmError(st, "sm_run_plain" if plain else "sm_run")
        return st

    def run_noalloc(self, batch: DeviceBatch, out: DeviceOut, stream=None,
                    check: bool = True) -> int:
        """sm_run_noalloc: the batched computation on the device's static
        scratch, with no allocation inside the call."""
        st = _lib.sm_run_noalloc(self.h, C.byref(batch.c), C.byref(out.c), _stream_ptr(stream))
        if check and st != OK:
            raise SmError(st, "sm_run_noalloc")
        return st

    def profile(self, batch: DeviceBatch, out: DeviceOut, stream=None) -> dict:
        t = KernelTimes()
        st = _lib.sm_profile(self.h, C.byref(batch.c), C.byref(out.c), _stream_ptr(stream),
                             C.byref(t))
        if st != OK:
            raise SmError(st, "sm_profile")
        return t.as_dict()

    def submit(self, batch: DeviceBatch, out: DeviceOut):
        return self.submit_c(batch.c, out.c)

    def submit_c(self, batch_c: Batch, out_c: Out):
        """sm_submit on raw structs; both must stay alive until the ticket completes."""
        t = C.c_int64()
        st = _lib.sm_submit(self.h, C.byref(batch_c), C.byref(out_c), C.byref(t))
        return st, t.value

    def run_c(self, batch_c: Batch, out_c: Out, stream=None, plain: bool = False) -> int:
        fn = _lib.sm_run_plain if plain else _lib.sm_run
        st = fn(self.h, C.byref(batch_c), C.byref(out_c), _stream_ptr(stream))
        if st != OK:
            raise SmError(st, "sm_run_plain" if plain else "sm_run")
        return st

    def poll(self, ticket: int, wait: bool = False) -> int:
        return _lib.sm_poll(self.h, C.c_int64(ticket), int(wait))

    def batch_bytes(self, n_events, n_hits, n_velo) -> int:
        return _lib.sm_batch_bytes(self.h, n_events, n_hits, n_velo)


def _tuned_shapes(device: int) -> list:
    """The autotuner's committed launch shapes for this device (or none)."""
    try:
        import torch
        name = torch.cuda.get_device_properties(device).name
    except Exception:
        return []
    from . import autotune
    return autotune.shapes_for(name)


def reconstruct(ctx: Context, host_batch, plain: bool = False, seed_cap=None, long_cap=None):
    """Convenience: copy a host batch to the device, run, return host arrays.
    If the outputs do not fit the first guess, runs once more with the sizes
    the library reported."""
    db = DeviceBatch(host_batch)
    out = DeviceOut(host_batch.n_events, seed_cap or max(host_batch.n_hits // 4, 16),
                    long_cap or max(host_batch.n_velo * 2, 16))
    st = ctx.run(db, out, plain=plain, check=False)
    if st == ERR_CAPACITY:
        out = DeviceOut(host_batch.n_events, max(out.n_seeds, 16), max(out.n_longs, 16))
        st = ctx.run(db, out, plain=plain, check=False)
    if st != OK:
        raise SmError(st, "sm_run_plain" if plain else "sm_run")
    return out.to_host()
