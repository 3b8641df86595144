"""Trigger-style serving loop over the C-ABI (continuous batching).

Event batches arrive as a Poisson process.  A batch is admitted as soon as a
serving slot of the library is free and its device memory fits the budget;
admitted batches run on their slots' streams while later ones are admitted,
so their work overlaps on the device.  Each slot keeps its input and output
buffers resident in device memory (sized for the largest batch) and only
copies a request's hits and VELO states in.  Latency is arrival -> results
ready.  The same stream can be replayed through the plain form (one kernel
sequence per event) for comparison.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


_FIELDS = ("zone_off", "hit_x", "hit_z", "hit_id", "velo_off", "velo_id", "velo_x", "velo_y",
           "velo_z", "velo_tx", "velo_ty")
_ALIGN = 256


def layout(n_events: int, n_hits: int, n_velo: int):
    """Byte offsets of every input array of a batch packed into one buffer
    (each array 256-byte aligned), and the total size."""
    counts = {"zone_off": n_events * 24 + 1, "hit_x": n_hits, "hit_z": n_hits, "hit_id": n_hits,
              "velo_off": n_events + 1, "velo_id": n_velo, "velo_x": n_velo, "velo_y": n_velo,
              "velo_z": n_velo, "velo_tx": n_velo, "velo_ty": n_velo}
    off, pos = {}, 0
    for f in _FIELDS:
        off[f] = (pos, counts[f])
        pos += -(-counts[f] * 4 // _ALIGN) * _ALIGN
    return off, max(pos, _ALIGN)


@dataclasses.dataclass
class Packed:
    """A batch packed into one pinned host buffer (where a trigger's network
    receive would leave it), ready for a single asynchronous DMA."""
    buf: object            # torch uint8 tensor, pinned
    offsets: dict
    nbytes: int


def _pack_into(batch, host_u8: np.ndarray, offsets: dict):
    for f in _FIELDS:
        a = np.ascontiguousarray(getattr(batch, f))
        o, n = offsets[f]
        if n:
            host_u8[o:o + 4 * n] = a.view(np.uint8)


def pin(batch) -> Packed:
    import torch
    offsets, nbytes = layout(batch.n_events, batch.n_hits, batch.n_velo)
    t = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    _pack_into(batch, t.numpy(), offsets)
    return Packed(t, offsets, nbytes)


class EventPool:
    """Events packed once into one pinned host buffer (where a trigger's
    network receive would leave them).  A request is a run of consecutive
    events of the pool: its hits and VELO states are contiguous slices of
    the pool's arrays, copied straight from there; only its zone and VELO
    offsets are rebased on the host."""

    def __init__(self, batch):
        self.n_events = batch.n_events
        self.offsets, self.nbytes = layout(batch.n_events, batch.n_hits, batch.n_velo)
        self.packed = pin(batch)
        self.zone_off = np.asarray(batch.zone_off, np.int64)
        self.velo_off = np.asarray(batch.velo_off, np.int64)

    def sizes(self, first: int, n: int):
        """(events, hits, VELO states) of events [first, first + n)."""
        h = self.zone_off[(first + n) * 24] - self.zone_off[first * 24]
        v = self.velo_off[first + n] - self.velo_off[first]
        return n, int(h), int(v)


@dataclasses.dataclass
class Request:
    rid: int
    batch: object          # events.Batch (host), or None for a slice of `pool`
    arrival: float         # seconds from the start of the run
    pinned: Packed | None = None
    pool: EventPool | None = None
    first: int = 0         # first event of the slice of `pool`
    count: int = 0         # events of the slice of `pool`

    @property
    def n_events(self) -> int:
        return self.batch.n_events if self.batch is not None else self.count

    def sizes(self):
        if self.batch is not None:
            return self.batch.n_events, self.batch.n_hits, self.batch.n_velo
        return self.pool.sizes(self.first, self.count)


@dataclasses.dataclass
class Result:
    rid: int
    n_events: int
    arrival: float
    admitted: float
    done: float
    seed_off: np.ndarray
    seeds: np.ndarray
    long_off: np.ndarray
    longs: np.ndarray

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_arrivals(rate_hz: float, n: int, seed: int = 7) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))


class SlotBuffers:
    """Resident buffers of one serving slot: one device input arena, the
    device outputs, and pinned host staging for inputs and results."""

    def __init__(self, max_events: int, max_hits: int, max_velo: int, device="cuda"):
        import torch
        from . import sm
        self.cap = (max_events, max_hits, max_velo)
        _, nbytes = layout(max_events, max_hits, max_velo)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.staging = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        seed_cap, long_cap = max_hits // 8 + 1024, max_velo + 1024
        self.out = sm.DeviceOut(max_events, seed_cap, long_cap, device)
        self.h_seed_off = torch.empty(max_events + 1, dtype=torch.int32, pin_memory=True)
        self.h_long_off = torch.empty(max_events + 1, dtype=torch.int32, pin_memory=True)
        self.h_seeds = torch.empty(self.out.seeds.numel(), dtype=torch.uint8, pin_memory=True)
        self.h_longs = torch.empty(self.out.longs.numel(), dtype=torch.uint8, pin_memory=True)
        self.c = sm.Batch()
        self.n_events = 0
        self.fetched = None

    def bytes(self) -> int:
        return self.arena.numel() + self.out.seeds.numel() + self.out.longs.numel() + \
            2 * 4 * (self.cap[0] + 1)

    def load(self, b, stream, packed: Packed | None = None):
        """Copy a host batch into the arena on `stream` with one DMA (straight
        from `packed` when the request arrived packed in pinned memory)."""
        import torch
        from . import sm
        e, h, v = b.n_events, b.n_hits, b.n_velo
        if e > self.cap[0] or h > self.cap[1] or v > self.cap[2]:
            raise ValueError("request larger than the slot buffers")
        if packed is None:
            offsets, nbytes = layout(e, h, v)
            _pack_into(b, self.staging.numpy(), offsets)
            src = self.staging[:nbytes]
        else:
            offsets, nbytes, src = packed.offsets, packed.nbytes, packed.buf
        with torch.cuda.stream(stream):
            self.arena[:nbytes].copy_(src, non_blocking=True)
        base = self.arena.data_ptr()
        ptr = {f: base + offsets[f][0] for f in _FIELDS}
        self.c = sm.Batch(n_events=e, pad=0, n_hits=h, n_velo=v, zone_off=ptr["zone_off"],
                          hit_x=ptr["hit_x"], hit_z=ptr["hit_z"], hit_id=ptr["hit_id"],
                          velo_off=ptr["velo_off"], velo_x=ptr["velo_x"], velo_y=ptr["velo_y"],
                          velo_z=ptr["velo_z"], velo_tx=ptr["velo_tx"], velo_ty=ptr["velo_ty"],
                          velo_id=ptr["velo_id"])
        self.n_events = e
        self.out.n_events = e

    def load_slice(self, pool: EventPool, first: int, n: int, stream):
        """Copy events [first, first + n) of `pool` into the arena on `stream`:
        the rebased offsets from this slot's pinned staging, every other array
        straight from its slice of the pool."""
        import torch
        from . import sm
        e, h, v = pool.sizes(first, n)
        if e > self.cap[0] or h > self.cap[1] or v > self.cap[2]:
            raise ValueError("request larger than the slot buffers")
        offsets, _ = layout(e, h, v)
        h0, v0 = int(pool.zone_off[first * 24]), int(pool.velo_off[first])
        st = self.staging.numpy()
        zo, zn = offsets["zone_off"]
        st[zo:zo + 4 * zn] = (pool.zone_off[first * 24:(first + n) * 24 + 1] - h0) \
            .astype(np.int32).view(np.uint8)
        vo, vn = offsets["velo_off"]
        st[vo:vo + 4 * vn] = (pool.velo_off[first:first + n + 1] - v0).astype(np.int32).view(np.uint8)
        src = pool.packed.buf
        with torch.cuda.stream(stream):
            for f in _FIELDS:
                o, cnt = offsets[f]
                if cnt == 0:
                    continue
                if f in ("zone_off", "velo_off"):
                    self.arena[o:o + 4 * cnt].copy_(self.staging[o:o + 4 * cnt], non_blocking=True)
                else:
                    po, _ = pool.offsets[f]
                    start = po + 4 * (h0 if f.startswith("hit") else v0)
                    self.arena[o:o + 4 * cnt].copy_(src[start:start + 4 * cnt], non_blocking=True)
        base = self.arena.data_ptr()
        ptr = {f: base + offsets[f][0] for f in _FIELDS}
        self.c = sm.Batch(n_events=e, pad=0, n_hits=h, n_velo=v, zone_off=ptr["zone_off"],
                          hit_x=ptr["hit_x"], hit_z=ptr["hit_z"], hit_id=ptr["hit_id"],
                          velo_off=ptr["velo_off"], velo_x=ptr["velo_x"], velo_y=ptr["velo_y"],
                          velo_z=ptr["velo_z"], velo_tx=ptr["velo_tx"], velo_ty=ptr["velo_ty"],
                          velo_id=ptr["velo_id"])
        self.n_events = e
        self.out.n_events = e

    def load_request(self, req, stream):
        if req.batch is not None:
            self.load(req.batch, stream, req.pinned)
        else:
            self.load_slice(req.pool, req.first, req.count, stream)

    def fetch(self, stream):
        """Start the copy of this slot's results into pinned host memory on
        `stream`; returns an event that completes with it."""
        import torch
        from . import sm
        e = self.n_events
        ns, nl = self.out.n_seeds, self.out.n_longs
        with torch.cuda.stream(stream):
            self.h_seed_off[:e + 1].copy_(self.out.seed_off[:e + 1], non_blocking=True)
            self.h_long_off[:e + 1].copy_(self.out.long_off[:e + 1], non_blocking=True)
            if ns:
                nb = ns * sm.SEED_DTYPE.itemsize
                self.h_seeds[:nb].copy_(self.out.seeds[:nb], non_blocking=True)
            if nl:
                nb = nl * sm.LONG_DTYPE.itemsize
                self.h_longs[:nb].copy_(self.out.longs[:nb], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.fetched = (e, ns, nl)
        return ev

    def collect(self):
        """Host copies of the fetched results (after the fetch event)."""
        from . import sm
        e, ns, nl = self.fetched
        so = self.h_seed_off.numpy()[:e + 1].copy()
        lo = self.h_long_off.numpy()[:e + 1].copy()
        seeds = self.h_seeds.numpy()[:ns * sm.SEED_DTYPE.itemsize].copy().view(sm.SEED_DTYPE)
        longs = self.h_longs.numpy()[:nl * sm.LONG_DTYPE.itemsize].copy().view(sm.LONG_DTYPE)
        return so, seeds, lo, longs


class Server:
    """Continuous batching over the library's serving slots."""

    def __init__(self, ctx, n_slots: int, max_events: int, max_hits: int, max_velo: int,
                 mem_budget: int | None = None):
        import torch
        self.ctx = ctx
        self.slots = [SlotBuffers(max_events, max_hits, max_velo) for _ in range(n_slots)]
        self.free = collections.deque(range(n_slots))
        self.copy_stream = torch.cuda.Stream()
        self.fetch_stream = torch.cuda.Stream()
        self.mem_budget = mem_budget
        self.in_use = 0
        self.peak_in_use = 0

    def _needs(self, req) -> int:
        return self.ctx.batch_bytes(*req.sizes())

    def serve(self, requests: list, clock=time.perf_counter, keep: bool = True) -> list:
        """Serve requests (sorted by arrival); returns Results in completion
        order.  A request's slot is busy from admission until its results are
        in pinned host memory: upload, kernels, then the result copy, each
        stream-ordered and each polled, so the loop never blocks on one
        request while others can make progress.  keep=False leaves the
        results in the slot's pinned buffers (a consumer would read them
        there) and returns only their sizes."""
        import torch
        from . import sm
        pending = collections.deque(requests)
        uploading = []  # (event, slot, request, admitted, need)
        inflight = {}   # ticket -> (slot, request, admitted, need)
        draining = []   # (event, slot, request, admitted, need)
        done = []
        t0 = clock()
        while pending or uploading or inflight or draining:
            now = clock() - t0
            busy = uploading or inflight or draining
            # admit every arrived request that finds a free slot and memory
            while pending and pending[0].arrival <= now and self.free:
                req = pending[0]
                need = self._needs(req)
                if self.mem_budget is not None and self.in_use + need > self.mem_budget and busy:
                    break
                pending.popleft()
                si = self.free.popleft()
                self.slots[si].load_request(req, self.copy_stream)
                ev = torch.cuda.Event()
                ev.record(self.copy_stream)
                self.in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                uploading.append((ev, si, req, clock() - t0, need))
                busy = True
            # uploaded requests: submit to a library slot
            still = []
            for item in uploading:
                ev, si, req, adm, need = item
                if not ev.query():
                    still.append(item)
                    continue
                out = self.slots[si].out
                out.c.seed_off = out.seed_off.data_ptr()
                out.c.long_off = out.long_off.data_ptr()
                st, ticket = self.ctx.submit_c(self.slots[si].c, out.c)
                if st == sm.ERR_BUSY:          # library slots all taken: retry later
                    still.append(item)
                    continue
                if st != sm.OK:
                    raise sm.SmError(st, "sm_submit")
                inflight[ticket] = (si, req, adm, need)
            uploading = still
            # finished batches: start their result copies
            for ticket in list(inflight):
                st = self.ctx.poll(ticket, wait=False)
                if st == sm.ERR_NOT_READY:
                    continue
                si, req, adm, need = inflight.pop(ticket)
                if st != sm.OK:
                    raise sm.SmError(st, "sm_poll")
                ev = self.slots[si].fetch(self.fetch_stream)
                draining.append((ev, si, req, adm, need))
            # results in host memory: hand them out and free the slot
            still = []
            for item in draining:
                ev, si, req, adm, need = item
                if not ev.query():
                    still.append(item)
                    continue
                t_done = clock() - t0
                slot = self.slots[si]
                if keep:
                    so, seeds, lo, longs = slot.collect()
                else:
                    e, ns, nl = slot.fetched
                    so = lo = np.zeros(0, np.int32)
                    seeds = np.zeros(0, sm.SEED_DTYPE)
                    longs = np.zeros(0, sm.LONG_DTYPE)
                done.append(Result(req.rid, req.n_events, req.arrival, adm, t_done,
                                   so, seeds, lo, longs))
                self.free.append(si)
                self.in_use -= need
            draining = still
            if not (uploading or inflight or draining) and pending and \
                    pending[0].arrival > clock() - t0:
                time.sleep(min(1e-4, max(0.0, pending[0].arrival - (clock() - t0))))
        return done


def serve_plain(ctx, requests: list, max_events: int, max_hits: int, max_velo: int,
                clock=time.perf_counter) -> list:
    """The same arrival stream, one request at a time through the plain form."""
    import torch
    slot = SlotBuffers(max_events, max_hits, max_velo)
    stream = torch.cuda.current_stream()
    out = []
    t0 = clock()
    for req in requests:
        while clock() - t0 < req.arrival:
            pass
        adm = clock() - t0
        slot.load_request(req, stream)
        ctx.run_c(slot.c, slot.out.c, plain=True)
        slot.fetch(stream).synchronize()
        so, seeds, lo, longs = slot.collect()
        out.append(Result(req.rid, req.n_events, req.arrival, adm, clock() - t0,
                          so, seeds, lo, longs))
    return out


def summarize(results: list, wall: float | None = None) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    n_ev = sum(r.n_events for r in results)
    span = wall if wall is not None else (max(r.done for r in results) - min(r.arrival for r in results))
    return {"requests": len(results), "events": n_ev, "events_per_s": n_ev / span,
            "latency_ms_p50": float(np.percentile(lat, 50)),
            "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_max": float(lat.max())}
