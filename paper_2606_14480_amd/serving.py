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


def pin(batch) -> dict:
    """The batch's arrays in pinned host memory (where a trigger's network
    receive would leave them), ready for an asynchronous DMA."""
    import torch
    out = {}
    for f in _FIELDS:
        a = np.ascontiguousarray(getattr(batch, f))
        t = torch.empty(len(a), dtype=torch.from_numpy(a[:0]).dtype, pin_memory=True)
        if len(a):
            t.numpy()[:] = a
        out[f] = t
    return out


@dataclasses.dataclass
class Request:
    rid: int
    batch: object          # events.Batch (host)
    arrival: float         # seconds from the start of the run
    pinned: dict | None = None


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
    """Resident device buffers of one serving slot (torch tensors)."""

    def __init__(self, max_events: int, max_hits: int, max_velo: int, device="cuda"):
        import torch
        from . import sm
        f32, i32 = torch.float32, torch.int32
        self.cap = (max_events, max_hits, max_velo)
        z = lambda n, dt: torch.zeros(max(n, 1), dtype=dt, device=device)
        self.zone_off = z(max_events * 24 + 1, i32)
        self.hit_x, self.hit_z, self.hit_id = z(max_hits, f32), z(max_hits, f32), z(max_hits, i32)
        self.velo_off = z(max_events + 1, i32)
        self.velo = {k: z(max_velo, f32) for k in ("x", "y", "z", "tx", "ty")}
        self.velo_id = z(max_velo, i32)
        self.out = sm.DeviceOut(max_events, max_hits // 4 + 1024, max_velo + 1024, device)
        self.c = sm.Batch()
        # pinned host staging, one buffer per device array
        self.pinned = {}
        for name, t in self._arrays().items():
            self.pinned[name] = torch.empty(t.numel(), dtype=t.dtype, pin_memory=True)

    def _arrays(self):
        d = {"zone_off": self.zone_off, "hit_x": self.hit_x, "hit_z": self.hit_z,
             "hit_id": self.hit_id, "velo_off": self.velo_off, "velo_id": self.velo_id}
        d.update({"velo_" + k: v for k, v in self.velo.items()})
        return d

    def bytes(self) -> int:
        e, h, v = self.cap
        return (e * 24 + 1) * 4 + h * 12 + (e + 1) * 4 + v * 24 + \
            self.out.seeds.numel() + self.out.longs.numel() + 2 * (e + 1) * 4

    def load(self, b, stream, pinned: dict | None = None):
        """Copy a host batch into the resident buffers on `stream` (straight
        from `pinned` when the request arrived in pinned memory)."""
        import torch
        from . import sm
        e, h, v = b.n_events, b.n_hits, b.n_velo
        if e > self.cap[0] or h > self.cap[1] or v > self.cap[2]:
            raise ValueError("request larger than the slot buffers")
        dev = self._arrays()
        with torch.cuda.stream(stream):
            for name in _FIELDS:
                a = getattr(b, name)
                n = len(a)
                if not n:
                    continue
                if pinned is not None:
                    src = pinned[name]
                else:
                    src = self.pinned[name][:n]
                    src.numpy()[:] = a
                dev[name][:n].copy_(src, non_blocking=True)
        self.c = sm.Batch(n_events=e, pad=0, n_hits=h, n_velo=v,
                          zone_off=self.zone_off.data_ptr(), hit_x=self.hit_x.data_ptr(),
                          hit_z=self.hit_z.data_ptr(), hit_id=self.hit_id.data_ptr(),
                          velo_off=self.velo_off.data_ptr(), velo_x=self.velo["x"].data_ptr(),
                          velo_y=self.velo["y"].data_ptr(), velo_z=self.velo["z"].data_ptr(),
                          velo_tx=self.velo["tx"].data_ptr(), velo_ty=self.velo["ty"].data_ptr(),
                          velo_id=self.velo_id.data_ptr())
        self.out.n_events = e


class Server:
    """Continuous batching over the library's serving slots."""

    def __init__(self, ctx, n_slots: int, max_events: int, max_hits: int, max_velo: int,
                 mem_budget: int | None = None):
        import torch
        self.ctx = ctx
        self.slots = [SlotBuffers(max_events, max_hits, max_velo) for _ in range(n_slots)]
        self.free = collections.deque(range(n_slots))
        self.copy_stream = torch.cuda.Stream()
        self.mem_budget = mem_budget
        self.in_use = 0
        self.peak_in_use = 0

    def _needs(self, b) -> int:
        return self.ctx.batch_bytes(b.n_events, b.n_hits, b.n_velo)

    def serve(self, requests: list, clock=time.perf_counter) -> list:
        """Serve requests (sorted by arrival); returns Results in completion order."""
        import torch
        from . import sm
        pending = collections.deque(requests)
        inflight = {}   # ticket -> (slot, request, admitted)
        done = []
        t0 = clock()
        while pending or inflight:
            now = clock() - t0
            # admit every arrived request that finds a free slot and memory
            while pending and pending[0].arrival <= now and self.free:
                req = pending[0]
                need = self._needs(req.batch)
                if self.mem_budget is not None and self.in_use + need > self.mem_budget and inflight:
                    break
                pending.popleft()
                si = self.free.popleft()
                slot = self.slots[si]
                slot.load(req.batch, self.copy_stream, req.pinned)
                self.copy_stream.synchronize()
                out = slot.out
                out.c.seed_off = out.seed_off.data_ptr()
                out.c.long_off = out.long_off.data_ptr()
                st, ticket = self.ctx.submit_c(slot.c, out.c)
                if st == sm.ERR_BUSY:          # library slots all taken: retry later
                    self.free.appendleft(si)
                    pending.appendleft(req)
                    break
                if st != sm.OK:
                    raise sm.SmError(st, "sm_submit")
                self.in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                inflight[ticket] = (si, req, clock() - t0, need)
            # retire finished batches
            for ticket in list(inflight):
                st = self.ctx.poll(ticket, wait=False)
                if st == sm.ERR_NOT_READY:
                    continue
                si, req, adm, need = inflight.pop(ticket)
                if st != sm.OK:
                    raise sm.SmError(st, "sm_poll")
                slot = self.slots[si]
                so, seeds, lo, longs = slot.out.to_host()
                done.append(Result(req.rid, req.batch.n_events, req.arrival, adm, clock() - t0,
                                   so[:req.batch.n_events + 1], seeds, lo[:req.batch.n_events + 1],
                                   longs))
                self.free.append(si)
                self.in_use -= need
            if not inflight and pending and pending[0].arrival > clock() - t0:
                time.sleep(min(1e-4, max(0.0, pending[0].arrival - (clock() - t0))))
        return done


def serve_plain(ctx, requests: list, max_events: int, max_hits: int, max_velo: int,
                clock=time.perf_counter) -> list:
    """The same arrival stream, one request at a time through the plain form."""
    slot = SlotBuffers(max_events, max_hits, max_velo)
    import torch
    stream = torch.cuda.current_stream()
    out = []
    t0 = clock()
    for req in requests:
        while clock() - t0 < req.arrival:
            pass
        adm = clock() - t0
        slot.load(req.batch, stream, req.pinned)
        ctx.run_c(slot.c, slot.out.c, plain=True)
        so, seeds, lo, longs = slot.out.to_host()
        out.append(Result(req.rid, req.batch.n_events, req.arrival, adm, clock() - t0,
                          so[:req.batch.n_events + 1], seeds, lo[:req.batch.n_events + 1], longs))
    return out


def summarize(results: list, wall: float | None = None) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    n_ev = sum(r.n_events for r in results)
    span = wall if wall is not None else (max(r.done for r in results) - min(r.arrival for r in results))
    return {"requests": len(results), "events": n_ev, "events_per_s": n_ev / span,
            "latency_ms_p50": float(np.percentile(lat, 50)),
            "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_max": float(lat.max())}
