"""Continuous-batching render server over resident layered models.

Layered models stay resident in HBM (the paper keeps only active layers on
the GPU, Sec. 3.3; here every layer of every model is resident and the
per-request layer mask and clip planes select what is drawn).  View requests
(mono or stereo, mixed resolutions, their own mask and clip planes) arrive
open-loop; the scheduler admits them in arrival order as launch slots and
the HBM budget allow, packs every admitted request into ONE gsr_render_batch
launch (one projection per model, one sort over a shared tile space, one
persistent blend), and keeps several launches in flight on separate streams
so that requests arriving while others render start on the device without
waiting for them.  A request whose pairs overflow its batch's capacity is
re-run alone with a larger capacity.

The scheduler (`Scheduler`) is independent of the device: `GpuExecutor`
drives the HIP library, `SimExecutor` replays a service-time model on a
virtual clock for host-side tests.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float           # scheduled arrival time (s, trace clock)
    model: int
    cams: list               # 1 or 2 camera dicts (scenes.make_camera)
    view: dict               # view state (scenes.view_state)
    alone: bool = False      # re-run by itself after a capacity overflow
    tries: int = 0
    admitted: float = math.nan
    done: float = math.nan
    status: int = 1          # 1 pending, 0 ok, <0 error

    @property
    def pixels(self):
        return sum(c["width"] * c["height"] for c in self.cams)


def requests_from_trace(trace):
    """scenes.poisson_trace entries -> Request objects."""
    return [Request(rid=i, arrival=t["arrival"], model=t["model"], cams=t["cams"], view=t["view"])
            for i, t in enumerate(trace)]


def nearest_rank(xs, q):
    """Nearest-rank percentile (q in [0, 100])."""
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = max(0, min(len(xs) - 1, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[k]


@dataclasses.dataclass
class ServeStats:
    latencies_ms: List[float]
    frames: int
    pixels: int
    span_s: float
    launches: int
    reruns: int
    max_bytes_in_flight: int

    def summary(self):
        lat = self.latencies_ms
        return {"requests": len(lat), "p50_ms": round(nearest_rank(lat, 50), 3),
                "p99_ms": round(nearest_rank(lat, 99), 3), "mean_ms": round(sum(lat) / max(len(lat), 1), 3),
                "frames_per_s": round(self.frames / self.span_s, 2) if self.span_s > 0 else None,
                "mpix_per_s": round(self.pixels / self.span_s / 1e6, 2) if self.span_s > 0 else None,
                "launches": self.launches, "reruns": self.reruns, "max_bytes_in_flight": self.max_bytes_in_flight}


class Scheduler:
    """Arrival-ordered admission into batched launches under a memory budget.

    executor must provide: cost(req) -> bytes, slots -> int, launch(reqs) ->
    handle, poll(handle) -> list of statuses or None while running, now() ->
    seconds, idle(seconds_hint) (sleep or advance a virtual clock).
    """

    def __init__(self, executor, budget_bytes: int, max_batch: int = 32, batched: bool = True,
                 max_tries: int = 3):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = max_batch if batched else 1
        self.batched = batched
        self.max_tries = max_tries

    def run(self, trace: List[Request]) -> ServeStats:
        ex = self.ex
        pending = collections.deque()
        arrivals = collections.deque(sorted(trace, key=lambda r: (r.arrival, r.rid)))
        in_flight = []  # (handle, reqs, bytes)
        used = 0
        max_used = 0
        launches = reruns = 0
        done = []
        t0 = ex.now()
        slots = ex.slots if self.batched else 1
        while arrivals or pending or in_flight:
            now = ex.now() - t0
            while arrivals and arrivals[0].arrival <= now:
                pending.append(arrivals.popleft())
            # retire finished launches
            still = []
            for h, reqs, nbytes in in_flight:
                st = ex.poll(h)
                if st is None:
                    still.append((h, reqs, nbytes))
                    continue
                used -= nbytes
                t_done = ex.now() - t0
                for r, s in zip(reqs, st):
                    if s == 0:
                        r.status, r.done = 0, t_done
                        done.append(r)
                    elif s == -2 and r.tries < self.max_tries:
                        r.alone, r.tries = True, r.tries + 1
                        reruns += 1
                        pending.appendleft(r)
                    else:
                        r.status, r.done = s, t_done
                        done.append(r)
            in_flight = still
            # admit in arrival order while a slot and the budget allow
            launched = False
            while pending and len(in_flight) < slots:
                batch, nbytes = [], 0
                while pending and len(batch) < self.max_batch:
                    r = pending[0]
                    c = ex.cost(r)
                    if r.alone and batch:
                        break
                    if used + nbytes + c > self.budget:
                        if not batch and not in_flight and c > self.budget:
                            # can never fit: fail it rather than block the queue
                            pending.popleft()
                            r.status, r.done = -2, ex.now() - t0
                            done.append(r)
                            continue
                        break
                    pending.popleft()
                    batch.append(r)
                    nbytes += c
                    if r.alone:
                        break
                if not batch:
                    break
                tnow = ex.now() - t0
                for r in batch:
                    r.admitted = tnow
                h = ex.launch(batch)
                launches += 1
                used += nbytes
                max_used = max(max_used, used)
                in_flight.append((h, batch, nbytes))
                launched = True
            if not launched:
                nxt = arrivals[0].arrival - (ex.now() - t0) if arrivals else None
                ex.idle(nxt if (nxt is not None and not in_flight) else None)
        span = max((r.done for r in done), default=0.0) - min((r.arrival for r in trace), default=0.0)
        ok = [r for r in done if r.status == 0]
        return ServeStats(latencies_ms=[(r.done - r.arrival) * 1e3 for r in ok], frames=sum(len(r.cams) for r in ok),
                          pixels=sum(r.pixels for r in ok), span_s=span, launches=launches, reruns=reruns,
                          max_bytes_in_flight=max_used)


class SimExecutor:
    """Virtual-clock executor: a launch of requests takes
    `fixed_s + per_pixel_s * pixels` on its slot; launches on different
    slots overlap."""

    def __init__(self, slots=2, fixed_s=2e-4, per_pixel_s=2e-10, cost_fn: Optional[Callable] = None,
                 fail: Optional[Callable] = None):
        self.slots = slots
        self.fixed_s, self.per_pixel_s = fixed_s, per_pixel_s
        self.t = 0.0
        self.cost_fn = cost_fn or (lambda r: 64 * r.pixels)
        self.fail = fail or (lambda reqs, r: 0)
        self.log = []

    def now(self):
        return self.t

    def cost(self, r):
        return self.cost_fn(r)

    def launch(self, reqs):
        dur = self.fixed_s + self.per_pixel_s * sum(r.pixels for r in reqs)
        h = {"end": self.t + dur, "status": [self.fail(reqs, r) for r in reqs]}
        self.log.append((self.t, [r.rid for r in reqs]))
        return h

    def poll(self, h):
        return h["status"] if self.t >= h["end"] - 1e-12 else None

    def idle(self, hint):
        self.t += 1e-5 if hint is None else max(hint, 1e-6)


class GpuExecutor:
    """Drives gsr_render_batch on `slots` streams over resident models."""

    def __init__(self, models, slots=2, pair_table=None, safety=1.3, device="cuda", timer=None):
        import torch
        from . import rasterizer as rz
        self.torch, self.rz = torch, rz
        self.models = models                       # list of device model dicts
        self.slots = slots
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free_streams = list(range(slots))
        self.pair_table = dict(pair_table or {})   # (model, W, H) -> pairs of one view
        self.safety = safety
        self.device = device
        self.ws = [None] * slots
        self.status = [None] * slots
        self.timer = timer
        self.n = [int(m["layer"].shape[0]) for m in models]

    def now(self):
        return time.perf_counter()

    def idle(self, hint):
        # hint: seconds until the next arrival (may already be <= 0), None = poll
        time.sleep(max(0.0, min(hint, 2e-3)) if hint is not None else 5e-5)

    def pairs_estimate(self, r):
        est = 0
        for c in r.cams:
            key = (r.model, c["width"], c["height"])
            k = self.pair_table.get(key)
            if k is None:
                k = 4 * self.n[r.model]
            est += int(k * self.safety * (2 ** r.tries)) + 1024
        return est

    def cost(self, r):
        # workspace of the request's share of a batch + its outputs
        pix = r.pixels
        tiles = sum(((c["width"] + 15) // 16) * ((c["height"] + 15) // 16) for c in r.cams)
        recs = self.n[r.model] * len(r.cams)
        return recs * (4 + 4 + 16 + 48) + self.pairs_estimate(r) * 24 + pix * (4 + 4 + 16) + tiles * 8 + 4096

    def calibrate(self, reqs):
        """Measure the pair count of one view per (model, resolution)."""
        for r in reqs:
            for c in r.cams:
                key = (r.model, c["width"], c["height"])
                if key in self.pair_table:
                    continue
                vs = {"layer_mask": 0xFFFFFFFF, "clips": [], "bg": (0.0, 0.0, 0.0)}
                _, _, st = self.rz.rasterize_forward(self.models[r.model], [c], [vs])
                self.pair_table[key] = st.n_pairs

    def launch(self, reqs):
        torch, rz = self.torch, self.rz
        slot = self.free_streams.pop(0)
        s = self.streams[slot]
        cap = sum(self.pairs_estimate(r) for r in reqs)
        reqd = [{"model": r.model, "cams": r.cams, "view": r.view} for r in reqs]
        with torch.cuda.stream(s):
            outs, status, ws = rz.render_batch(self.models, reqd, cap, workspace=self.ws[slot],
                                               status=self.status[slot], stream=s, timer=self.timer)
            ev = torch.cuda.Event()
            ev.record(s)
        self.ws[slot], self.status[slot] = ws, status
        return {"slot": slot, "event": ev, "outs": outs, "status": status, "n": len(reqs), "reqs": reqs}

    def poll(self, h):
        if not h["event"].query():
            return None
        st = h["status"][:h["n"]].cpu().tolist()
        for r, o in zip(h["reqs"], h["outs"]):
            r.result = o
        self.free_streams.append(h["slot"])
        return st
