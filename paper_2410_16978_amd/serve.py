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
    batch: int = 0           # requests in the launch that rendered it
    launch_ms: float = math.nan  # host time of that launch call

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
                h = ex.launch(batch)
                t_l = (ex.now() - t0 - tnow) * 1e3
                for r in batch:
                    r.admitted, r.batch, r.launch_ms = tnow, len(batch), t_l
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
    """Drives gsr_render_batch on `slots` streams over resident models.

    ws_bytes: each slot's workspace is allocated once at that size (a
    launch whose batch needs more regrows it; `regrows` counts those), so
    that no device allocation happens while serving; a request's budget cost
    is the workspace of a batch holding it alone (the library's own size
    function) plus its images.  out_pixels: each slot carves its requests'
    images from an arena of that many pixels allocated once (the images of a
    launch stay valid until its slot's next launch; a batch that does not
    fit gets fresh tensors).  keep_results=False drops a request's images
    when its launch completes (a server hands them on).
    Every launch records HIP events around itself on its stream, so that the
    device-busy time (the union of the launches' intervals) can be measured
    (busy_fraction)."""

    def __init__(self, models, slots=2, pair_table=None, safety=1.3, device="cuda", timer=None, ws_bytes=None,
                 keep_results=True, out_pixels=None):
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
        if ws_bytes:
            self.ws = [torch.empty(int(ws_bytes), dtype=torch.uint8, device=device) for _ in range(slots)]
        self.status = [None] * slots
        self.arena = [None] * slots
        if out_pixels:
            self.arena = [torch.empty(4 * int(out_pixels), dtype=torch.float32, device=device) for _ in range(slots)]
        self.mstructs = None
        self._cost = {}
        self.timer = timer
        self.keep_results = keep_results
        self.regrows = 0
        self.intervals = []  # (start event, end event) per launch
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
        # the workspace of a batch holding this request alone, plus its images
        key = (r.model, tuple((c["width"], c["height"]) for c in r.cams), r.tries)
        c = self._cost.get(key)
        if c is None:
            rz = self.rz
            if self.mstructs is None:
                self.mstructs = (rz.Model * len(self.models))(*[rz.model_struct(m) for m in self.models])
            q = rz.Request()
            q.model = int(r.model)
            q.n_views = len(r.cams)
            for e, cam in enumerate(r.cams):
                q.cam[e] = rz.camera_struct(cam)
            q.vs = rz.view_struct(r.view)
            c = rz.batch_workspace_size(self.mstructs, (rz.Request * 1)(q), self.pairs_estimate(r)) + 16 * r.pixels
            self._cost[key] = c
        return c

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
        outputs = None
        arena = self.arena[slot]
        if arena is not None and 4 * sum(r.pixels for r in reqs) <= arena.numel():
            outputs, off = [], 0
            for r in reqs:
                rgbs, alphas = [], []
                for c in r.cams:
                    H, W = c["height"], c["width"]
                    rgbs.append(arena[off:off + 3 * H * W].view(3, H, W))
                    alphas.append(arena[off + 3 * H * W:off + 4 * H * W].view(H, W))
                    off += 4 * H * W
                outputs.append((rgbs, alphas))
        with torch.cuda.stream(s):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev0.record(s)
            outs, status, ws = rz.render_batch(self.models, reqd, cap, workspace=self.ws[slot],
                                               status=self.status[slot], outputs=outputs, stream=s,
                                               timer=self.timer)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        if self.ws[slot] is not None and ws is not self.ws[slot]:
            self.regrows += 1
        self.ws[slot], self.status[slot] = ws, status
        self.intervals.append((ev0, ev))
        return {"slot": slot, "event": ev, "outs": outs, "status": status, "n": len(reqs), "reqs": reqs}

    def poll(self, h):
        if not h["event"].query():
            return None
        st = h["status"][:h["n"]].cpu().tolist()
        if self.keep_results:
            for r, o in zip(h["reqs"], h["outs"]):
                r.result = o
        h["outs"] = None
        self.free_streams.append(h["slot"])
        return st

    def busy_fraction(self):
        """Fraction of the span from the first launch's start to the last
        launch's end during which at least one launch was on the device
        (call after the work has completed); clears the interval log."""
        if not self.intervals:
            return 0.0
        ref = self.intervals[0][0]
        iv = sorted((ref.elapsed_time(a), ref.elapsed_time(b)) for a, b in self.intervals)
        self.intervals = []
        busy, cur_s, cur_e = 0.0, iv[0][0], iv[0][1]
        for a, b in iv[1:]:
            if a > cur_e:
                busy += cur_e - cur_s
                cur_s, cur_e = a, b
            else:
                cur_e = max(cur_e, b)
        busy += cur_e - cur_s
        span = max(b for _, b in iv) - iv[0][0]
        return busy / span if span > 0 else 0.0
