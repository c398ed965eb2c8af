"""Host-side tests of the continuous-batching scheduler on a virtual clock
(no GPU): completion, arrival-order admission, the memory budget, overflow
re-runs, percentiles, and batching versus one request per launch."""
import math

import numpy as np

from paper_2410_16978_amd import scenes
from paper_2410_16978_amd.serve import Request, Scheduler, SimExecutor, nearest_rank, requests_from_trace


def _trace(rate=400, dur=0.5, seed=0):
    tr = scenes.poisson_trace(rate, dur, seed=seed, resolutions=((64, 64, 1), (128, 128, 1), (96, 80, 2)))
    return requests_from_trace(tr)


def test_nearest_rank():
    xs = [5, 1, 4, 2, 3]
    assert nearest_rank(xs, 50) == 3
    assert nearest_rank(xs, 99) == 5
    assert nearest_rank(xs, 0) == 1
    assert nearest_rank(list(range(1, 101)), 99) == 99
    assert math.isnan(nearest_rank([], 50))


def test_all_requests_complete_in_order_under_budget():
    reqs = _trace()
    budget = 64 * 128 * 128 * 3  # about three large requests
    in_use = {"now": 0, "max": 0}

    class Ex(SimExecutor):
        def launch(self, batch):
            h = super().launch(batch)
            in_use["now"] += sum(self.cost(r) for r in batch)
            in_use["max"] = max(in_use["max"], in_use["now"])
            h["cost"] = sum(self.cost(r) for r in batch)
            return h

        def poll(self, h):
            st = super().poll(h)
            if st is not None and not h.get("retired"):
                h["retired"] = True
                in_use["now"] -= h["cost"]
            return st

    ex = Ex(slots=2)
    stats = Scheduler(ex, budget, max_batch=8).run(reqs)
    assert all(r.status == 0 for r in reqs)
    assert len(stats.latencies_ms) == len(reqs)
    assert in_use["max"] <= budget and stats.max_bytes_in_flight <= budget
    order = [rid for _, rids in ex.log for rid in rids]
    assert order == sorted(order)  # admitted in arrival order
    assert all(r.admitted >= r.arrival - 1e-12 for r in reqs)


def test_batching_beats_one_request_per_launch():
    reqs_b = _trace(rate=2000, dur=0.2, seed=3)
    reqs_p = _trace(rate=2000, dur=0.2, seed=3)
    kw = dict(slots=2, fixed_s=1e-3, per_pixel_s=1e-9)
    sb = Scheduler(SimExecutor(**kw), 1 << 40, max_batch=32).run(reqs_b)
    sp = Scheduler(SimExecutor(**kw), 1 << 40, batched=False).run(reqs_p)
    assert sp.launches == len(reqs_p)
    assert sb.launches < sp.launches
    assert nearest_rank(sb.latencies_ms, 99) < nearest_rank(sp.latencies_ms, 99)


def test_overflow_reruns_alone():
    reqs = _trace(rate=5000, dur=0.1, seed=5)

    def fail(batch, r):
        # a request that shares its launch overflows the first time
        return -2 if (len(batch) > 1 and r.rid % 3 == 0 and not r.alone) else 0

    ex = SimExecutor(slots=2, fail=fail)
    st = Scheduler(ex, 1 << 40, max_batch=8).run(reqs)
    assert all(r.status == 0 for r in reqs)
    assert st.reruns > 0
    for r in reqs:
        if r.tries:
            assert r.alone


def test_request_larger_than_budget_fails_without_blocking():
    reqs = _trace(rate=200, dur=0.2, seed=7)
    big = Request(rid=10_000, arrival=0.0, model=0, cams=[scenes.front_camera(4096, 4096)], view=scenes.view_state())
    ex = SimExecutor(slots=2)
    Scheduler(ex, 64 * 1024 * 1024, max_batch=8).run([big] + reqs)
    assert big.status == -2
    assert all(r.status == 0 for r in reqs)
