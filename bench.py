#!/usr/bin/env python3
"""Benchmark of the layered Gaussian-splat rasterizer on one MI355X.

Default workload: one training step of 200k Gaussians in 4 nested shell
layers (50k each), SH degree 3, one 800x800 view: forward render, L1 loss on
RGB and alpha against a target rendered from a perturbed copy of the scene
(random background per step, the paper's alpha-channel training), and the
backward to every Gaussian parameter.  All inputs are synthetic and resident
in HBM before timing.  Prints ONE JSON line.

Beside the step throughput it reports the forward render rate (Mpix/s) and
p50/p99 latencies, a live per-stage timing (HIP events recorded by the
library on the stream it launches on), the roofline of the dominant kernel,
a layered stereo render (1M Gaussians, two 1832x1920 eyes) and a serving
trace (two resident models, Poisson requests), each against the plain
one-request-per-launch path, and, on the host, the CPU oracle timed on one
full step of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "render Mpix/s + p50/p99 frame latency; fwd+bwd iters/s; vs plain, 1 GPU"
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector (packed) peak, published
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E, published
STAGES = ("project", "scan", "duplicate", "sort", "ranges", "blend", "blend_bwd", "project_bwd", "bwd_order")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_training_step_200k.json")


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = max(0, min(len(xs) - 1, int(np.ceil(q / 100.0 * len(xs))) - 1))  # nearest rank
    return float(xs[k])


def kernel_source_hash():
    """Hash of the sources the blend kernels are built from (the stored
    traffic figure is the backward blend's)."""
    h = hashlib.sha256()
    for f in ("blend.hip", "cull.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2410_16978_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_work(orc_fwd, scene, n_pix):
    """Per-launch algorithmic flops/bytes of each stage from the oracle's
    exact counts on the same scene: K pairs, E evaluated (pixel, pair) tests,
    A blended pairs, Eb tests of the backward (per pixel, its tile's pairs up
    to its last blended one); flops count an FMA as 2 and exp as 1."""
    K, E, A = orc_fwd["counts"]["K"], orc_fwd["counts"]["E"], orc_fwd["counts"]["A"]
    last = orc_fwd["last"].reshape(-1).astype(np.int64)
    ranges = orc_fwd["ranges"]
    # evaluated pairs of the backward: per pixel, the tile's pairs up to its last blended one
    H, W = orc_fwd["last"].shape[-2:]
    tx = (W + 15) // 16
    ys, xs = np.divmod(np.arange(H * W), W)
    tile = (ys // 16) * tx + xs // 16
    start = ranges[tile, 0].astype(np.int64)
    Eb = int(np.where(last > 0, last - start, 0).sum())
    n = scene["mean"].shape[1]
    nv = int((orc_fwd["n_tiles"] > 0).sum())
    D = scene["sh_degree"]
    nc = (D + 1) ** 2
    tiles = orc_fwd["counts"]["tiles"]
    return {
        "K": K, "E": E, "A": A, "Eb": Eb, "visible": nv,
        "blend": {"flops": 14 * E + 9 * A},
        "blend_bwd": {"flops": 14 * Eb + 50 * A},
        # bytes: all Gaussians read mean/opacity/layer/quat/scale (+ SH when visible), records written
        "project": {"bytes": n * (12 + 4 + 1 + 16 + 12 + 4) + nv * (12 * nc + 48 + 16)},
        # one-pass tile grouping (at most 4096 tiles: counts, keys and values in
        # and out, 4 B block counts per (block of 4096 pairs, tile) written, read
        # twice, written once) + per-tile depth sort (8 + 4 B in, 4 B record id, 8 B out)
        "sort": {"bytes": (8 + 24 + 24) * K + 16 * 4096 * ((K + 4095) // 4096)},
        "duplicate": {"bytes": nv * 24 + 12 * K},
        "ranges": {"bytes": 8 * K + 8 * tiles},
        "scan": {"bytes": 8 * n},
        "project_bwd": {"bytes": nv * (36 + 48 + 12 * nc + 40 + 4 * (10 + 3 * nc)) + 4 * n * (11 + 3 * nc)},
        "pixels": n_pix,
    }


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(workload, threads, min_seconds, max_steps=200):
    """The oracle (as it stands) on full steps (forward + backward) of the
    same workload, repeated until min_seconds have passed: the forward of
    the first step, the step count and the forward and backward seconds."""
    import oracle
    sc, cams, views = workload.scene, workload.cams, workload.views
    H, W = cams[0]["height"], cams[0]["width"]
    rng = np.random.default_rng(7)
    Gr = (rng.standard_normal((1, 3, H, W)) * 1e-6).astype(np.float32)
    Ga = (rng.standard_normal((1, H, W)) * 1e-6).astype(np.float32)
    first, steps, t_f, t_b = None, 0, 0.0, 0.0
    while steps < max_steps and (steps == 0 or t_f + t_b < min_seconds):
        t0 = time.perf_counter()
        fwd = oracle.render(sc, cams, views, pairs=False, n_threads=threads)
        t1 = time.perf_counter()
        oracle.backward(sc, cams, views, Gr, Ga, n_threads=threads)
        t2 = time.perf_counter()
        first = fwd if first is None else first
        steps, t_f, t_b = steps + 1, t_f + (t1 - t0), t_b + (t2 - t1)
    return first, steps, t_f, t_b


def bench_compressed(rz, torch, scene, cams, vstates, st, out, frames, warmup):
    """The same batched stereo frames from compressed attributes (Sec. 4.3):
    16-bit parameters with packed SH triplets, and with a 16k-entry K-means
    SH codebook; frame time, projection time and device bytes per Gaussian
    against the float model (the codebook is built on the host first; its
    time is reported, not timed with the frames)."""
    from paper_2410_16978_amd import compress
    res = {"float32_bytes_per_gaussian": 4 * (3 + 3 + 4 + 1 + 3 * (int(scene["sh_degree"]) + 1) ** 2) + 1}
    for name, mode in (("half_packed", "packed"), ("half_codebook", "codebook")):
        t0 = time.perf_counter()
        comp = compress.compress(scene, mode, codebook_size=16384, iters=4, sample=65536)
        enc = time.perf_counter() - t0
        model = rz.to_device_compressed(comp)
        tm = rz.Timer()
        for i in range(3):
            rz.rasterize_forward(model, cams, [vstates[i]] * 2, state=st, sync=False, out=out, timer=tm)
        stage = {k: round(v[0] / 3, 4) for k, v in tm.read().items() if v[1]}
        tm.close()
        for i in range(warmup):
            rz.rasterize_forward(model, cams, [vstates[i]] * 2, state=st, sync=False, out=out)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(frames):
            rz.rasterize_forward(model, cams, [vstates[warmup + i]] * 2, state=st, sync=False, out=out)
        ev[1].record()
        torch.cuda.synchronize()
        rz.forward_check(st)
        mean = ev[0].elapsed_time(ev[1]) / frames
        W, H = cams[0]["width"], cams[0]["height"]
        res[name] = {"mpix_s": round(2 * W * H / (mean * 1e-3) / 1e6, 1), "ms_per_frame": round(mean, 4),
                     "project_ms": stage.get("project"), "bytes_per_gaussian": round(compress.nbytes_per_gaussian(comp), 2),
                     "encode_s": round(enc, 2)}
        if mode == "codebook":
            res[name]["codebook_bytes"] = int(comp["codebook"].nbytes)
        del model
    return res


def bench_stereo(rz, scenes, torch, frames, warmup):
    """Layered stereo frames: 1M Gaussians in 5 CT-like shells, SH3, two eyes
    of 1832x1920, a random 5-bit layer mask and 1-3 clip planes per frame.
    Both eyes in one launch chain vs the plain path (one launch chain per
    eye).  Inputs resident in HBM; frame latency from HIP events."""
    wl = scenes.layered_stereo()
    model = rz.to_device(wl.scene)
    cams = wl.cams
    W, H = cams[0]["width"], cams[0]["height"]
    rng = np.random.default_rng(1)
    vstates = [scenes.random_view_state(rng, 5) for _ in range(frames + warmup)]
    full = scenes.view_state(0x1F)
    # pair buffers sized for every layer drawn (masks and clips only remove pairs)
    _, _, st2 = rz.rasterize_forward(model, cams, [full, full])
    _, _, st1 = rz.rasterize_forward(model, cams[:1], [full])
    _, _, st1b = rz.rasterize_forward(model, cams[1:], [full])
    n = int(model["layer"].shape[0])
    cap2 = int(st2.n_pairs * 1.02) + 4096
    st2 = rz.make_state(n, 2, W, H, cap2)
    st2s = rz.make_state(n, 2, W, H, cap2, shared=True)
    st1 = rz.make_state(n, 1, W, H, int(max(st1.n_pairs, st1b.n_pairs) * 1.02) + 4096)
    out2 = (torch.empty((2, 3, H, W), device="cuda"), torch.empty((2, H, W), device="cuda"))
    out2s = (torch.empty((2, 3, H, W), device="cuda"), torch.empty((2, H, W), device="cuda"))
    outs = [(torch.empty((1, 3, H, W), device="cuda"), torch.empty((1, H, W), device="cuda")) for _ in range(2)]
    centre = scenes.centre_camera(cams[0], cams[1])

    def batched(vs):
        rz.rasterize_forward(model, cams, [vs, vs], state=st2, sync=False, out=out2)

    def shared(vs):
        vs_s = scenes.with_sort_cam(vs, centre)
        rz.rasterize_forward(model, cams, [vs_s, vs_s], state=st2s, sync=False, out=out2s)

    def plain(vs):
        for e in range(2):
            rz.rasterize_forward(model, cams[e:e + 1], [vs], state=st1, sync=False, out=outs[e])

    # one frame both ways: the shared order's image error against per-eye sorting
    batched(vstates[0])
    shared(vstates[0])
    torch.cuda.synchronize()
    diff = float((out2s[0] - out2[0]).abs().max().item())
    stages = {}
    for name, fn in (("batched", batched), ("shared_order", shared)):
        tm = rz.Timer()
        st = st2 if name == "batched" else st2s
        for i in range(3):
            rz.rasterize_forward(model, cams, [vstates[i]] * 2 if name == "batched" else
                                 [scenes.with_sort_cam(vstates[i], centre)] * 2, state=st, sync=False,
                                 out=out2 if name == "batched" else out2s, timer=tm)
        stages[name] = {k: round(v[0] / 3, 4) for k, v in tm.read().items() if v[1]}
        tm.close()

    res = {}
    for name, fn in (("batched", batched), ("shared_order", shared), ("plain", plain)):
        for i in range(warmup):
            fn(vstates[i])
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(frames + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(frames):
            fn(vstates[warmup + i])
            ev[i + 1].record()
        torch.cuda.synchronize()
        ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(frames)]
        mean = ev[0].elapsed_time(ev[-1]) / frames
        res[name] = {"mpix_s": round(2 * W * H / (mean * 1e-3) / 1e6, 1), "ms_per_frame": round(mean, 4),
                     "p50_ms": round(percentile(ms, 50), 4), "p99_ms": round(percentile(ms, 99), 4)}
    rz.forward_check(st2)
    rz.forward_check(st2s)
    rz.forward_check(st1)
    comp_res = bench_compressed(rz, torch, wl.scene, cams, vstates, st2, out2, frames, warmup)
    return {"workload": wl.name, "frames": frames, "pairs": st2.capacity, **res, "compressed": comp_res,
            "speedup_vs_plain": round(res["plain"]["ms_per_frame"] / res["batched"]["ms_per_frame"], 3),
            "shared_order_speedup_vs_plain": round(res["plain"]["ms_per_frame"] / res["shared_order"]["ms_per_frame"],
                                                   3),
            "shared_order_image_max_abs_vs_per_eye": diff, "stage_ms_per_frame": stages}


def bench_plain_forward(rz, scenes, torch, frames=1000, warmup=50):
    """Plain forward render: 4096 Gaussians (uniform in [-1, 1]^3, SH0), one
    128x128 view, one launch chain per frame; per-frame latency from HIP
    events over `frames` frames (p50 / p99), Mpix/s, and the launch chain
    broken down by stage (library-recorded events)."""
    wl = scenes.plain_forward_4k()
    model = rz.to_device(wl.scene)
    cams, views = wl.cams, wl.views
    W, H = cams[0]["width"], cams[0]["height"]
    _, _, st = rz.rasterize_forward(model, cams, views)
    st = rz.make_state(wl.scene["mean"].shape[1], 1, W, H, int(st.n_pairs * 1.05) + 1024)
    out = (torch.empty((1, 3, H, W), device="cuda"), torch.empty((1, H, W), device="cuda"))
    for _ in range(warmup):
        rz.rasterize_forward(model, cams, views, state=st, sync=False, out=out)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(frames + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(frames):
        rz.rasterize_forward(model, cams, views, state=st, sync=False, out=out)
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(frames)]
    mean = ev[0].elapsed_time(ev[-1]) / frames
    tm = rz.Timer()
    for _ in range(100):
        rz.rasterize_forward(model, cams, views, state=st, sync=False, out=out, timer=tm)
    stages = {k: round(v[0] / 100 * 1e3, 2) for k, v in tm.read().items() if v[1]}
    tm.close()
    rz.forward_check(st)
    return {"workload": wl.name, "frames": frames, "mpix_s": round(W * H / (mean * 1e-3) / 1e6, 2),
            "ms_per_frame": round(mean, 4), "p50_ms": round(percentile(ms, 50), 4),
            "p99_ms": round(percentile(ms, 99), 4), "pairs": st.n_pairs if st.n_pairs else None,
            "stage_us_per_frame": stages}


def bench_serving(rz, scenes, torch, seconds, rates=(200.0,), budgets=(16 << 30,), saturation=True):
    """Serving: resident models of 500k and 2M Gaussians (5 layers, SH3);
    open-loop Poisson requests (resolution 512^2, 1024^2 or stereo
    1832x1920, random layer mask and clip planes).  Continuous batching
    (arrival-order admission into batched launches on two streams) vs the
    plain path (one request per launch, one stream) on the same trace, per
    HBM budget and arrival rate; optionally the same requests all at once
    (saturation throughput).  Each slot's workspace is allocated once at
    the budget and frames are dropped on completion (no device allocation
    while serving: each slot's images are carved from an arena allocated
    once); the cyclic garbage collector is paused during the timed runs (as
    a latency-critical server would run it); the device-busy fraction is the
    union of the launches' device intervals over their span; the five
    slowest requests are listed with their admission delay, batch size and
    launch host time."""
    import gc
    from paper_2410_16978_amd.serve import GpuExecutor, Scheduler, requests_from_trace
    models = [rz.to_device(m) for m in scenes.serving_models()]
    ex0 = GpuExecutor(models, slots=2)
    for rate in rates:
        ex0.calibrate(requests_from_trace(scenes.poisson_trace(rate, seconds, seed=0)))
    table = ex0.pair_table
    del ex0
    res = {"models": [500_000, 2_000_000], "trace_s": seconds, "runs": []}
    plans = [("open_loop", budget, rate) for budget in budgets for rate in rates]
    if saturation:
        plans.append(("saturation", budgets[-1], rates[0]))
    for mode, budget, rate in plans:
        trace = scenes.poisson_trace(rate, seconds, seed=0)
        entry = {"mode": mode, "budget_gib": budget / (1 << 30), "rate_hz": rate, "requests": len(trace)}
        max_pix = max(sum(c["width"] * c["height"] for c in t["cams"]) for t in trace)
        for name, batched in (("batched", True), ("plain", False)):
            # a batch's workspace can exceed the sum of its requests' costs a
            # little (per-call sort words): the slots get a quarter more
            ex = GpuExecutor(models, slots=2 if batched else 1, pair_table=table, ws_bytes=budget * 5 // 4,
                             keep_results=False, out_pixels=(16 if batched else 1) * max_pix)
            warm = requests_from_trace(trace[:400])
            if mode == "saturation":
                for r in warm:
                    r.arrival = 0.0
            Scheduler(ex, budget, max_batch=16, batched=batched).run(warm)
            torch.cuda.synchronize()
            ex.busy_fraction()
            reqs = requests_from_trace(trace)
            if mode == "saturation":
                for r in reqs:
                    r.arrival = 0.0
            regrows0 = ex.regrows
            gc.collect()
            gc.disable()
            try:
                stats = Scheduler(ex, budget, max_batch=16, batched=batched).run(reqs)
                torch.cuda.synchronize()
            finally:
                gc.enable()
            sm = stats.summary()
            out = {k: sm[k] for k in ("p50_ms", "p99_ms", "frames_per_s", "mpix_per_s", "launches", "reruns")}
            out["device_busy"] = round(ex.busy_fraction(), 3)
            out["workspace_regrows"] = ex.regrows - regrows0
            slow = sorted((r for r in reqs if r.status == 0), key=lambda r: r.arrival - r.done)[:5]
            out["slowest"] = [{"latency_ms": round((r.done - r.arrival) * 1e3, 2),
                               "admit_delay_ms": round((r.admitted - r.arrival) * 1e3, 2), "batch": r.batch,
                               "launch_host_ms": round(r.launch_ms, 2), "pixels": r.pixels} for r in slow]
            if any(r.status != 0 for r in reqs):
                out["failed"] = sum(r.status != 0 for r in reqs)
            entry[name] = out
            print(f"serving {mode} budget {budget >> 30} GiB rate {rate:g}/s {name}: p50 {out['p50_ms']} ms, "
                  f"p99 {out['p99_ms']} ms, busy {out['device_busy']}", file=sys.stderr, flush=True)
            del ex
        res["runs"].append(entry)
    return res


def bench_layered_training(args, torch, rz, ag, scenes):
    """Layered training at scale: 4M Gaussians in 8 shells (SH3), 8 views of
    1024^2 per fwd+bwd launch drawn from a pool of 64, layer 7 trainable and
    layers 0-6 frozen (Sec. 3.2), Adam, inactive pruning every 100 steps
    (Sec. 3.2.2) - iters/s and the pruned fraction per criterion; and the
    plain path (8 sequential single-view launches per step) for the same
    steps."""
    from paper_2410_16978_amd.train import FusedAdam, LayeredTrainer, PruneConfig
    wl = scenes.layered_training_4m()
    pool = wl.extra["pool"]
    tgt = rz.to_device(wl.extra["target_scene"])
    W, H = pool[0]["width"], pool[0]["height"]
    t_rgb = torch.empty((len(pool), 3, H, W), device="cuda")
    t_alpha = torch.empty((len(pool), H, W), device="cuda")
    for i in range(0, len(pool), 8):
        r, a, _ = rz.rasterize_forward(tgt, pool[i:i + 8], [scenes.view_state(bg=(0, 0, 0))] * len(pool[i:i + 8]))
        t_rgb[i:i + 8], t_alpha[i:i + 8] = r, a
    del tgt
    trainable = wl.extra["trainable_layers"]
    # inactive pruning: the window's average activity against T (T0 = 0.015, decay 0.975) under the chosen
    # reading of the norms, plus the max-contribution criterion
    tr = LayeredTrainer(wl.scene, pool, (t_rgb, t_alpha), trainable_layers=trainable, views_per_step=8,
                        prune=PruneConfig(interval=100, measure=args.activity_measure,
                                          threshold=args.prune_threshold), seed=0)
    n0 = tr.n
    n_trainable0 = int(((trainable >> tr.layer.to(torch.int64)) & 1).sum())
    for _ in range(args.warmup):  # sizes the pair buffers (synchronising forwards)
        tr.step()
    cap = tr.rctx.state.capacity
    tr.rctx.state = rz.make_state(tr.n, 8, W, H, int(cap * 1.3) + 4096)
    tr.rctx.sync = False
    steps = args.train_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prunes = []
    for _ in range(steps):
        out = tr.step()
        if "prune" in out:
            prunes.append(out["prune"])
            tr.rctx.state = rz.make_state(tr.n, 8, W, H, int(cap * 1.3) + 4096)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rz.forward_check(tr.rctx.state)
    # plain: the same training, one view per launch (8 launches per step)
    plain_steps = max(5, min(steps // 10, 20))
    params = {k: v.detach().clone().requires_grad_(True) for k, v in tr.params.items()}
    opt = FusedAdam(params, tr.lrs)
    ctxs = [ag.RenderContext(trainable_layers=trainable) for _ in range(8)]
    rng = np.random.default_rng(1)
    for it in range(plain_steps + 2):
        if it == 2:
            torch.cuda.synchronize()
            tp = time.perf_counter()
        idx = rng.choice(len(pool), 8, replace=False)
        bg = tuple(float(x) for x in rng.uniform(0, 1, 3))
        for p in params.values():
            p.grad = None
        for v, i in enumerate(idx):
            rgb, alpha = ag.render_params(params, tr.layer, tr.sh_degree, [pool[i]], [scenes.view_state(bg=bg)],
                                          ctxs[v])
            (ag.l1_alpha_loss(rgb, alpha, t_rgb[i:i + 1], t_alpha[i:i + 1], [bg]) / 8.0).backward()
        opt.step(params, tr.layer, tr.sh_degree, trainable)
    torch.cuda.synchronize()
    dt_plain = (time.perf_counter() - tp) / plain_steps
    pr = {"activity": [p["activity"] for p in prunes], "max_contrib": [p["max_contrib"] for p in prunes],
          "both": [p["both"] for p in prunes], "pruned": sum(p["pruned"] for p in prunes),
          "thresholds": [round(p["threshold"], 6) for p in prunes],
          "avg_activity_p10_p50_p90_p99_max": [[float("%.4g" % x) for x in p.get("avg_quantiles", [])]
                                               for p in prunes]}
    return {"metric": "layered training iters/s (8 views of 1024^2 per step), 1 GPU", "value": round(steps / dt, 3),
            "unit": "iters/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
            "ms_per_step": round(dt / steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "gaussians": n0, "layers": 8, "sh_degree": 3, "views_per_step": 8,
                       "width": W, "height": H, "trainable_layers": trainable, "prune_interval": 100,
                       "activity_measure": args.activity_measure, "prune_threshold_T0": args.prune_threshold,
                       "step": "forward + L1(rgb, alpha) + backward + Adam, random background"},
            "plain_ms_per_step": round(dt_plain * 1e3, 3),
            "speedup_vs_plain": round(dt_plain / (dt / steps), 3),
            "prunes": len(prunes), "pruned": pr,
            "pruned_fraction_of_trainable": round(pr["pruned"] / max(n_trainable0, 1), 4),
            "gaussians_after": tr.n}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing (profiling runs)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0: all host cores, at most 16)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle steps are repeated until this much time has passed (at most 200 steps)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the layered-stereo and serving measurements (profiling runs)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="length of the serving trace")
    ap.add_argument("--workload", default="training_step_200k",
                    choices=["training_step_200k", "layered_training_4m", "layered_stereo_1m", "serving_c4"],
                    help="training_step_200k (default): the 200k/800x800 step; layered_training_4m: 4M Gaussians, "
                         "8 views of 1024^2 per step, pruning every 100 steps; layered_stereo_1m: only the layered "
                         "stereo frames (1M Gaussians, 2 x 1832x1920; profiling runs); serving_c4: the serving "
                         "trace of --serve-seconds (30 by default here) at 200 and 800 requests/s under 2 GiB and "
                         "16 GiB budgets")
    ap.add_argument("--train-steps", type=int, default=200, help="steps of the layered_training_4m workload")
    ap.add_argument("--activity-measure", default="update", choices=["update", "gradient"],
                    help="reading of the inactive-pruning norms (layered_training_4m)")
    ap.add_argument("--prune-threshold", type=float, default=1.5e-4,
                    help="inactive-pruning T0 of the layered_training_4m workload (the paper's 0.015 was tuned on its "
                         "data; under the update reading every trainable Gaussian of this scene averages below it)")
    ap.add_argument("--extra-train-steps", type=int, default=100,
                    help="steps of the layered_training_4m entry of the default run (0: left out)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_16978_amd import autograd as ag
    from paper_2410_16978_amd import rasterizer as rz
    from paper_2410_16978_amd import scenes

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = "cuda"
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)
        return
    if args.workload == "layered_training_4m":
        print(json.dumps(bench_layered_training(args, torch, rz, ag, scenes)), flush=True)
        return
    if args.workload == "layered_stereo_1m":
        print(json.dumps(bench_stereo(rz, scenes, torch, frames=args.steps, warmup=args.warmup)), flush=True)
        return
    if args.workload == "serving_c4":
        secs = args.serve_seconds if "--serve-seconds" in sys.argv else 30.0
        print(json.dumps(bench_serving(rz, scenes, torch, secs, rates=(200.0, 800.0), budgets=(2 << 30, 16 << 30),
                                       saturation=False)), flush=True)
        return
    wl = scenes.training_step_200k(seed=0)
    sc = wl.scene
    cam = wl.cams[0]
    H, W = cam["height"], cam["width"]
    n = sc["mean"].shape[1]
    D = sc["sh_degree"]

    # ---------------- inputs resident in HBM
    params = {k: torch.tensor(sc[k], device=dev, requires_grad=True)
              for k in ("mean", "log_scale", "quat", "opacity_logit", "sh")}
    layer = torch.tensor(sc["layer"], device=dev)
    target_model = rz.to_device(wl.extra["target_scene"])
    t_rgb, t_alpha, _ = rz.rasterize_forward(target_model, wl.cams, [scenes.view_state(0xF, bg=(0, 0, 0))])
    bg_rng = np.random.default_rng(123)
    bgs = [tuple(float(x) for x in bg_rng.uniform(0, 1, 3)) for _ in range(args.steps + args.warmup + 1)]
    views_per_step = [[scenes.view_state(0xF, bg=b)] for b in bgs]

    # The step on the library's entry points: forward on the raw parameters,
    # the fused L1 loss with its gradient, backward into preallocated
    # gradients (what the autograd wrapper does, without its Python work).
    model = {"mean": params["mean"].detach(), "scale": params["log_scale"].detach(),
             "quat": params["quat"].detach(), "opacity": params["opacity_logit"].detach(),
             "sh": params["sh"].detach(), "layer": layer, "sh_degree": D, "raw": True}
    out = (torch.empty((1, 3, H, W), device=dev), torch.empty((1, H, W), device=dev))
    grads = {"mean": torch.empty((3, n), device=dev), "scale": torch.empty((3, n), device=dev),
             "quat": torch.empty((4, n), device=dev), "opacity": torch.empty((n,), device=dev),
             "sh": torch.empty_like(params["sh"])}
    # first call sizes the pair buffers (one synchronising call), then no host syncs
    _, _, st0 = rz.rasterize_forward(model, wl.cams, views_per_step[0])
    torch.cuda.synchronize()
    K0 = st0.n_pairs
    state = rz.make_state(n, 1, W, H, int(K0 * 1.25) + 4096, dev)
    del st0
    timer = None

    def step(i):
        vs = views_per_step[i]
        rgb, alpha, st = rz.rasterize_forward(model, wl.cams, vs, state=state, sync=False, out=out, timer=timer)
        loss, g_rgb, g_a = rz.l1_alpha_loss(rgb, alpha, t_rgb, t_alpha, [bgs[i]], loss=True, grads=True)
        rz.rasterize_backward(model, wl.cams, vs, st, g_rgb, g_a, grads=grads, timer=timer)
        return loss

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    # ---------------- timed: K training steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        step(args.warmup + i)
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rz.forward_check(state)  # pair capacity held for every step
    step_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.steps

    # ---------------- the same step through the autograd wrapper (Python-side cost)
    rctx = ag.RenderContext(sync=False)
    rctx.state = state
    one = torch.ones((), device=dev)

    def step_autograd(i):
        vs = views_per_step[i]
        rgb, alpha = ag.render_params(params, layer, D, wl.cams, vs, rctx)
        loss = ag.l1_alpha_loss(rgb, alpha, t_rgb, t_alpha, [bgs[i]])
        loss.backward(one)
        for p in params.values():
            p.grad = None
        return loss

    for i in range(args.warmup):
        step_autograd(i)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    aev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    aev[0].record()
    for i in range(args.steps):
        step_autograd(args.warmup + i)
    aev[1].record()
    torch.cuda.synchronize()
    autograd_ms = aev[0].elapsed_time(aev[1]) / args.steps
    autograd_wall_ms = (time.perf_counter() - ta) * 1e3 / args.steps

    # ---------------- forward-only render rate (same scene, no autograd)
    with torch.no_grad():
        model = {"mean": params["mean"].detach(), "scale": torch.exp(params["log_scale"]).detach(),
                 "quat": params["quat"].detach(), "opacity": torch.sigmoid(params["opacity_logit"]).detach(),
                 "sh": params["sh"].detach(), "layer": layer, "sh_degree": D}
        fst = rz.make_state(n, 1, W, H, rctx.state.capacity, dev)
        out = (torch.empty((1, 3, H, W), device=dev), torch.empty((1, H, W), device=dev))
        for i in range(args.warmup):
            rz.rasterize_forward(model, wl.cams, views_per_step[i], state=fst, sync=False, out=out)
        fevs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        fevs[0].record()
        for i in range(args.steps):
            rz.rasterize_forward(model, wl.cams, views_per_step[i], state=fst, sync=False, out=out)
            fevs[i + 1].record()
        torch.cuda.synchronize()
        fwd_ms = [fevs[i].elapsed_time(fevs[i + 1]) for i in range(args.steps)]
        fwd_mean = fevs[0].elapsed_time(fevs[-1]) / args.steps

    # ---------------- per-stage timing over K steps (library-recorded HIP events)
    timer = rz.Timer()
    timer.read()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    stages = timer.read()
    timer = None
    # per step: a stage may be timed in several pieces per call (the sort is split by the ranges)
    stage_ms = {s: ms / args.steps for s, (ms, c) in stages.items()}

    result = {
        "metric": METRIC,
        "value": round(1000.0 / ms_per_step, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "gaussians": n, "layers": 4, "sh_degree": D, "width": W, "height": H,
                   "views_per_step": 1, "step": "forward + L1(rgb, alpha) + backward, random background"},
        "p50_ms": round(percentile(step_ms, 50), 4),
        "p99_ms": round(percentile(step_ms, 99), 4),
        "render_mpix_s": round(W * H / (fwd_mean * 1e-3) / 1e6, 2),
        "render_p50_ms": round(percentile(fwd_ms, 50), 4),
        "render_p99_ms": round(percentile(fwd_ms, 99), 4),
        "wall_s": round(wall, 3),
        "autograd_step": {"ms_per_step": round(autograd_ms, 4), "host_ms_per_step": round(autograd_wall_ms, 4)},
        "pairs": K0,
        "stage_ms": {s: round(v, 4) for s, v in stage_ms.items()},
    }

    # ---------------- layered stereo render and serving, each vs the plain path
    if not args.no_extra:
        result["plain_forward_4k_128px"] = bench_plain_forward(rz, scenes, torch)
        result["stereo_render"] = bench_stereo(rz, scenes, torch, frames=max(10, min(args.steps, 50)),
                                               warmup=max(2, min(args.warmup, 5)))
        result["serving"] = bench_serving(rz, scenes, torch, args.serve_seconds, rates=(200.0, 800.0))
        if args.extra_train_steps > 0:
            sub = argparse.Namespace(warmup=3, train_steps=args.extra_train_steps, activity_measure=args.activity_measure,
                                     prune_threshold=args.prune_threshold)
            lt = bench_layered_training(sub, torch, rz, ag, scenes)
            result["layered_training_4m"] = {k: lt[k] for k in (
                "value", "unit", "steps", "ms_per_step", "plain_ms_per_step", "speedup_vs_plain", "prunes",
                "pruned", "pruned_fraction_of_trainable", "gaussians_after")}
            result["layered_training_4m"]["workload"] = lt["config"]["workload"]

    # ---------------- CPU oracle on one step of the same workload
    threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
    orc_fwd = None
    if not args.no_cpu_baseline:
        orc_fwd, n_cpu, t_f, t_b = run_cpu_baseline(wl, threads, args.cpu_seconds)
        _, n1, t1f, t1b = run_cpu_baseline(wl, 1, 0.0, max_steps=1)
        result["cpu_baseline"] = {"value": round(n_cpu / (t_f + t_b), 4), "unit": "iters/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": "%d full steps (forward + backward) of the same 200k/800x800 "
                                            "workload in %.1f s; forward %.2f s, backward %.2f s per step"
                                            % (n_cpu, t_f + t_b, t_f / n_cpu, t_b / n_cpu),
                                  "single_thread": {"value": round(n1 / (t1f + t1b), 4), "cores": 1,
                                                    "sample": "1 full step: forward %.2f s, backward %.2f s"
                                                              % (t1f, t1b)},
                                  "cpu_model": cpu_model()}
    else:
        import oracle
        orc_fwd = oracle.render(wl.scene, wl.cams, wl.views, n_threads=threads)

    # ---------------- roofline of the dominant kernel
    work = algorithmic_work(orc_fwd, sc, W * H)
    dom = max(stage_ms, key=lambda s: stage_ms[s])
    sec = stage_ms[dom] * 1e-3
    if "flops" in work.get(dom, {}):
        ach = work[dom]["flops"] / sec / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4)}
    else:
        ach = work[dom]["bytes"] / sec / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4)}
    roof["traffic"] = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel") == dom and tr.get("source_hash") == kernel_source_hash():
            roof["traffic"] = tr.get("bytes_per_launch")
    roof["launch_ms"] = round(stage_ms[dom], 4)
    result["roofline"] = roof
    result["algorithmic"] = {k: v for k, v in work.items() if k in ("K", "E", "A", "Eb", "visible")}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
