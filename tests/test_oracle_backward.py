"""Pins of the CPU oracle's gradient: central finite differences in float64,
linearity over views, frozen layers, occlusion and the activity measure."""
import json
import os

import numpy as np
import pytest

from paper_2410_16978_amd import scenes
from tests.helpers import make_scene, to64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(seed=3, W=48, H=40, n_views=1):
    s = scenes.shell_scene(150, 2, 3, seed=seed, log_scale_mu=-3.0, log_scale_sigma=0.3, opacity="normal")
    s64 = to64(s)
    cams = [scenes.orbit_camera([0.3 + 0.4 * v, 0.2, -1.0], W, H) for v in range(n_views)]
    vss = [scenes.view_state(0x3, bg=(0.2, 0.3, 0.1))] * n_views
    rng = np.random.default_rng(seed)
    Gr = rng.standard_normal((n_views, 3, H, W))
    Ga = rng.standard_normal((n_views, H, W))
    return s64, cams, vss, Gr, Ga


def _loss(orc, sc, cams, vss, Gr, Ga):
    r = orc.render(sc, cams, vss, dtype=np.float64)
    return float((r["rgb"] * Gr).sum() + (r["alpha"] * Ga).sum())


def _with_raw(sc):
    """Recompute the activated arrays in float64 from the raw ones."""
    sc["scale"] = np.exp(sc["log_scale"])
    sc["opacity"] = 1.0 / (1.0 + np.exp(-sc["opacity_logit"]))
    return sc


def test_gradient_matches_central_differences(orc):
    """32 parameters: 4 each from mean, log-scale, quaternion, opacity logit and
    the four SH bands; FD on the raw parameters, analytic through the
    activations (d/dlog s = s d/ds, d/dlogit = o(1-o) d/do)."""
    s64, cams, vss, Gr, Ga = _setup(n_views=2)
    s64["log_scale"] = s64["log_scale"].astype(np.float64)
    s64["opacity_logit"] = s64["opacity_logit"].astype(np.float64)
    _with_raw(s64)
    g = orc.backward(s64, cams, vss, Gr, Ga, dtype=np.float64)
    g_logs = g["scale"] * s64["scale"]
    g_logit = g["opacity"] * s64["opacity"] * (1 - s64["opacity"])
    active = np.nonzero(g["max_contrib"] > 0.05)[0]
    assert len(active) > 30
    rng = np.random.default_rng(11)
    bands = {0: [0], 1: [1, 2, 3], 2: [4, 5, 6, 7, 8], 3: list(range(9, 16))}
    groups = [("mean", 3), ("log_scale", 3), ("quat", 4), ("opacity_logit", None)] + [("sh", b) for b in range(4)]
    n_checked = 0
    for name, spec in groups:
        got = 0
        tries = 0
        while got < 4:
            tries += 1
            assert tries < 40, f"could not find smooth samples for {name}"
            i = int(rng.choice(active))
            if name == "opacity_logit":
                idx = (i,)
            elif name == "sh":
                idx = (int(rng.choice(bands[spec])), int(rng.integers(0, 3)), i)
            else:
                idx = (int(rng.integers(0, spec)), i)
            arr = s64[name]
            th = float(arr[idx])
            h = 1e-4 * max(1.0, abs(th))

            def f(val):
                arr[idx] = val
                _with_raw(s64)
                out = _loss(orc, s64, cams, vss, Gr, Ga)
                arr[idx] = th
                _with_raw(s64)
                return out

            fd = (f(th + h) - f(th - h)) / (2 * h)
            fd2 = (f(th + h / 2) - f(th - h / 2)) / h
            if abs(fd - fd2) > 1e-2 * max(abs(fd), 1e-6):
                continue  # crosses a threshold (cutoff, stop, clamp): resample
            an = {"mean": g["mean"], "log_scale": g_logs, "quat": g["quat"], "opacity_logit": g_logit,
                  "sh": g["sh"]}[name][idx]
            assert abs(an - fd) <= 1e-3 * max(abs(fd), 1e-4), (name, idx, an, fd)
            got += 1
            n_checked += 1
    assert n_checked == 32


def test_float_backward_close_to_double(orc):
    s64, cams, vss, Gr, Ga = _setup(seed=4)
    s32 = {k: (v.astype(np.float32) if isinstance(v, np.ndarray) and v.dtype == np.float64 else v)
           for k, v in s64.items()}
    g64 = orc.backward(s64, cams, vss, Gr, Ga, dtype=np.float64)
    g32 = orc.backward(s32, cams, vss, Gr.astype(np.float32), Ga.astype(np.float32), dtype=np.float32)
    for k in ("mean", "scale", "quat", "opacity", "sh"):
        ref = g64[k]
        err = np.abs(g32[k] - ref)
        tol = 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.sqrt(np.mean(ref ** 2)))
        assert np.mean(err <= tol) > 0.995, k


def test_gradient_is_sum_over_views(orc):
    s64, cams, vss, Gr, Ga = _setup(seed=5, n_views=2)
    both = orc.backward(s64, cams, vss, Gr, Ga, dtype=np.float64)
    parts = [orc.backward(s64, [cams[v]], [vss[v]], Gr[v:v + 1], Ga[v:v + 1], dtype=np.float64) for v in range(2)]
    for k in ("mean", "scale", "quat", "opacity", "sh"):
        np.testing.assert_allclose(both[k], parts[0][k] + parts[1][k], rtol=1e-9, atol=1e-12)
    np.testing.assert_array_equal(both["max_contrib"], np.maximum(parts[0]["max_contrib"], parts[1]["max_contrib"]))


def test_frozen_layers_get_no_gradient(orc):
    s64, cams, vss, Gr, Ga = _setup(seed=6)
    full = orc.backward(s64, cams, vss, Gr, Ga, dtype=np.float64)
    part = orc.backward(s64, cams, vss, Gr, Ga, trainable=0b10, dtype=np.float64)
    frozen = s64["layer"] == 0
    for k in ("mean", "scale", "quat", "opacity", "sh"):
        assert np.all(part[k][..., frozen] == 0)
        np.testing.assert_array_equal(part[k][..., ~frozen], full[k][..., ~frozen])
        assert np.any(full[k][..., frozen] != 0)


def test_hidden_gaussians_have_zero_contribution(orc):
    """An opaque front layer stops every pixel before the layer behind it is
    reached: the hidden Gaussians' max contribution and gradient are zero."""
    xs = np.linspace(-0.7, 0.7, 15)
    front = [[x, y, 2.0 + 0.001 * (i * 15 + j)] for i, x in enumerate(xs) for j, y in enumerate(xs)]
    back = [[x, y, 3.0] for x in (-0.1, 0.05, 0.2) for y in (-0.15, 0.0, 0.12)]
    n_f, n_b = len(front), len(back)
    sc = make_scene(front + back, [[0.15, 0.15, 0.01]] * n_f + [[0.05] * 3] * n_b,
                    opacity=[0.99] * n_f + [0.9] * n_b, layer=[1] * n_f + [0] * n_b, sh_degree=1)
    cam = scenes.make_camera(np.eye(3), [0, 0, 0], 64, 64, fx=60, fy=60)
    vs = scenes.view_state()
    r = orc.render(sc, [cam], [vs])
    assert np.all(r["final_T"][0, 18:46, 18:46] < 1e-2)  # the window behind which layer 0 sits
    assert np.all(r["n_tiles"][n_f:] > 0)  # the hidden Gaussians are on screen and listed
    rng = np.random.default_rng(0)
    g = orc.backward(to64(sc), [cam], [vs], rng.standard_normal((1, 3, 64, 64)), rng.standard_normal((1, 64, 64)),
                     dtype=np.float64)
    assert np.all(g["max_contrib"][n_f:] == 0)
    assert np.all(g["mean"][:, n_f:] == 0) and np.all(g["sh"][..., n_f:] == 0)
    assert np.all(g["max_contrib"][:n_f] > 0)


def test_activity_weights_follow_the_paper(orc):
    """activity = 2 |dL/dmean| + 0.1 |dL/dSH| + 0.1 |dL/dlog s| (weights from the
    paper's AvgSample definition)."""
    with open(os.path.join(GOLDEN, "pruning_constants.json")) as f:
        gold = json.load(f)
    wp, wc, ws = gold["weights_position_color_scale"]
    s64, cams, vss, Gr, Ga = _setup(seed=7)
    g = orc.backward(s64, cams, vss, Gr, Ga, dtype=np.float64)
    n = s64["mean"].shape[1]
    want = (wp * np.linalg.norm(g["mean"], axis=0) + wc * np.linalg.norm(g["sh"].reshape(-1, n), axis=0)
            + ws * np.linalg.norm(g["scale"] * s64["scale"], axis=0))
    np.testing.assert_allclose(g["activity"], want, rtol=1e-12, atol=1e-300)
