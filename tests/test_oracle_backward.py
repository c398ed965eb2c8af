"""Pins of the CPU oracle's gradient: central finite differences in float64,
linearity over views, frozen layers, occlusion and the activity measure."""
import json
import os

import numpy as np
import pytest

from paper_2410_16978_amd import scenes
import math

from tests.helpers import Y00, axis_camera, make_scene, to64

KAPPA = 0.3

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


# ---------------------------------------------------------------- closed forms
# Dtypes of the oracle backward: float32 and float64 throughout, the float32
# forward's decisions with the gradient in float64 ("exact"), and the same
# with the forward's own per-pixel values ("exact_fwd_values"); the last two
# take float32 records and SH constants, hence their float32-level tolerance.
DTYPES = [(np.float32, 2e-5), (np.float64, 1e-9), ("exact", 2e-7), ("exact_fwd_values", 2e-7)]


def _scene_for(dtype, sc):
    return to64(sc) if dtype is np.float64 else sc


def _upstream(dtype, Gr, Ga):
    """Upstream gradients at float32 values (every dtype sees the same numbers)."""
    Gr, Ga = Gr.astype(np.float32), Ga.astype(np.float32)
    if dtype is np.float64:
        return Gr.astype(np.float64), Ga.astype(np.float64)
    return Gr, Ga


def _axis_pair():
    """Two isotropic splats on the optical axis, the front one wider (screen
    sigma 2.27 px vs 0.91 px), whose centres project exactly onto the centre
    of pixel (64, 64) (principal point 64.5)."""
    sc = make_scene([[0, 0, 2.0], [0, 0, 3.0]], [[0.04] * 3, [0.02] * 3], opacity=[0.5, 0.8],
                    rgb=[[0.9, 0.2, 0.4], [0.1, 0.7, 0.3]], sh_degree=0)
    return sc, axis_camera(f=110.0), scenes.view_state(bg=(0.2, 0.3, 0.1))


@pytest.mark.parametrize("dtype,rtol", DTYPES)
def test_max_contribution_is_alpha_times_transmittance(orc, dtype, rtol):
    """Front splat: max alpha*T = o1 at the centre pixel (G = 1, T = 1).  Back
    splat: alpha*T = o2 * G2 * (1 - o1 G1); with the front splat wider, G2 is a
    power > 4 of G1, so the product grows with G1 and peaks at the centre
    pixel: o2 (1 - o1).  alpha alone (o2) or T alone (1 - o1) differ."""
    sc, cam, vs = _axis_pair()
    H = W = 128
    Gr, Ga = _upstream(dtype, np.zeros((1, 3, H, W)), np.zeros((1, H, W)))
    g = orc.backward(_scene_for(dtype, sc), [cam], [vs], Gr, Ga, dtype=dtype)
    o1, o2 = (float(np.float32(x)) for x in (0.5, 0.8))
    assert g["max_contrib"][0] == pytest.approx(o1, rel=rtol)
    assert g["max_contrib"][1] == pytest.approx(o2 * (1 - o1), rel=rtol)
    assert abs(g["max_contrib"][1] - o2) > 0.1 and abs(g["max_contrib"][1] - (1 - o1)) > 0.05


@pytest.mark.parametrize("dtype,rtol", DTYPES)
def test_stacked_pair_single_pixel_gradient(orc, dtype, rtol):
    """Upstream gradient on the centre pixel only, where both splats have G = 1
    and alpha = o: C = c1 a1 + c2 a2 (1 - a1) + bg (1 - a1)(1 - a2),
    alpha_out = 1 - (1 - a1)(1 - a2).  Opacity and DC-colour gradients in
    closed form; the offsets are zero, so mean, scale and rotation get none."""
    sc, cam, vs = _axis_pair()
    H = W = 128
    g_rgb, g_a = np.array([0.7, -1.3, 0.4]), -0.6
    Gr = np.zeros((1, 3, H, W))
    Ga = np.zeros((1, H, W))
    Gr[0, :, 64, 64] = g_rgb
    Ga[0, 64, 64] = g_a
    Gr, Ga = _upstream(dtype, Gr, Ga)
    g = orc.backward(_scene_for(dtype, sc), [cam], [vs], Gr, Ga, dtype=dtype)
    rec = orc.render(_scene_for(dtype, sc), [cam], [vs],
                     dtype=np.float64 if dtype is np.float64 else np.float32)["rec"].astype(np.float64)
    c1, c2 = rec[0, 7:10], rec[1, 7:10]
    a1, a2 = (float(np.float32(x)) for x in (0.5, 0.8))
    bg = np.array([float(np.float32(x)) for x in vs["bg"]])
    gr = g_rgb.astype(np.float32).astype(np.float64)
    ga = float(np.float32(g_a))
    want_o1 = float(gr @ (c1 - c2 * a2 - bg * (1 - a2))) + ga * (1 - a2)
    want_o2 = float(gr @ ((1 - a1) * (c2 - bg))) + ga * (1 - a1)
    np.testing.assert_allclose(g["opacity"], [want_o1, want_o2], rtol=rtol)
    np.testing.assert_allclose(g["sh"][0, :, 0], gr * Y00 * a1, rtol=rtol)
    np.testing.assert_allclose(g["sh"][0, :, 1], gr * Y00 * a2 * (1 - a1), rtol=rtol)
    for k in ("mean", "scale", "quat"):
        assert np.all(g[k] == 0), k


@pytest.mark.parametrize("dtype,rtol", DTYPES)
def test_offset_pixel_gradient_closed_form(orc, dtype, rtol):
    """One isotropic splat on the axis (screen variance a = (f s / z)^2 + kappa),
    upstream gradient on the pixel two to the right of its centre only
    (dx = u - x = -2, dy = 0): alpha = o exp(-dx^2 / (2a)) and, with
    D = g . (c - bg) + g_alpha,
      dL/dmu_x = D alpha (-dx / a) f / z,  dL/dmu_z = -D alpha dx^2 f^2 s^2 / (a^2 z^3),
      dL/ds_x = D alpha dx^2 f^2 s / (a^2 z^2),  dL/do = D alpha / o,
    and no gradient for mu_y, s_y, s_z (b = 0, dy = 0)."""
    s, z, f, o = 0.03, 2.5, 110.0, 0.7
    sc = make_scene([[0, 0, z]], [[s] * 3], opacity=o, rgb=[[0.8, 0.3, 0.5]], sh_degree=0)
    cam = axis_camera(f=f)
    vs = scenes.view_state(bg=(0.1, 0.2, 0.3))
    H = W = 128
    g_rgb, g_a = np.array([0.9, -0.4, 1.1]), 0.35
    Gr = np.zeros((1, 3, H, W))
    Ga = np.zeros((1, H, W))
    Gr[0, :, 64, 66] = g_rgb
    Ga[0, 64, 66] = g_a
    Gr, Ga = _upstream(dtype, Gr, Ga)
    g = orc.backward(_scene_for(dtype, sc), [cam], [vs], Gr, Ga, dtype=dtype)
    rec = orc.render(_scene_for(dtype, sc), [cam], [vs],
                     dtype=np.float64 if dtype is np.float64 else np.float32)["rec"].astype(np.float64)
    s, z, o = (float(np.float32(x)) for x in (s, z, o))
    a = (f * s / z) ** 2 + KAPPA
    dx = -2.0
    alpha = o * math.exp(-0.5 * dx * dx / a)
    c = rec[0, 7:10]
    bg = np.array([float(np.float32(x)) for x in vs["bg"]])
    D = float(g_rgb.astype(np.float32).astype(np.float64) @ (c - bg)) + float(np.float32(g_a))
    np.testing.assert_allclose(g["mean"][:, 0], [D * alpha * (-dx / a) * f / z, 0.0,
                                                 -D * alpha * dx * dx * f * f * s * s / (a * a * z ** 3)],
                               rtol=10 * rtol, atol=1e-6 * abs(D))
    np.testing.assert_allclose(g["scale"][:, 0], [D * alpha * dx * dx * f * f * s / (a * a * z * z), 0.0, 0.0],
                               rtol=10 * rtol, atol=1e-6 * abs(D))
    assert g["opacity"][0] == pytest.approx(D * alpha / o, rel=10 * rtol)


def test_exact_gradient_matches_central_differences(orc):
    """The float32 forward's gradient evaluated in float64 ("exact") against
    central differences of the float64 render at the same (float32) parameter
    values, 24 parameters of the smooth kind."""
    s32 = scenes.shell_scene(150, 2, 3, seed=8, log_scale_mu=-3.0, log_scale_sigma=0.3, opacity="normal")
    cams = [scenes.orbit_camera([0.3, 0.2, -1.0], 48, 40)]
    vss = [scenes.view_state(0x3, bg=(0.2, 0.3, 0.1))]
    rng = np.random.default_rng(8)
    Gr = rng.standard_normal((1, 3, 40, 48)).astype(np.float32)
    Ga = rng.standard_normal((1, 40, 48)).astype(np.float32)
    g = orc.backward(s32, cams, vss, Gr, Ga, dtype="exact")
    s64 = to64(s32)
    active = np.nonzero(g["max_contrib"] > 0.05)[0]
    n_checked = 0
    for name, comps in (("mean", 3), ("scale", 3), ("quat", 4), ("opacity", None), ("sh", 16)):
        got = 0
        for i in rng.permutation(active)[:30]:
            if name == "opacity":
                idx = (int(i),)
            elif name == "sh":
                idx = (int(rng.integers(0, comps)), int(rng.integers(0, 3)), int(i))
            else:
                idx = (int(rng.integers(0, comps)), int(i))
            arr = s64[name]
            th = float(arr[idx])
            h = 1e-5 * max(1.0, abs(th))

            def f(val):
                arr[idx] = val
                out = _loss(orc, s64, cams, vss, Gr.astype(np.float64), Ga.astype(np.float64))
                arr[idx] = th
                return out

            fd = (f(th + h) - f(th - h)) / (2 * h)
            fd2 = (f(th + h / 2) - f(th - h / 2)) / h
            if abs(fd - fd2) > 1e-3 * max(abs(fd), 1e-6):
                continue
            assert abs(g[name][idx] - fd) <= 1e-3 * max(abs(fd), 1e-4), (name, idx, g[name][idx], fd)
            got += 1
            if got == 5:
                break
        assert got >= 4, name
        n_checked += got
    assert n_checked >= 20


def test_float32_backward_within_the_plain_bar_of_exact(orc):
    """On test-sized scenes the float32 oracle's gradient is within
    1e-3 max(|g|, 1e-3 RMS) of the exact one on every entry."""
    sc = scenes.shell_scene(300, 3, 3, seed=6, log_scale_mu=-3.2, log_scale_sigma=0.4, opacity="normal")
    cams = [scenes.orbit_camera([0.3 + 0.5 * v, 0.2, -1.0], 72, 56) for v in range(2)]
    vss = [scenes.view_state(0x7, clips=[([0.2, 0.1, 1.0], 0.3, 0b1)], bg=(0.2, 0.3, 0.1))] * 2
    rng = np.random.default_rng(6)
    Gr = rng.standard_normal((2, 3, 56, 72)).astype(np.float32)
    Ga = rng.standard_normal((2, 56, 72)).astype(np.float32)
    ex = orc.backward(sc, cams, vss, Gr, Ga, dtype="exact")
    g32 = orc.backward(sc, cams, vss, Gr, Ga)
    for k in ("mean", "scale", "quat", "opacity", "sh"):
        ref = ex[k]
        tol = 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.sqrt(np.mean(ref ** 2)))
        assert np.all(np.abs(g32[k] - ref) <= tol), k
    np.testing.assert_allclose(g32["max_contrib"], ex["max_contrib"], rtol=1e-5)


def test_condition_of_the_stacked_pair(orc):
    """cond of the two opacity entries of the stacked pair on one pixel: one
    slot (opacity) and one pixel with 2 blended pairs, so
    cond = (2 + 16) * G * [sum_ch |g_ch| (|c_ch| T + |S_ch| / (1 - a)) + |g_a| T_fin / (1 - a)]
    with G = 1, T the transmittance in front, S the colour behind."""
    sc, cam, vs = _axis_pair()
    H = W = 128
    g_rgb, g_a = np.array([0.7, -1.3, 0.4]), -0.6
    Gr = np.zeros((1, 3, H, W), np.float32)
    Ga = np.zeros((1, H, W), np.float32)
    Gr[0, :, 64, 64] = g_rgb
    Ga[0, 64, 64] = g_a
    g = orc.backward(sc, [cam], [vs], Gr, Ga, dtype="exact", cond=True)
    rec = orc.render(sc, [cam], [vs])["rec"].astype(np.float64)
    c1, c2 = rec[0, 7:10], rec[1, 7:10]
    a1, a2 = (float(np.float32(x)) for x in (0.5, 0.8))
    bg = np.array([float(np.float32(x)) for x in vs["bg"]])
    gr = np.abs(g_rgb.astype(np.float32).astype(np.float64))
    ga = abs(float(np.float32(g_a)))
    t_fin = (1 - a1) * (1 - a2)
    s2 = bg * t_fin
    s1 = s2 + c2 * a2 * (1 - a1)
    want1 = 18 * (float(gr @ (np.abs(c1) * 1.0 + np.abs(s1) / (1 - a1))) + ga * t_fin / (1 - a1))
    want2 = 18 * (float(gr @ (np.abs(c2) * (1 - a1) + np.abs(s2) / (1 - a2))) + ga * t_fin / (1 - a2))
    np.testing.assert_allclose(g["cond"]["opacity"], [want1, want2], rtol=1e-12)


def test_condition_bounds_the_entries_and_their_float32_rounding(orc):
    """On a layered scene: cond >= 16 |g| on every entry (a depth-weighted
    magnitude sum bounds the sum), and feeding the gradient the float32
    forward's own per-pixel values moves no entry by more than 2^-24 cond."""
    sc = scenes.shell_scene(300, 3, 3, seed=11, log_scale_mu=-3.2, log_scale_sigma=0.4, opacity="normal")
    cams = [scenes.orbit_camera([0.3 + 0.5 * v, 0.2, -1.0], 72, 56) for v in range(2)]
    vss = [scenes.view_state(0x7, bg=(0.2, 0.3, 0.1))] * 2
    rng = np.random.default_rng(11)
    Gr = rng.standard_normal((2, 3, 56, 72)).astype(np.float32)
    Ga = rng.standard_normal((2, 56, 72)).astype(np.float32)
    ex = orc.backward(sc, cams, vss, Gr, Ga, dtype="exact", cond=True)
    fv = orc.backward(sc, cams, vss, Gr, Ga, dtype="exact_fwd_values")
    for k in ("mean", "scale", "quat", "opacity", "sh"):
        c = ex["cond"][k]
        assert np.all(c >= 16 * np.abs(ex[k]) * (1 - 1e-12)), k
        assert np.all(np.abs(fv[k] - ex[k]) <= 2.0 ** -24 * c), k
        assert np.any(c > 0), k


# ---------------------------------------------------------------- per-layer opacity (fading)
FADE = [0.45, 0.8]


def test_layer_fade_gradient_is_the_premultiplied_scenes(orc):
    """Drawing with opacity o f is drawing the scene whose opacity is o' = o f:
    every gradient but the opacity's is that scene's, and dL/do = f dL/do'."""
    s64, cams, vss, Gr, Ga = _setup(seed=8, n_views=2)
    vf = [scenes.view_state(0x3, bg=(0.2, 0.3, 0.1), layer_opacity=FADE)] * 2
    pre = dict(s64)
    # the factors as the view carries them (float32); o f is then exact in float64
    f = np.asarray(FADE, np.float32).astype(np.float64)[s64["layer"].astype(np.int64)]
    pre["opacity"] = s64["opacity"] * f
    a = orc.backward(s64, cams, vf, Gr, Ga, dtype=np.float64)
    b = orc.backward(pre, cams, vss, Gr, Ga, dtype=np.float64)
    for k in ("mean", "scale", "quat", "sh", "max_contrib"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    np.testing.assert_allclose(a["opacity"], f * b["opacity"], rtol=1e-12, atol=1e-300)
    assert np.any(a["opacity"] != 0)


def test_layer_fade_opacity_gradient_matches_central_differences(orc):
    s64, cams, vss, Gr, Ga = _setup(seed=9, n_views=1)
    vf = [scenes.view_state(0x3, bg=(0.2, 0.3, 0.1), layer_opacity=FADE)]
    s64["opacity"] = s64["opacity"].astype(np.float64)
    g = orc.backward(s64, cams, vf, Gr, Ga, dtype=np.float64)
    active = np.nonzero(g["max_contrib"] > 0.05)[0]
    rng = np.random.default_rng(4)
    checked = 0
    for i in rng.permutation(active):
        arr = s64["opacity"]
        th = float(arr[i])
        h = 1e-5

        def f(val):
            arr[i] = val
            out = _loss(orc, s64, cams, vf, Gr, Ga)
            arr[i] = th
            return out

        fd = (f(th + h) - f(th - h)) / (2 * h)
        fd2 = (f(th + h / 2) - f(th - h / 2)) / h
        if abs(fd - fd2) > 1e-2 * max(abs(fd), 1e-6):
            continue  # crosses a threshold: take another
        assert abs(g["opacity"][i] - fd) <= 1e-3 * max(abs(fd), 1e-4), (i, g["opacity"][i], fd)
        checked += 1
        if checked == 8:
            break
    assert checked == 8
    # both layers were sampled
    assert len(set(s64["layer"][active].tolist())) == 2


# ---------------------------------------------------------------- density-control statistic
def test_densify_statistic_is_the_ndc_gradient_of_the_centre(orc):
    """One Gaussian, two views: the principal point (cx, cy) moves the
    projected centre (u, v) one for one and nothing else that the image
    depends on near the axis, so central differences over cx and cy give
    dL/du and dL/dv per view; the statistic is the sum over the views of
    |(dL/du W/2, dL/dv H/2)| and the count is 2."""
    sc = make_scene([[0.05, -0.03, 0.0]], [[0.08, 0.05, 0.03]], quats=[[0.9, 0.2, -0.3, 0.1]], opacity=[0.7],
                    rgb=[[0.8, 0.3, 0.2]], layer=[1], dtype=np.float64)
    W, H = 40, 32
    cams = [scenes.orbit_camera([0.2, 0.1, -1.0], W, H), scenes.orbit_camera([-0.3, 0.2, -1.0], W, H)]
    vss = [scenes.view_state(bg=(0.1, 0.2, 0.3))] * 2
    rng = np.random.default_rng(2)
    Gr = rng.standard_normal((2, 3, H, W))
    Ga = rng.standard_normal((2, H, W))
    g = orc.backward(sc, cams, vss, Gr, Ga, trainable=0b10, dtype=np.float64)
    want = 0.0
    for v in range(2):
        d = []
        for key in ("cx", "cy"):
            h = 2.0 ** -12  # cameras hold float32: a step that is exact there

            def f(delta):
                cs = [dict(c) for c in cams]
                cs[v][key] = cams[v][key] + delta
                return _loss(orc, sc, cs, vss, Gr, Ga)

            d.append((f(h) - f(-h)) / (2 * h))
        want += np.hypot(d[0] * W / 2, d[1] * H / 2)
    assert g["densify_count"][0] == 2
    assert abs(g["densify_grad"][0] - want) <= 1e-6 * want, (g["densify_grad"][0], want)
    # frozen: nothing accumulated
    g0 = orc.backward(sc, cams, vss, Gr, Ga, trainable=0b01, dtype=np.float64)
    assert g0["densify_grad"][0] == 0 and g0["densify_count"][0] == 0
