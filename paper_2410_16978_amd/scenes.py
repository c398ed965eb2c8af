"""Seeded synthetic inputs for the layered splat rasterizer.

This module draws scenes, cameras, per-view layer/clip state and request
traces with numpy's PCG64 generator.  It holds none of the rasterizer's
arithmetic (no projection, colour evaluation, sorting or blending); both the
GPU path and the CPU oracle consume the arrays it returns.

Array layout (structure of arrays, float32 unless noted):
  mean    [3, n]          world-space centres
  scale   [3, n]          activated scales, exp(log_scale)
  quat    [4, n]          rotation quaternion (w, x, y, z), unit length
  opacity [n]             activated opacity, sigmoid(logit)
  sh      [(D+1)^2, 3, n] spherical-harmonic coefficients, coefficient-major
  layer   [n] uint8       layer id (0 = innermost)
Raw parameters (log_scale, opacity_logit) are kept beside the activated ones
for training.

The layered anatomy of the paper (bone, then muscle, then soft tissue,
trained as consecutive layers; Sec. 3.2) is stood in for by nested
ellipsoidal shells with interior fill, since the CT volumes and trained
models are not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Value of the degree-0 real spherical harmonic, used only to express a target
# base colour as a DC coefficient (colour = dc * Y00 + 0.5).
_Y00 = 0.28209479177387814

MAX_CLIP = 8


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------
def _finish(mean, log_scale, quat, logit, sh, layer):
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    log_scale = np.ascontiguousarray(log_scale, dtype=np.float32)
    quat = np.ascontiguousarray(quat, dtype=np.float32)
    logit = np.ascontiguousarray(logit, dtype=np.float32)
    sh = np.ascontiguousarray(sh, dtype=np.float32)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    return {
        "mean": mean,
        "log_scale": log_scale,
        "scale": np.exp(log_scale).astype(np.float32),
        "quat": quat,
        "opacity_logit": logit,
        "opacity": (1.0 / (1.0 + np.exp(-logit.astype(np.float64)))).astype(np.float32),
        "sh": sh,
        "layer": layer,
        "sh_degree": int(round(math.sqrt(sh.shape[0]))) - 1,
    }


def refresh_activations(scene):
    """Recompute the activated arrays after the raw ones were edited."""
    scene["scale"] = np.exp(scene["log_scale"]).astype(np.float32)
    scene["opacity"] = (1.0 / (1.0 + np.exp(-scene["opacity_logit"].astype(np.float64)))).astype(np.float32)
    return scene


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def uniform_cube_scene(n=4096, sh_degree=0, seed=0, log_scale_mu=-4.0, log_scale_sigma=0.5):
    """Means uniform in [-1,1]^3, one layer, colours uniform in [0,1].

    Draw order: means, log-scales, quaternions, opacity logits, colours.
    Higher SH bands (if any) are zero.
    """
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, (3, n))
    log_scale = rng.normal(log_scale_mu, log_scale_sigma, (3, n))
    quat = _unit_quats(rng, n)
    logit = rng.standard_normal(n)
    rgb = rng.uniform(0.0, 1.0, (3, n))
    nc = (sh_degree + 1) ** 2
    sh = np.zeros((nc, 3, n))
    sh[0] = (rgb - 0.5) / _Y00
    layer = np.zeros(n, dtype=np.uint8)
    return _finish(mean, log_scale, quat, logit, sh, layer)


# per-layer base colours, innermost first (bone, organs, vessels, muscle, skin,
# then generic tissue colours for deeper stacks)
_PALETTE = np.array([
    [0.92, 0.89, 0.80],
    [0.70, 0.35, 0.30],
    [0.75, 0.10, 0.12],
    [0.62, 0.22, 0.20],
    [0.93, 0.76, 0.65],
    [0.55, 0.60, 0.45],
    [0.40, 0.45, 0.70],
    [0.85, 0.65, 0.40],
])


def _random_dirs(rng, n):
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return d


def shell_scene(n_per_layer, n_layers, sh_degree=3, seed=0, log_scale_mu=-5.0,
                log_scale_sigma=0.7, palette=False, opacity="ct", surface_frac=0.8):
    """Nested ellipsoidal shells with interior fill, one shell per layer.

    Layer l of L has semi-axes r_l * (0.6, 0.75, 1.0) with
    r_l = 0.3 + 0.7 * l / (L - 1).  A fraction `surface_frac` of its points sit
    on the surface (radial jitter N(0, 0.01^2)); the rest fill the space inside
    shell l and outside shell l-1.  Layer 0 is innermost.

    opacity: "ct"     -> outermost layer logits N(-1,1), the others N(1,1)
             "normal" -> all logits N(0,1)
    palette: True  -> DC from a per-layer base colour plus N(0, 0.1^2)
             False -> every SH coefficient N(0, 0.1^2)
    """
    rng = np.random.default_rng(seed)
    L = n_layers
    n = n_per_layer * L
    axes = np.array([0.6, 0.75, 1.0])
    means = np.empty((3, n))
    layer = np.repeat(np.arange(L, dtype=np.uint8), n_per_layer)
    for l in range(L):
        r = 0.3 + 0.7 * l / (L - 1) if L > 1 else 1.0
        semi = (r * axes)[:, None]
        n_surf = int(round(surface_frac * n_per_layer))
        n_fill = n_per_layer - n_surf
        d = _random_dirs(rng, n_surf)
        jitter = rng.normal(0.0, 0.01, n_surf)
        surf = d * semi + d * jitter
        r_in = 0.3 + 0.7 * (l - 1) / (L - 1) if (L > 1 and l > 0) else 0.0
        semi_in = (r_in * axes)[:, None]
        fill = np.empty((3, 0))
        while fill.shape[1] < n_fill:
            cand = rng.uniform(-1.0, 1.0, (3, 4 * max(n_fill, 16))) * semi
            inside = np.sum((cand / semi) ** 2, axis=0) <= 1.0
            if r_in > 0:
                inside &= np.sum((cand / semi_in) ** 2, axis=0) > 1.0
            fill = np.concatenate([fill, cand[:, inside]], axis=1)
        base = l * n_per_layer
        means[:, base:base + n_surf] = surf
        means[:, base + n_surf:base + n_per_layer] = fill[:, :n_fill]
    log_scale = rng.normal(log_scale_mu, log_scale_sigma, (3, n))
    quat = _unit_quats(rng, n)
    if opacity == "ct":
        mu = np.where(layer == L - 1, -1.0, 1.0)
        logit = rng.normal(0.0, 1.0, n) + mu
    else:
        logit = rng.standard_normal(n)
    nc = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.1, (nc, 3, n))
    if palette:
        base_rgb = _PALETTE[np.arange(L) % len(_PALETTE)][layer].T  # [3, n]
        sh[0] += (base_rgb - 0.5) / _Y00
    return _finish(means, log_scale, quat, logit, sh, layer)


def perturbed_copy(scene, seed=1, mean_sigma=0.005, log_scale_sigma=0.05, sh_sigma=0.02, logit_sigma=0.1):
    """A copy of `scene` with Gaussian noise on the raw parameters (a target scene)."""
    rng = np.random.default_rng(seed)
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    out["mean"] = (out["mean"] + rng.normal(0, mean_sigma, out["mean"].shape)).astype(np.float32)
    out["log_scale"] = (out["log_scale"] + rng.normal(0, log_scale_sigma, out["log_scale"].shape)).astype(np.float32)
    out["sh"] = (out["sh"] + rng.normal(0, sh_sigma, out["sh"].shape)).astype(np.float32)
    out["opacity_logit"] = (out["opacity_logit"] + rng.normal(0, logit_sigma, out["opacity_logit"].shape)).astype(np.float32)
    return refresh_activations(out)


def subset(scene, idx):
    """Scene restricted to the Gaussians `idx` (order kept)."""
    out = dict(scene)
    for k in ("mean", "log_scale", "scale", "quat"):
        out[k] = np.ascontiguousarray(scene[k][:, idx])
    for k in ("opacity_logit", "opacity", "layer"):
        out[k] = np.ascontiguousarray(scene[k][idx])
    out["sh"] = np.ascontiguousarray(scene["sh"][:, :, idx])
    return out


def n_gaussians(scene):
    return int(scene["mean"].shape[1])


# --------------------------------------------------------------------------
# cameras (pinhole, OpenCV axes: x right, y down, z forward; p_cam = R p + t)
# --------------------------------------------------------------------------
def focal_for_fov(height, fov_y_deg=60.0):
    return (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)


def make_camera(R, t, width, height, fx=None, fy=None, cx=None, cy=None, fov_y_deg=60.0,
                znear=0.2, guard=1.3):
    f = focal_for_fov(height, fov_y_deg)
    return {
        "R": np.ascontiguousarray(np.asarray(R, dtype=np.float32).reshape(3, 3)),
        "t": np.ascontiguousarray(np.asarray(t, dtype=np.float32).reshape(3)),
        "fx": float(np.float32(f if fx is None else fx)),
        "fy": float(np.float32(f if fy is None else fy)),
        "cx": float(np.float32(width / 2.0 if cx is None else cx)),
        "cy": float(np.float32(height / 2.0 if cy is None else cy)),
        "width": int(width),
        "height": int(height),
        "znear": float(np.float32(znear)),
        "guard": float(np.float32(guard)),
    }


def look_at_rotation(center, target=(0.0, 0.0, 0.0)):
    """World->camera rotation whose z axis points from `center` to `target`."""
    c = np.asarray(center, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - c
    z /= np.linalg.norm(z)
    hint = np.array([0.0, 1.0, 0.0])
    if abs(np.dot(hint, z)) > 0.99:
        hint = np.array([0.0, 0.0, 1.0])
    x = np.cross(hint, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z])


def orbit_camera(direction, width, height, distance=3.0, fov_y_deg=60.0, offset_x=0.0):
    """Camera at distance*direction looking at the origin.

    offset_x shifts the camera centre along its own x axis (stereo eyes keep
    parallel axes)."""
    d = np.asarray(direction, dtype=np.float64)
    d /= np.linalg.norm(d)
    center = distance * d
    R = look_at_rotation(center)
    center = center + offset_x * R[0]
    t = -R @ center
    return make_camera(R, t, width, height, fov_y_deg=fov_y_deg)


def front_camera(width=128, height=128, distance=3.0, fov_y_deg=60.0):
    """Camera at (0,0,-distance) with R = I, looking along +z."""
    return make_camera(np.eye(3), [0.0, 0.0, distance], width, height, fov_y_deg=fov_y_deg)


def stereo_cameras(direction, width, height, ipd=0.064, distance=3.0, fov_y_deg=60.0):
    """Two eyes with parallel axes, centres at head -/+ ipd/2 along camera x."""
    return [orbit_camera(direction, width, height, distance, fov_y_deg, offset_x=-ipd / 2),
            orbit_camera(direction, width, height, distance, fov_y_deg, offset_x=+ipd / 2)]


def stereo_rig(direction, width, height, ipd=0.064, distance=3.0, fov_y_deg=60.0, toe_in_deg=0.0):
    """Left eye, right eye and the camera at their centre (the head camera,
    which also gives a shared depth order).  toe_in_deg = 0: parallel eyes
    (as stereo_cameras); > 0: each eye turned inwards by that angle about
    the head's y axis (converging eyes)."""
    d = np.asarray(direction, dtype=np.float64)
    d /= np.linalg.norm(d)
    head = distance * d
    Rh = look_at_rotation(head)
    eyes = []
    for sign in (-1.0, 1.0):
        c = head + sign * (ipd / 2) * Rh[0]
        a = math.radians(-sign * toe_in_deg)  # the left eye turns right, the right eye left
        Ry = np.array([[math.cos(a), 0.0, math.sin(a)], [0.0, 1.0, 0.0], [-math.sin(a), 0.0, math.cos(a)]])
        R = Ry @ Rh
        eyes.append(make_camera(R, -R @ c, width, height, fov_y_deg=fov_y_deg))
    centre = make_camera(Rh, -Rh @ head, width, height, fov_y_deg=fov_y_deg)
    return eyes[0], eyes[1], centre


def centre_camera(left, right):
    """The camera half way between two parallel eyes (their rotation, the
    midpoint of their centres): the camera of a shared stereo depth order."""
    R = np.asarray(left["R"], np.float64)
    c = 0.5 * (camera_center(left) + camera_center(right))
    return make_camera(R, -R @ c, left["width"], left["height"], fx=left["fx"], fy=left["fy"], cx=left["cx"],
                       cy=left["cy"], znear=left["znear"], guard=left["guard"])


def random_direction(rng):
    d = rng.standard_normal(3)
    return d / np.linalg.norm(d)


def camera_center(cam):
    R = np.asarray(cam["R"], np.float64)
    return -R.T @ np.asarray(cam["t"], np.float64)


# --------------------------------------------------------------------------
# view state: layer-activation mask, clip planes, background
# --------------------------------------------------------------------------
def view_state(layer_mask=0xFFFFFFFF, clips=(), bg=(0.0, 0.0, 0.0), sort_cam=None, layer_opacity=None,
               mip_2d_var=None):
    """sort_cam (optional): one depth order for all views of the call, the
    depth in this camera (the eye centre of a stereo frame).
    layer_opacity (optional): up to 32 factors in [0, 1], one per layer; a
    Gaussian of layer l is drawn with its opacity times factor l (layers not
    listed keep factor 0).
    mip_2d_var (optional): render with Mip-Splatting's 2D filter of this
    variance (px^2) instead of the fixed 0.3 px^2 dilation."""
    clips = list(clips)
    assert len(clips) <= MAX_CLIP
    vs = {
        "layer_mask": int(layer_mask) & 0xFFFFFFFF,
        "clips": [(np.asarray(n, np.float32).reshape(3), float(np.float32(d)), int(bits) & 0xFFFFFFFF)
                  for (n, d, bits) in clips],
        "bg": np.asarray(bg, np.float32).reshape(3),
    }
    if sort_cam is not None:
        vs["sort_cam"] = sort_cam
    if layer_opacity is not None:
        f = np.asarray(layer_opacity, np.float32).reshape(-1)
        assert f.size <= 32 and np.all((f >= 0) & (f <= 1))
        vs["layer_opacity"] = np.concatenate([f, np.zeros(32 - f.size, np.float32)])
    if mip_2d_var is not None:
        assert mip_2d_var > 0
        vs["mip_2d_var"] = float(np.float32(mip_2d_var))
    return vs


def with_sort_cam(vs, sort_cam):
    """A copy of view state vs with a shared depth order in sort_cam."""
    out = dict(vs)
    out["sort_cam"] = sort_cam
    return out


def random_view_state(rng, n_layers, n_clip_range=(1, 3), bg=(0.0, 0.0, 0.0)):
    """Random non-empty layer mask over n_layers and 1-3 random clip planes."""
    mask = int(rng.integers(1, 2 ** n_layers))
    k = int(rng.integers(n_clip_range[0], n_clip_range[1] + 1))
    clips = []
    for _ in range(k):
        nrm = random_direction(rng)
        d = float(rng.uniform(-0.3, 0.3))
        bits = int(rng.integers(1, 2 ** n_layers))
        clips.append((nrm, d, bits))
    return view_state(mask, clips, bg)


# --------------------------------------------------------------------------
# distinct depths
# --------------------------------------------------------------------------
def enforce_distinct_depths(scene, cams, seed=12345, rel_gap=4e-6, max_rounds=50):
    """Re-draw the means of Gaussians whose camera depths nearly coincide.

    Depths are taken in float64 along each camera's forward axis; any two
    Gaussians closer than rel_gap*depth in some view have the later index
    moved by a small random offset (in index order, deterministically) until no
    such pair remains.  The gap is wide enough that float32 evaluations of the
    depth cannot tie.
    """
    rng = np.random.default_rng(seed)
    mean = scene["mean"].astype(np.float64)
    for _ in range(max_rounds):
        bad = set()
        for cam in cams:
            R = np.asarray(cam["R"], np.float64)
            t = np.asarray(cam["t"], np.float64)
            z = R[2] @ mean + t[2]
            order = np.argsort(z, kind="stable")
            zs = z[order]
            close = np.nonzero(np.diff(zs) <= rel_gap * np.maximum(np.abs(zs[1:]), 1.0))[0]
            for k in close:
                a, b = order[k], order[k + 1]
                bad.add(int(max(a, b)))
        if not bad:
            scene["mean"] = mean.astype(np.float32)
            return scene
        for i in sorted(bad):
            mean[:, i] += rng.normal(0.0, 1e-3, 3)
        mean = mean.astype(np.float32).astype(np.float64)
    raise RuntimeError("could not separate depths")


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    scene: dict
    cams: list
    views: list
    extra: dict = field(default_factory=dict)


def plain_forward_4k(seed=0, distinct=True):
    """4,096 Gaussians, one layer, SH0, 128x128 from distance 3, fov 60."""
    scene = uniform_cube_scene(4096, 0, seed)
    cam = front_camera(128, 128)
    if distinct:
        enforce_distinct_depths(scene, [cam])
    return Workload("plain_forward_4k_128px", scene, [cam], [view_state(0x1)])


def training_step_200k(seed=0, n_per_layer=50_000, width=800, height=800, distinct=False):
    """4 nested shells x 50k, SH3 coefficients N(0, 0.1^2), one 800x800 view."""
    scene = shell_scene(n_per_layer, 4, 3, seed, log_scale_mu=-5.0, log_scale_sigma=0.7,
                        palette=False, opacity="normal")
    rng = np.random.default_rng(seed + 100)
    cam = orbit_camera(random_direction(rng), width, height)
    if distinct:
        enforce_distinct_depths(scene, [cam])
    target = perturbed_copy(scene, seed + 1)
    return Workload(f"training_step_{4 * n_per_layer // 1000}k_{width}px", scene, [cam],
                    [view_state(0xF)], {"target_scene": target})


def layered_stereo(n_per_layer=200_000, width=1832, height=1920, seed=0, frame_seed=0):
    """5 CT-like shells, SH3, two eyes with IPD 0.064, random mask and clips."""
    scene = shell_scene(n_per_layer, 5, 3, seed, log_scale_mu=-5.0, log_scale_sigma=0.7, palette=True)
    rng = np.random.default_rng(frame_seed + 200)
    cams = stereo_cameras(random_direction(rng), width, height)
    vs = random_view_state(rng, 5)
    return Workload(f"layered_stereo_{5 * n_per_layer // 1000}k_{width}x{height}x2", scene, cams, [vs, vs])


def poisson_trace(rate_hz, duration_s, seed=0, n_models=2, n_layers=5,
                  resolutions=((512, 512, 1), (1024, 1024, 1), (1832, 1920, 2))):
    """Open-loop Poisson arrivals with random model, resolution, mask and clips."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        model = int(rng.integers(0, n_models))
        w, h, eyes = resolutions[int(rng.integers(0, len(resolutions)))]
        d = random_direction(rng)
        cams = stereo_cameras(d, w, h) if eyes == 2 else [orbit_camera(d, w, h)]
        vs = random_view_state(rng, n_layers)
        out.append({"arrival": t, "model": model, "cams": cams, "view": vs})
    return out


def serving_models(n_a=500_000, n_b=2_000_000, n_layers=5):
    """The two resident models of the serving workload (CT-like shells, SH3)."""
    return [shell_scene(n_a // n_layers, n_layers, 3, seed=1, log_scale_mu=-5.0, log_scale_sigma=0.7, palette=True),
            shell_scene(n_b // n_layers, n_layers, 3, seed=2, log_scale_mu=-5.0, log_scale_sigma=0.7, palette=True)]


def layered_training_4m(n_per_layer=500_000, n_layers=8, width=1024, height=1024, pool=64, views_per_step=8,
                        seed=0):
    """8 shells x 500k, SH3 coefficients N(0, 0.1^2), a pool of orbit views
    of which `views_per_step` are rendered per step; layer n_layers-1
    trainable, the others frozen; the target is a perturbed copy."""
    scene = shell_scene(n_per_layer, n_layers, 3, seed, log_scale_mu=-5.0, log_scale_sigma=0.7,
                        palette=False, opacity="normal")
    rng = np.random.default_rng(seed + 300)
    cams = [orbit_camera(random_direction(rng), width, height) for _ in range(pool)]
    target = perturbed_copy(scene, seed + 1)
    name = f"layered_training_{n_layers * n_per_layer // 1000}k_{views_per_step}x{width}px"
    return Workload(name, scene, cams[:views_per_step], [view_state(0xFFFFFFFF)] * views_per_step,
                    {"target_scene": target, "pool": cams, "trainable_layers": 1 << (n_layers - 1)})

