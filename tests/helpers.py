"""Hand-built scenes for the closed-form tests (no rasterizer arithmetic)."""
import numpy as np

from paper_2410_16978_amd import scenes

Y00 = 0.28209479177387814


def make_scene(means, scales, quats=None, opacity=None, rgb=None, layer=None, sh_degree=0, sh=None,
               dtype=np.float32):
    means = np.asarray(means, np.float64).reshape(-1, 3).T
    n = means.shape[1]
    scales = np.broadcast_to(np.asarray(scales, np.float64).reshape(-1, 3).T, (3, n))
    if quats is None:
        quats = np.tile(np.array([[1.0], [0.0], [0.0], [0.0]]), (1, n))
    else:
        quats = np.asarray(quats, np.float64).reshape(-1, 4).T
    opacity = np.full(n, 0.8) if opacity is None else np.broadcast_to(np.asarray(opacity, np.float64), (n,))
    if sh is None:
        nc = (sh_degree + 1) ** 2
        sh = np.zeros((nc, 3, n))
        rgb = np.full((3, n), 0.5) if rgb is None else np.asarray(rgb, np.float64).reshape(-1, 3).T
        sh[0] = (rgb - 0.5) / Y00
    layer = np.zeros(n, np.uint8) if layer is None else np.asarray(layer, np.uint8).reshape(n)
    return {
        "mean": np.ascontiguousarray(means, dtype), "scale": np.ascontiguousarray(scales, dtype),
        "log_scale": np.ascontiguousarray(np.log(scales), dtype),
        "quat": np.ascontiguousarray(quats, dtype), "opacity": np.ascontiguousarray(opacity, dtype),
        "opacity_logit": np.ascontiguousarray(np.log(opacity / (1 - opacity)), dtype),
        "sh": np.ascontiguousarray(sh, dtype), "layer": layer, "sh_degree": int(round(np.sqrt(sh.shape[0]))) - 1,
    }


def axis_camera(width=128, height=128, f=110.0, cx=64.5, cy=64.5):
    """Camera at the origin looking down +z (R = I, t = 0)."""
    return scenes.make_camera(np.eye(3), [0, 0, 0], width, height, fx=f, fy=f, cx=cx, cy=cy)


def to64(scene):
    return {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype == np.float32 else v)
            for k, v in scene.items()}


def small_layered_scene(seed=0, n_per_layer=120, n_layers=3, sh_degree=3, log_scale_mu=-3.2):
    return scenes.shell_scene(n_per_layer, n_layers, sh_degree, seed, log_scale_mu=log_scale_mu,
                              log_scale_sigma=0.3, palette=True)
