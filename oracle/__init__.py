"""Python access to the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the product path never imports it.  It marshals numpy arrays into the
plain C++ reference in oracle.cpp (see oracle.h for the definitions) and
shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("znear", C.c_float), ("guard", C.c_float)]


class Clip(C.Structure):
    _fields_ = [("n", C.c_float * 3), ("d", C.c_float), ("layer_bits", C.c_uint32)]


class View(C.Structure):
    _fields_ = [("layer_mask", C.c_uint32), ("n_clip", C.c_int32), ("clip", Clip * 8), ("bg", C.c_float * 3),
                ("layer_fade", C.c_int32), ("layer_opacity", C.c_float * 32), ("mip_2d", C.c_int32),
                ("mip_2d_var", C.c_float)]


def _model_struct(ptr_t):
    class M(C.Structure):
        _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("mean", ptr_t), ("scale", ptr_t),
                    ("quat", ptr_t), ("opacity", ptr_t), ("sh", ptr_t), ("layer", C.POINTER(C.c_uint8)),
                    ("filter_3d", ptr_t)]
    return M


Model32 = _model_struct(C.POINTER(C.c_float))
Model64 = _model_struct(C.POINTER(C.c_double))


class Outputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("alpha", C.c_void_p), ("final_T", C.c_void_p),
                ("last", C.POINTER(C.c_uint32)), ("n_contrib", C.POINTER(C.c_uint32)),
                ("margin", C.POINTER(C.c_float)), ("rec", C.c_void_p), ("rect", C.POINTER(C.c_int32)),
                ("n_tiles", C.POINTER(C.c_uint32)), ("clamp", C.POINTER(C.c_uint32)),
                ("keys_emit", C.POINTER(C.c_uint64)), ("vals_emit", C.POINTER(C.c_uint32)),
                ("keys", C.POINTER(C.c_uint64)), ("vals", C.POINTER(C.c_uint32)),
                ("pair_cap", C.c_uint64), ("ranges", C.POINTER(C.c_uint32)), ("counts", C.c_uint64 * 4),
                ("near_rec", C.POINTER(C.c_uint8))]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        for name, mtype, rtype in (("oracle_render_f32", Model32, C.c_float), ("oracle_render_f64", Model64, C.c_double)):
            f = getattr(_lib, name)
            f.argtypes = [C.c_int, C.POINTER(mtype), C.POINTER(Camera), C.POINTER(View), C.c_int, C.c_int,
                          C.POINTER(Outputs), C.c_int, C.POINTER(Camera)]
            f.restype = C.c_int
        for name, mtype, in_t, out_t in (("oracle_backward_f32", Model32, C.c_float, C.c_float),
                                         ("oracle_backward_f64", Model64, C.c_double, C.c_double),
                                         ("oracle_backward_exact", Model32, C.c_float, C.c_double)):
            f = getattr(_lib, name)
            Pi, Po = C.POINTER(in_t), C.POINTER(out_t)
            f.argtypes = [C.c_int, C.POINTER(mtype), C.POINTER(Camera), C.POINTER(View), Pi, Pi, C.c_uint32,
                          Po, Po, Po, Po, Po, Po, Po] + ([Po, C.c_int] if name.endswith("exact") else []) + [
                              C.c_int, Po, Po]
            f.restype = C.c_int
        _lib.oracle_sh_basis_f64.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib.oracle_sh_basis_f32.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float)]
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def camera_struct(cam):
    c = Camera()
    R = np.asarray(cam["R"], np.float32).reshape(9)
    t = np.asarray(cam["t"], np.float32).reshape(3)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.fx, c.fy, c.cx, c.cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    c.width, c.height = cam["width"], cam["height"]
    c.znear, c.guard = cam["znear"], cam["guard"]
    return c


def view_struct(vs):
    v = View()
    v.layer_mask = vs["layer_mask"] & 0xFFFFFFFF
    v.n_clip = len(vs["clips"])
    for k, (n, d, bits) in enumerate(vs["clips"]):
        for j in range(3):
            v.clip[k].n[j] = float(n[j])
        v.clip[k].d = float(d)
        v.clip[k].layer_bits = bits & 0xFFFFFFFF
    for j in range(3):
        v.bg[j] = float(vs["bg"][j])
    if vs.get("layer_opacity") is not None:
        v.layer_fade = 1
        for l, f in enumerate(vs["layer_opacity"]):
            v.layer_opacity[l] = float(f)
    if vs.get("mip_2d_var") is not None:
        v.mip_2d = 1
        v.mip_2d_var = float(vs["mip_2d_var"])
    return v


class _ModelArrays:
    """Keeps the converted arrays alive while the C call runs."""

    def __init__(self, scene, dtype):
        self.dtype = np.dtype(dtype)
        ct = C.c_float if self.dtype == np.float32 else C.c_double
        self.arrs = {k: np.ascontiguousarray(scene[k], dtype=self.dtype)
                     for k in ("mean", "scale", "quat", "opacity", "sh")}
        self.layer = np.ascontiguousarray(scene["layer"], dtype=np.uint8)
        self.filter_3d = None
        if scene.get("filter_3d") is not None:
            self.filter_3d = np.ascontiguousarray(scene["filter_3d"], dtype=self.dtype)
        M = Model32 if self.dtype == np.float32 else Model64
        self.struct = M(int(self.layer.shape[0]), int(scene["sh_degree"]),
                        *[_ptr(self.arrs[k], ct) for k in ("mean", "scale", "quat", "opacity", "sh")],
                        _ptr(self.layer, C.c_uint8),
                        None if self.filter_3d is None else _ptr(self.filter_3d, ct))


def render(scenes, cams, views, tile=16, brute_force=False, dtype=np.float32, pairs=False, n_threads=0,
           sort_cams=None):
    """Render views; `scenes` is one scene for every view or a list, one per view.
    sort_cams (optional, one camera per view): the depth order of each view's
    pairs is the depth in that camera (the eyes of a stereo frame given the
    same centre camera share one order); default each view's own.

    Returns a dict of numpy arrays: rgb [V][3][H][W] (list if resolutions
    differ), alpha, final_T, last, n_contrib, margin, rec [R][10], rect, n_tiles,
    clamp, near_rec (records with a threshold decision below margin 1), ranges,
    counts (K, E, A, tiles), and with pairs=True keys_emit,
    vals_emit, keys, vals.
    """
    if isinstance(scenes, dict):
        scenes = [scenes] * len(cams)
    assert len(scenes) == len(cams) == len(views)
    dtype = np.dtype(dtype)
    L = lib()
    models_keep = {}
    mstructs = []
    for s in scenes:
        key = id(s)
        if key not in models_keep:
            models_keep[key] = _ModelArrays(s, dtype)
        mstructs.append(models_keep[key].struct)
    V = len(cams)
    M = Model32 if dtype == np.float32 else Model64
    marr = (M * max(V, 1))(*mstructs)
    carr = (Camera * max(V, 1))(*[camera_struct(c) for c in cams])
    varr = (View * max(V, 1))(*[view_struct(v) for v in views])
    sarr = None if sort_cams is None else (Camera * max(V, 1))(*[camera_struct(c) for c in sort_cams])
    n_pix = sum(c["width"] * c["height"] for c in cams)
    n_rec = sum(int(s["mean"].shape[1]) for s in scenes)
    tiles = sum(((c["width"] + tile - 1) // tile) * ((c["height"] + tile - 1) // tile) for c in cams)
    res = {
        "rgb": np.zeros(3 * n_pix, dtype), "alpha": np.zeros(n_pix, dtype), "final_T": np.zeros(n_pix, dtype),
        "last": np.zeros(n_pix, np.uint32), "n_contrib": np.zeros(n_pix, np.uint32),
        "margin": np.zeros(n_pix, np.float32), "rec": np.zeros((max(n_rec, 1), 10), dtype),
        "rect": np.zeros((max(n_rec, 1), 4), np.int32), "n_tiles": np.zeros(max(n_rec, 1), np.uint32),
        "clamp": np.zeros(max(n_rec, 1), np.uint32), "ranges": np.zeros((max(tiles, 1), 2), np.uint32),
        "near_rec": np.zeros(max(n_rec, 1), np.uint8),
    }
    out = Outputs()
    ct = C.c_float if dtype == np.float32 else C.c_double
    out.rgb = res["rgb"].ctypes.data
    out.alpha = res["alpha"].ctypes.data
    out.final_T = res["final_T"].ctypes.data
    out.last = _ptr(res["last"], C.c_uint32)
    out.n_contrib = _ptr(res["n_contrib"], C.c_uint32)
    out.margin = _ptr(res["margin"], C.c_float)
    out.rec = res["rec"].ctypes.data
    out.rect = _ptr(res["rect"], C.c_int32)
    out.n_tiles = _ptr(res["n_tiles"], C.c_uint32)
    out.clamp = _ptr(res["clamp"], C.c_uint32)
    out.ranges = _ptr(res["ranges"], C.c_uint32)
    out.near_rec = _ptr(res["near_rec"], C.c_uint8)
    fn = L.oracle_render_f32 if dtype == np.float32 else L.oracle_render_f64
    if pairs:
        # first call sizes the pair arrays
        out.pair_cap = 0
        probe = Outputs()
        probe.pair_cap = 0
        rc = fn(V, marr, carr, varr, tile, int(brute_force), C.byref(probe), n_threads, sarr)
        if rc != 0:
            raise RuntimeError(f"oracle render failed: {rc}")
        K = int(probe.counts[0])
        for k, t in (("keys_emit", np.uint64), ("vals_emit", np.uint32), ("keys", np.uint64), ("vals", np.uint32)):
            res[k] = np.zeros(max(K, 1), t)
        out.keys_emit = _ptr(res["keys_emit"], C.c_uint64)
        out.vals_emit = _ptr(res["vals_emit"], C.c_uint32)
        out.keys = _ptr(res["keys"], C.c_uint64)
        out.vals = _ptr(res["vals"], C.c_uint32)
        out.pair_cap = K
    rc = fn(V, marr, carr, varr, tile, int(brute_force), C.byref(out), n_threads, sarr)
    if rc != 0:
        raise RuntimeError(f"oracle render failed: {rc}")
    K, E, A, T = (int(x) for x in out.counts)
    res["counts"] = {"K": K, "E": E, "A": A, "tiles": T}
    res["rec"] = res["rec"][:n_rec]
    res["rect"] = res["rect"][:n_rec]
    res["n_tiles"] = res["n_tiles"][:n_rec]
    res["clamp"] = res["clamp"][:n_rec]
    res["near_rec"] = res["near_rec"][:n_rec]
    res["ranges"] = res["ranges"][:tiles]
    if pairs:
        for k in ("keys_emit", "vals_emit", "keys", "vals"):
            res[k] = res[k][:K]
    # per-view image views
    same = len({(c["width"], c["height"]) for c in cams}) <= 1
    if same and V > 0:
        H, W = cams[0]["height"], cams[0]["width"]
        res["rgb"] = res["rgb"].reshape(V, 3, H, W)
        for k in ("alpha", "final_T", "last", "n_contrib", "margin"):
            res[k] = res[k].reshape(V, H, W)
    else:
        rgbs, others = [], {k: [] for k in ("alpha", "final_T", "last", "n_contrib", "margin")}
        po = 0
        for c in cams:
            H, W = c["height"], c["width"]
            rgbs.append(res["rgb"][3 * po:3 * (po + H * W)].reshape(3, H, W))
            for k in others:
                others[k].append(res[k][po:po + H * W].reshape(H, W))
            po += H * W
        res["rgb"] = rgbs
        res.update(others)
    return res


def backward(scene, cams, views, dL_drgb, dL_dalpha, trainable=0xFFFFFFFF, dtype=np.float32, n_threads=0,
             cond=False):
    """Exact gradients of sum(dL_drgb*rgb) + sum(dL_dalpha*alpha) w.r.t. the
    activated parameters of one scene rendered in every view.

    dtype float32 / float64: forward and gradient in that precision.
    dtype "exact": the float32 forward's decisions (records, pair lists,
    skips, clamps, stops) with the gradient evaluated in float64 from the
    float32 records; inputs are taken as float32, results are float64.
    dtype "exact_fwd_values": as "exact", but each blended pair's pixel
    offset, G, alpha and transmittance are the float32 forward's own values.
    cond=True (exact dtypes): g["cond"] holds each entry's condition (the
    magnitude sum of its per-pixel contributions, see oracle.h), keyed and
    shaped like the gradients."""
    fwd_values = isinstance(dtype, str) and dtype == "exact_fwd_values"
    exact = isinstance(dtype, str) and dtype in ("exact", "exact_fwd_values")
    in_dt = np.dtype(np.float32) if exact else np.dtype(dtype)
    out_dt = np.dtype(np.float64) if exact else in_dt
    L = lib()
    ma = _ModelArrays(scene, in_dt)
    V = len(cams)
    carr = (Camera * max(V, 1))(*[camera_struct(c) for c in cams])
    varr = (View * max(V, 1))(*[view_struct(v) for v in views])
    n = int(ma.layer.shape[0])
    nc = (int(scene["sh_degree"]) + 1) ** 2
    g = {"mean": np.zeros((3, n), out_dt), "scale": np.zeros((3, n), out_dt), "quat": np.zeros((4, n), out_dt),
         "opacity": np.zeros(n, out_dt), "sh": np.zeros((nc, 3, n), out_dt), "max_contrib": np.zeros(n, out_dt),
         "activity": np.zeros(n, out_dt), "densify_grad": np.zeros(n, out_dt), "densify_count": np.zeros(n, out_dt)}
    drgb = np.ascontiguousarray(dL_drgb, in_dt).reshape(-1)
    dal = np.ascontiguousarray(dL_dalpha, in_dt).reshape(-1)
    ci = C.c_float if in_dt == np.float32 else C.c_double
    co = C.c_float if out_dt == np.float32 else C.c_double
    fn = L.oracle_backward_exact if exact else (L.oracle_backward_f32 if in_dt == np.float32
                                                 else L.oracle_backward_f64)
    packed = np.zeros((11 + 3 * nc) * n, np.float64) if (cond and exact) else None
    extra = (_ptr(packed, C.c_double), int(fwd_values)) if exact else ()
    rc = fn(V, C.byref(ma.struct), carr, varr, _ptr(drgb, ci), _ptr(dal, ci), trainable & 0xFFFFFFFF,
            _ptr(g["mean"], co), _ptr(g["scale"], co), _ptr(g["quat"], co), _ptr(g["opacity"], co),
            _ptr(g["sh"], co), _ptr(g["max_contrib"], co), _ptr(g["activity"], co), *extra, n_threads,
            _ptr(g["densify_grad"], co), _ptr(g["densify_count"], co))
    if rc != 0:
        raise RuntimeError(f"oracle backward failed: {rc}")
    if packed is not None:
        g["cond"] = {"mean": packed[:3 * n].reshape(3, n), "scale": packed[3 * n:6 * n].reshape(3, n),
                     "quat": packed[6 * n:10 * n].reshape(4, n), "opacity": packed[10 * n:11 * n],
                     "sh": packed[11 * n:].reshape(nc, 3, n)}
    return g


def sh_basis(d, dtype=np.float64):
    dtype = np.dtype(dtype)
    L = lib()
    d = np.ascontiguousarray(d, dtype)
    out = np.zeros(16, dtype)
    if dtype == np.float64:
        L.oracle_sh_basis_f64(_ptr(d, C.c_double), _ptr(out, C.c_double))
    else:
        L.oracle_sh_basis_f32(_ptr(d, C.c_float), _ptr(out, C.c_float))
    return out
