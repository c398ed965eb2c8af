"""Python binding of the HIP rasterizer's C ABI (include/gsr.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every stage of the rasterizer runs in the library's
kernels.  There is no fallback: if libgsr.so is missing or fails to load,
every call raises.

Entry points (same names as the C ABI):
  rasterize_forward(model, cams, views, ...)   -> rgb, alpha, ForwardState
  rasterize_backward(model, cams, views, state, dL_drgb, dL_dalpha, ...)
  render_batch(models, requests, ...)          -> per-request images + status
  workspace_size(n, n_views, width, height, pair_capacity)

`model` is a dict of CUDA tensors in the structure-of-arrays layout of
gsr.h: mean [3,n], scale [3,n] (activated), quat [4,n] (w,x,y,z),
opacity [n] (activated), sh [(D+1)^2,3,n], layer [n] uint8, and an int
"sh_degree".  Cameras and view states are the dicts of `scenes`.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")
_lib = None

GSR_OK, GSR_EINVAL, GSR_ENOSPACE, GSR_EHIP, GSR_EDEVICE = 0, -1, -2, -3, -4
MAX_CLIP = 8
RECORD_FLOATS = 12
TILE = 16


class GsrError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("znear", C.c_float), ("guard", C.c_float)]


class ClipPlane(C.Structure):
    _fields_ = [("n", C.c_float * 3), ("d", C.c_float), ("layer_bits", C.c_uint32)]


class ViewState(C.Structure):
    _fields_ = [("layer_mask", C.c_uint32), ("n_clip", C.c_int32), ("clip", ClipPlane * MAX_CLIP),
                ("bg", C.c_float * 3), ("sort_shared", C.c_int32), ("sort_cam", Camera),
                ("layer_fade", C.c_int32), ("layer_opacity", C.c_float * 32), ("mip_2d", C.c_int32),
                ("mip_2d_var", C.c_float)]


class Compressed(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p), ("opacity", C.c_void_p),
                ("sh_dc", C.c_void_p), ("sh_packed", C.c_void_p), ("sh_lo", C.c_float * 3),
                ("sh_step", C.c_float * 3), ("sh_index", C.c_void_p), ("codebook", C.c_void_p),
                ("codebook_size", C.c_int32), ("reserved", C.c_int32)]


class Model(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("mean", C.c_void_p), ("scale", C.c_void_p),
                ("quat", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p), ("layer", C.c_void_p),
                ("raw", C.c_int32), ("format", C.c_int32), ("compressed", C.c_void_p), ("filter_3d", C.c_void_p)]


FORMATS = {"f32": 0, "half_packed": 1, "half_codebook": 2}


class FwdState(C.Structure):
    _fields_ = [("records", C.c_void_p), ("offsets", C.c_void_p), ("pair_vals", C.c_void_p),
                ("sort_sel", C.c_void_p), ("pair_emit", C.c_void_p), ("ranges", C.c_void_p),
                ("pixel_state", C.c_void_p), ("last", C.c_void_p), ("checkpoints", C.c_void_p),
                ("batch_map", C.c_void_p), ("counters", C.c_void_p), ("pair_capacity", C.c_uint32),
                ("batch_capacity", C.c_uint32)]


class Debug(C.Structure):
    _fields_ = [("n_tiles", C.c_void_p), ("tile_box", C.c_void_p), ("keys_emit", C.c_void_p),
                ("vals_emit", C.c_void_p), ("keys_sorted", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("g_mean", C.c_void_p), ("g_scale", C.c_void_p), ("g_quat", C.c_void_p),
                ("g_opacity", C.c_void_p), ("g_sh", C.c_void_p), ("densify_grad", C.c_void_p),
                ("densify_count", C.c_void_p)]


class AdamGroup(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("exp_avg", C.c_void_p), ("exp_avg_sq", C.c_void_p),
                ("lr", C.c_float)]


class Request(C.Structure):
    _fields_ = [("model", C.c_int32), ("n_views", C.c_int32), ("cam", Camera * 2), ("vs", ViewState),
                ("rgb", C.c_void_p * 2), ("alpha", C.c_void_p * 2)]


def lib():
    """Load libgsr.so (built by paper_2410_16978_amd/build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP rasterizer library not built: {LIB_PATH} is missing "
                           "(run paper_2410_16978_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    L.gsr_status_string.restype = C.c_char_p
    L.gsr_status_string.argtypes = [C.c_int]
    L.gsr_batch_capacity.restype = C.c_uint32
    L.gsr_batch_capacity.argtypes = [C.c_uint32, C.c_uint32]
    L.gsr_workspace_size.restype = C.c_size_t
    L.gsr_workspace_size.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint32, C.c_int32]
    L.gsr_rasterize_forward.restype = C.c_int
    L.gsr_rasterize_forward.argtypes = [C.POINTER(Model), C.c_int32, C.POINTER(Camera), C.POINTER(ViewState),
                                        C.POINTER(FwdState), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_uint32), C.POINTER(Debug), C.c_void_p, C.c_void_p]
    L.gsr_rasterize_forward_noalloc.restype = C.c_int
    L.gsr_rasterize_forward_noalloc.argtypes = [C.POINTER(Model), C.c_int32, C.POINTER(Camera), C.POINTER(ViewState),
                                                C.POINTER(FwdState), C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32),
                                                C.c_void_p]
    L.gsr_forward_check.restype = C.c_int
    L.gsr_forward_check.argtypes = [C.POINTER(FwdState), C.POINTER(C.c_uint32), C.c_void_p]
    L.gsr_rasterize_backward.restype = C.c_int
    L.gsr_rasterize_backward.argtypes = [C.POINTER(Model), C.c_int32, C.POINTER(Camera), C.POINTER(ViewState),
                                         C.POINTER(FwdState), C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                         C.c_size_t, C.POINTER(Grads), C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]
    L.gsr_batch_workspace_size.restype = C.c_size_t
    L.gsr_batch_workspace_size.argtypes = [C.POINTER(Model), C.c_int32, C.POINTER(Request), C.c_int32, C.c_uint32]
    L.gsr_render_batch.restype = C.c_int
    L.gsr_render_batch.argtypes = [C.POINTER(Model), C.c_int32, C.POINTER(Request), C.c_int32, C.c_uint32,
                                   C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p]
    L.gsr_l1_loss_workspace_size.restype = C.c_size_t
    L.gsr_l1_loss_workspace_size.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    L.gsr_l1_alpha_loss.restype = C.c_int
    L.gsr_l1_alpha_loss.argtypes = [C.c_int32, C.c_int32, C.c_int32] + [C.c_void_p] * 4 + [
        C.POINTER(C.c_float), C.c_void_p, C.c_size_t] + [C.c_void_p] * 4 + [C.c_void_p]
    L.gsr_adam_step.restype = C.c_int
    L.gsr_adam_step.argtypes = [C.c_int32, C.c_int32, C.c_uint32, C.c_void_p, C.POINTER(AdamGroup), C.c_float,
                                C.c_float, C.c_float, C.c_int32, C.c_void_p, C.c_void_p]
    L.gsr_update_activity.restype = C.c_int
    L.gsr_update_activity.argtypes = [C.c_int32, C.c_int32, C.c_uint32] + [C.c_void_p] * 8 + [C.c_void_p]
    L.gsr_activate.restype = C.c_int
    L.gsr_activate.argtypes = [C.POINTER(Model), C.c_void_p, C.c_void_p, C.c_void_p]
    L.gsr_timer_create.restype = C.c_int
    L.gsr_timer_create.argtypes = [C.POINTER(C.c_void_p)]
    L.gsr_timer_destroy.restype = None
    L.gsr_timer_destroy.argtypes = [C.c_void_p]
    L.gsr_timer_read.restype = C.c_int
    L.gsr_timer_read.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_uint32)]
    _lib = L
    return L


def status_string(status):
    return lib().gsr_status_string(int(status)).decode()


def _check(status, what):
    if status != GSR_OK:
        raise GsrError(status, what)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


# ---------------------------------------------------------------- marshalling
def camera_struct(cam):
    c = Camera()
    R = np.asarray(cam["R"], np.float32).reshape(9)
    t = np.asarray(cam["t"], np.float32).reshape(3)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.fx, c.fy, c.cx, c.cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.znear, c.guard = cam["znear"], cam["guard"]
    return c


def view_struct(vs):
    v = ViewState()
    v.layer_mask = int(vs["layer_mask"]) & 0xFFFFFFFF
    clips = vs.get("clips", ())
    if len(clips) > MAX_CLIP:
        raise ValueError("at most 8 clip planes")
    v.n_clip = len(clips)
    for k, (n, d, bits) in enumerate(clips):
        for j in range(3):
            v.clip[k].n[j] = float(n[j])
        v.clip[k].d = float(d)
        v.clip[k].layer_bits = int(bits) & 0xFFFFFFFF
    bg = vs.get("bg", (0.0, 0.0, 0.0))
    for j in range(3):
        v.bg[j] = float(bg[j])
    if vs.get("sort_cam") is not None:  # one depth order, in this camera, for all views of the call
        v.sort_shared = 1
        v.sort_cam = camera_struct(vs["sort_cam"])
    fade = vs.get("layer_opacity")
    if fade is not None:  # per-layer opacity factors of this view
        if len(fade) > 32:
            raise ValueError("at most 32 layer opacity factors")
        v.layer_fade = 1
        for l, f in enumerate(fade):
            v.layer_opacity[l] = float(f)
    if vs.get("mip_2d_var") is not None:  # Mip-Splatting 2D filter of this variance
        v.mip_2d = 1
        v.mip_2d_var = float(vs["mip_2d_var"])
    return v


def shared_order(views):
    """Whether a call with these view states uses one shared depth order."""
    return len(views) > 0 and views[0].get("sort_cam") is not None


_MODEL_KEYS = ("mean", "scale", "quat", "opacity", "sh", "layer")


def to_device(scene, device="cuda"):
    """Scene dict of numpy arrays -> dict of contiguous CUDA tensors."""
    out = {"sh_degree": int(scene["sh_degree"])}
    for k in _MODEL_KEYS:
        a = scene[k]
        dtype = torch.uint8 if k == "layer" else torch.float32
        out[k] = torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dtype).contiguous()
    if scene.get("filter_3d") is not None:  # Mip-Splatting 3D filter variances
        out["filter_3d"] = torch.as_tensor(np.ascontiguousarray(scene["filter_3d"], np.float32)).to(device)
    return out


def to_device_compressed(comp, device="cuda"):
    """Compressed attribute arrays (compress.compress) -> a model dict for
    the forward and batch calls (half bit patterns held as int16 tensors,
    packed words as int32)."""
    def dev(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a).view(dt)).to(device).contiguous()

    out = {"sh_degree": int(comp["sh_degree"]), "format": comp["format"],
           "layer": torch.as_tensor(np.ascontiguousarray(comp["layer"], np.uint8)).to(device)}
    for k in ("mean", "scale", "quat", "opacity", "sh_dc"):
        out[k] = dev(comp[k], np.int16)
    cs = Compressed(*[out[k].data_ptr() for k in ("mean", "scale", "quat", "opacity", "sh_dc")])
    if comp["format"] == "half_packed":
        out["sh_packed"] = dev(comp["sh_packed"], np.int32)
        cs.sh_packed = out["sh_packed"].data_ptr() if out["sh_packed"].numel() else None
        for ch in range(3):
            cs.sh_lo[ch] = float(comp["sh_lo"][ch])
            cs.sh_step[ch] = float(comp["sh_step"][ch])
    elif comp["format"] == "half_codebook":
        out["sh_index"] = dev(comp["sh_index"], np.int16)
        out["codebook"] = dev(comp["codebook"], np.int16)
        cs.sh_index = out["sh_index"].data_ptr()
        cs.codebook = out["codebook"].data_ptr()
        cs.codebook_size = int(comp["codebook_size"])
    else:
        raise ValueError(f"unknown format {comp['format']!r}")
    out["_cstruct"] = cs  # host struct the model struct points to (lives with the dict)
    if comp.get("filter_3d") is not None:
        out["filter_3d"] = torch.as_tensor(np.ascontiguousarray(comp["filter_3d"], np.float32)).to(device)
    return out


def _filter_3d_ptr(model, n):
    """Device pointer of the optional Mip-Splatting 3D filter variances."""
    f = model.get("filter_3d")
    if f is None:
        return None
    if not f.is_cuda or f.dtype != torch.float32 or tuple(f.shape) != (n,) or not f.is_contiguous():
        raise ValueError("model['filter_3d'] must be a contiguous CUDA float32 tensor [n]")
    return f.data_ptr()


def _compressed_model_struct(model):
    n = int(model["layer"].shape[0])
    D = int(model["sh_degree"])
    M = (D + 1) ** 2 - 1
    shapes = {"mean": (3, n), "scale": (3, n), "quat": (4, n), "opacity": (n,), "sh_dc": (3, n)}
    if model["format"] == "half_packed":
        shapes["sh_packed"] = (M, n)
    else:
        shapes["sh_index"] = (n,)
    for k, shp in shapes.items():
        t = model[k]
        if not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp or t.element_size() != (
                4 if k == "sh_packed" else 2):
            raise ValueError(f"compressed model[{k!r}]: contiguous CUDA {shp} of 16-bit (32-bit packed) words")
    if model["format"] == "half_codebook":
        cb = model["codebook"]
        S = (3 * M + 7) // 8 * 8
        if cb.dim() != 2 or cb.shape[1] != S or cb.element_size() != 2 or not cb.is_contiguous() or \
                cb.data_ptr() % 16:
            raise ValueError(f"compressed model['codebook']: contiguous 16-byte aligned [K, {S}] half bits")
    lay = model["layer"]
    if not lay.is_cuda or lay.dtype != torch.uint8 or tuple(lay.shape) != (n,):
        raise ValueError("model['layer'] must be a CUDA uint8 tensor [n]")
    return Model(n, D, None, None, None, None, None, lay.data_ptr(), 0, FORMATS[model["format"]],
                 C.addressof(model["_cstruct"]), _filter_3d_ptr(model, n))


def model_struct(model):
    if model.get("format", "f32") != "f32":
        return _compressed_model_struct(model)
    n = int(model["layer"].shape[0])
    D = int(model["sh_degree"])
    nc = (D + 1) ** 2
    shapes = {"mean": (3, n), "scale": (3, n), "quat": (4, n), "opacity": (n,), "sh": (nc, 3, n), "layer": (n,)}
    for k, shp in shapes.items():
        t = model[k]
        if not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
            raise ValueError(f"model[{k!r}] must be a contiguous CUDA tensor of shape {shp}, got "
                             f"{tuple(t.shape)} on {t.device}")
        want = torch.uint8 if k == "layer" else torch.float32
        if t.dtype != want:
            raise ValueError(f"model[{k!r}] must be {want}")
    return Model(n, D, *[model[k].data_ptr() for k in _MODEL_KEYS], 1 if model.get("raw", False) else 0, 0, None,
                 _filter_3d_ptr(model, n))


def activate(model, stream=None):
    """(scale [3,n], opacity [n]) as the kernels compute them from `model`
    (exp / logistic of the raw parameters if model["raw"], else copies)."""
    m = model_struct(model)
    n = int(model["layer"].shape[0])
    dev = model["mean"].device
    scale = torch.empty((3, n), dtype=torch.float32, device=dev)
    opacity = torch.empty((n,), dtype=torch.float32, device=dev)
    _check(lib().gsr_activate(C.byref(m), _ptr(scale), _ptr(opacity), _stream(stream)), "gsr_activate")
    return scale, opacity


# ---------------------------------------------------------------- timer
STAGES = ("project", "scan", "duplicate", "sort", "ranges", "blend", "blend_bwd", "project_bwd", "bwd_order")


class Timer:
    """Per-stage HIP-event timer of the library (gsr_timer)."""

    def __init__(self):
        h = C.c_void_p()
        _check(lib().gsr_timer_create(C.byref(h)), "gsr_timer_create")
        self.handle = h

    def read(self):
        """{stage: (total ms, launches)} since the last read (synchronises)."""
        ms = (C.c_float * len(STAGES))()
        calls = (C.c_uint32 * len(STAGES))()
        _check(lib().gsr_timer_read(self.handle, ms, calls), "gsr_timer_read")
        return {s: (float(ms[i]), int(calls[i])) for i, s in enumerate(STAGES)}

    def close(self):
        if self.handle:
            lib().gsr_timer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _timer(t):
    return t.handle if t is not None else None


# ---------------------------------------------------------------- forward
@dataclass
class ForwardState:
    """Device buffers carrying a forward to its backward (see gsr_fwd_state)."""
    records: torch.Tensor
    offsets: torch.Tensor
    pair_vals: torch.Tensor
    sort_sel: torch.Tensor
    pair_emit: torch.Tensor
    ranges: torch.Tensor
    pixel_state: torch.Tensor
    last: torch.Tensor
    checkpoints: torch.Tensor
    batch_map: torch.Tensor
    counters: torch.Tensor
    capacity: int
    batch_capacity: int
    workspace: torch.Tensor
    n_views: int
    width: int
    height: int
    n: int
    n_pairs: int = None
    generation: int = 0  # forwards run on this state (a backward checks its forward is the latest)
    shared: bool = False  # workspace sized for a shared depth order

    @property
    def final_T(self):
        return self.pixel_state.view(-1, 4)[:, 0]

    def struct(self):
        return FwdState(self.records.data_ptr(), self.offsets.data_ptr(), self.pair_vals.data_ptr(),
                        self.sort_sel.data_ptr(), self.pair_emit.data_ptr(), self.ranges.data_ptr(),
                        self.pixel_state.data_ptr(), self.last.data_ptr(), self.checkpoints.data_ptr(),
                        self.batch_map.data_ptr(), self.counters.data_ptr(), self.capacity, self.batch_capacity)


def workspace_size(n, n_views, width, height, pair_capacity, shared=False):
    return int(lib().gsr_workspace_size(int(n), int(n_views), int(width), int(height), int(pair_capacity),
                                        1 if shared else 0))


def _tiles(w, h):
    return ((w + TILE - 1) // TILE) * ((h + TILE - 1) // TILE)


def make_state(n, n_views, width, height, capacity, device="cuda", old=None, shared=False):
    """Allocate (or reuse, when the shapes match) a forward state; shared:
    its workspace also holds the buffers of a shared depth order."""
    capacity = int(max(capacity, 1))
    R = n * n_views
    X = _tiles(width, height) * n_views
    Q = n_views * width * height
    if old is not None and old.n == n and old.n_views == n_views and old.width == width and old.height == height \
            and old.capacity >= capacity and (old.shared or not shared):
        return old
    ws = workspace_size(n, n_views, width, height, capacity, shared)
    if ws == 0:
        raise GsrError(GSR_EINVAL, "workspace_size")
    B = int(lib().gsr_batch_capacity(capacity, X))
    kw = dict(device=device)
    return ForwardState(
        records=torch.empty(max(R, 1) * RECORD_FLOATS, dtype=torch.float32, **kw),
        offsets=torch.empty(R + 1, dtype=torch.int32, **kw),
        pair_vals=torch.empty(2 * capacity, dtype=torch.int32, **kw),
        sort_sel=torch.zeros(1, dtype=torch.int32, **kw),
        pair_emit=torch.empty(capacity, dtype=torch.int32, **kw),
        ranges=torch.empty(2 * max(X, 1), dtype=torch.int32, **kw),
        pixel_state=torch.empty(4 * max(Q, 1), dtype=torch.float32, **kw),
        last=torch.empty(max(Q, 1), dtype=torch.int32, **kw),
        checkpoints=torch.empty(B * 256 * 4, dtype=torch.float32, **kw),
        batch_map=torch.empty(X + 1 + B, dtype=torch.int32, **kw),
        counters=torch.zeros(4, dtype=torch.int32, **kw),
        capacity=capacity, batch_capacity=B, workspace=torch.empty(ws, dtype=torch.uint8, **kw),
        n_views=n_views, width=width, height=height, n=n, shared=bool(shared))


def rasterize_forward(model, cams, views, state=None, capacity=None, sync=True, debug=False, stream=None,
                      out=None, timer=None):
    """Render len(cams) views of one model (equal resolution).

    sync=True: the library reads the pair count once; when the pair buffers
    are too small they are regrown to the exact need and the call repeats.
    sync=False: no host synchronisation (the caller checks state later with
    forward_check).  Returns (rgb [V,3,H,W], alpha [V,H,W], state[, debug]).
    """
    L = lib()
    V = len(cams)
    if V == 0 or len(views) != V:
        raise ValueError("need one view state per camera")
    W, H = int(cams[0]["width"]), int(cams[0]["height"])
    n = int(model["layer"].shape[0])
    dev = model["mean"].device
    m = model_struct(model)
    carr = (Camera * V)(*[camera_struct(c) for c in cams])
    varr = (ViewState * V)(*[view_struct(v) for v in views])
    if capacity is None:
        capacity = state.capacity if state is not None else max(1024, 4 * n * V)
    shared = shared_order(views)
    st = make_state(n, V, W, H, capacity, dev, state, shared)
    if out is None:
        rgb = torch.empty((V, 3, H, W), dtype=torch.float32, device=dev)
        alpha = torch.empty((V, H, W), dtype=torch.float32, device=dev)
    else:
        rgb, alpha = out
    s = _stream(stream)
    dbg = None
    dbg_struct = None
    for _attempt in range(3):
        if debug:
            R = n * V
            dbg = {"n_tiles": torch.zeros(max(R, 1), dtype=torch.int32, device=dev),
                   "tile_box": torch.zeros((max(R, 1), 4), dtype=torch.int32, device=dev),
                   "keys_emit": torch.zeros(st.capacity, dtype=torch.int64, device=dev),
                   "vals_emit": torch.zeros(st.capacity, dtype=torch.int32, device=dev),
                   "keys_sorted": torch.zeros(st.capacity, dtype=torch.int64, device=dev)}
            dbg_struct = Debug(*[dbg[k].data_ptr() for k in ("n_tiles", "tile_box", "keys_emit", "vals_emit",
                                                             "keys_sorted")])
        fs = st.struct()
        npairs = C.c_uint32(0)
        rc = L.gsr_rasterize_forward(C.byref(m), V, carr, varr, C.byref(fs), _ptr(st.workspace),
                                     st.workspace.numel(), _ptr(rgb), _ptr(alpha),
                                     C.byref(npairs) if sync else None,
                                     C.byref(dbg_struct) if dbg_struct is not None else None, _timer(timer), s)
        if rc == GSR_ENOSPACE and sync:
            st = make_state(n, V, W, H, int(npairs.value * 1.125) + 1024, dev, None, shared)
            continue
        _check(rc, "gsr_rasterize_forward")
        st.n_pairs = int(npairs.value) if sync else None
        st.generation += 1
        if debug:
            return rgb, alpha, st, dbg
        return rgb, alpha, st
    raise GsrError(GSR_ENOSPACE, "gsr_rasterize_forward (capacity)")


NOALLOC_SCRATCH_BYTES = 64 << 20  # GSR_NOALLOC_SCRATCH_BYTES


def rasterize_forward_noalloc(model, cams, views, state, out, n_pairs=False, stream=None):
    """gsr_rasterize_forward_noalloc: the forward on the library's own scratch
    (no workspace, no device allocation in the call).  `state` (a
    ForwardState, make_state) and `out` = (rgb [V,3,H,W], alpha [V,H,W]) are
    the caller's; nothing is allocated or regrown here.  n_pairs=True
    synchronises once and returns the pair count (the call returns ENOSPACE,
    raised as GsrError, when it exceeds the state's capacity).  Returns
    (rgb, alpha, state)."""
    V = len(cams)
    if V == 0 or len(views) != V:
        raise ValueError("need one view state per camera")
    m = model_struct(model)
    carr = (Camera * V)(*[camera_struct(c) for c in cams])
    varr = (ViewState * V)(*[view_struct(v) for v in views])
    rgb, alpha = out
    fs = state.struct()
    npairs = C.c_uint32(0)
    rc = lib().gsr_rasterize_forward_noalloc(C.byref(m), V, carr, varr, C.byref(fs), _ptr(rgb), _ptr(alpha),
                                             C.byref(npairs) if n_pairs else None, _stream(stream))
    _check(rc, "gsr_rasterize_forward_noalloc")
    state.n_pairs = int(npairs.value) if n_pairs else None
    state.generation += 1
    return rgb, alpha, state


def forward_check(state, stream=None):
    """After a sync=False forward: returns the pair count, raises on overflow/error."""
    fs = state.struct()
    npairs = C.c_uint32(0)
    rc = lib().gsr_forward_check(C.byref(fs), C.byref(npairs), _stream(stream))
    if rc == GSR_ENOSPACE:
        raise GsrError(rc, f"forward needs {npairs.value} pairs, capacity {state.capacity}")
    _check(rc, "gsr_forward_check")
    return int(npairs.value)


# ---------------------------------------------------------------- backward
def rasterize_backward(model, cams, views, state, dL_drgb=None, dL_dalpha=None, trainable=0xFFFFFFFF,
                       max_contrib=None, activity=None, grads=None, stream=None, timer=None, densify=None):
    """Gradients w.r.t. the activated parameters (dict of tensors like model).
    densify (optional): (grad_sum, count) float32 [n] tensors accumulated
    with the density-control statistic (see gsr_grads in gsr.h)."""
    L = lib()
    V = len(cams)
    n = int(model["layer"].shape[0])
    D = int(model["sh_degree"])
    nc = (D + 1) ** 2
    dev = model["mean"].device
    m = model_struct(model)
    carr = (Camera * V)(*[camera_struct(c) for c in cams])
    varr = (ViewState * V)(*[view_struct(v) for v in views])
    if grads is None:
        grads = {"mean": torch.empty((3, n), dtype=torch.float32, device=dev),
                 "scale": torch.empty((3, n), dtype=torch.float32, device=dev),
                 "quat": torch.empty((4, n), dtype=torch.float32, device=dev),
                 "opacity": torch.empty((n,), dtype=torch.float32, device=dev),
                 "sh": torch.empty((nc, 3, n), dtype=torch.float32, device=dev)}
    g = Grads(*[grads[k].data_ptr() for k in ("mean", "scale", "quat", "opacity", "sh")])
    if densify is not None:
        for t in densify:
            if tuple(t.shape) != (n,) or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError("densify accumulators must be contiguous float32 [n]")
        g.densify_grad, g.densify_count = densify[0].data_ptr(), densify[1].data_ptr()
    for t in (dL_drgb, dL_dalpha):
        if t is not None and (not t.is_contiguous() or t.dtype != torch.float32):
            raise ValueError("upstream gradients must be contiguous float32")
    fs = state.struct()
    rc = L.gsr_rasterize_backward(C.byref(m), V, carr, varr, C.byref(fs), _ptr(dL_drgb), _ptr(dL_dalpha),
                                  int(trainable) & 0xFFFFFFFF, _ptr(state.workspace), state.workspace.numel(),
                                  C.byref(g), _ptr(max_contrib), _ptr(activity), _timer(timer), _stream(stream))
    _check(rc, "gsr_rasterize_backward")
    return grads


# ---------------------------------------------------------------- batch
def request_struct(model_index, cams, vs, rgbs, alphas):
    r = Request()
    r.model = int(model_index)
    r.n_views = len(cams)
    for e, cam in enumerate(cams):
        r.cam[e] = camera_struct(cam)
        r.rgb[e] = rgbs[e].data_ptr()
        r.alpha[e] = alphas[e].data_ptr()
    r.vs = view_struct(vs)
    return r


def batch_workspace_size(models_struct, reqs_struct, capacity):
    return int(lib().gsr_batch_workspace_size(models_struct, len(models_struct), reqs_struct, len(reqs_struct),
                                              int(capacity)))


def render_batch(models, requests, capacity, workspace=None, status=None, outputs=None, stream=None, timer=None):
    """Render requests [{"model": i, "cams": [cam] or [left, right], "view": vs}]
    over resident models in one pass.  Returns (outputs, status tensor,
    workspace); outputs[q] = (rgb list, alpha list).  Never synchronises."""
    L = lib()
    dev = models[0]["mean"].device
    mstructs = (Model * len(models))(*[model_struct(m) for m in models])
    if outputs is None:
        outputs = []
        for rq in requests:
            rgbs = [torch.empty((3, c["height"], c["width"]), dtype=torch.float32, device=dev) for c in rq["cams"]]
            alphas = [torch.empty((c["height"], c["width"]), dtype=torch.float32, device=dev) for c in rq["cams"]]
            outputs.append((rgbs, alphas))
    rstructs = (Request * len(requests))(*[request_struct(rq["model"], rq["cams"], rq["view"], o[0], o[1])
                                           for rq, o in zip(requests, outputs)])
    need = batch_workspace_size(mstructs, rstructs, capacity)
    if need == 0:
        raise GsrError(GSR_EINVAL, "gsr_batch_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if status is None or status.numel() < len(requests):
        status = torch.empty(len(requests), dtype=torch.int32, device=dev)
    rc = L.gsr_render_batch(mstructs, len(models), rstructs, len(requests), int(capacity), _ptr(workspace),
                            workspace.numel(), _ptr(status), _timer(timer), _stream(stream))
    _check(rc, "gsr_render_batch")
    return outputs, status, workspace


# ---------------------------------------------------------------- loss
_loss_ws = {}


def _loss_workspace(V, W, H, device, stream):
    """Workspace of the fused loss (block partial sums) per (device, stream, shape)."""
    key = (str(device), int(stream.value or 0), V, W, H)
    ws = _loss_ws.get(key)
    if ws is None:
        n = int(lib().gsr_l1_loss_workspace_size(V, W, H))
        if n == 0:
            raise ValueError("bad loss shape (n_views must be 1..16)")
        ws = torch.empty(n, dtype=torch.uint8, device=device)
        _loss_ws[key] = ws
    return ws


def l1_alpha_loss(rgb, alpha, target_rgb, target_alpha, bgs, loss=True, grads=False, g_loss=None, stream=None):
    """L1 loss of alpha-channel training (Sec. 3.2.1) on the library's fused
    kernels: target colour = target_rgb + (1 - target_alpha) * bg per view,
    L = mean|rgb - target| + mean|alpha - target_alpha|.  rgb [V,3,H,W],
    alpha [V,H,W]; bgs: V background colours.  Returns (loss [1] or None,
    dL_drgb or None, dL_dalpha or None); g_loss: incoming gradient [1]
    (None = 1)."""
    V, _, H, W = rgb.shape
    for t, shp in ((rgb, (V, 3, H, W)), (target_rgb, (V, 3, H, W)), (alpha, (V, H, W)), (target_alpha, (V, H, W))):
        if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("l1_alpha_loss: contiguous float32 rgb [V,3,H,W] and alpha [V,H,W] expected")
    bg = np.ascontiguousarray(np.asarray(bgs, np.float32).reshape(V, 3))
    s = _stream(stream)
    ws = _loss_workspace(V, W, H, rgb.device, s)
    out = torch.empty(1, dtype=torch.float32, device=rgb.device) if loss else None
    g_rgb = torch.empty_like(rgb) if grads else None
    g_a = torch.empty_like(alpha) if grads else None
    rc = lib().gsr_l1_alpha_loss(V, W, H, _ptr(rgb), _ptr(alpha), _ptr(target_rgb), _ptr(target_alpha),
                                 bg.ctypes.data_as(C.POINTER(C.c_float)), _ptr(ws), ws.numel(), _ptr(out),
                                 _ptr(g_loss), _ptr(g_rgb), _ptr(g_a), s)
    _check(rc, "gsr_l1_alpha_loss")
    return out, g_rgb, g_a



def update_activity(before, after, layer, sh_degree, trainable, activity, stream=None):
    """activity[i] += 2|d mean| + 0.1|d sh| + 0.1|d log_scale| for the
    Gaussians of trainable layers (gsr_update_activity); before / after map
    "mean" [3,n], "log_scale" [3,n] and "sh" [(D+1)^2,3,n] to contiguous
    float32 device tensors, layer uint8 [n], activity float32 [n]."""
    n = int(layer.shape[0])
    nc = (int(sh_degree) + 1) ** 2
    shapes = {"mean": (3, n), "log_scale": (3, n), "sh": (nc, 3, n)}
    for d in (before, after):
        for k, shp in shapes.items():
            t = d[k]
            if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"update_activity: {k} must be contiguous float32 {shp}")
    if tuple(activity.shape) != (n,) or activity.dtype != torch.float32 or layer.dtype != torch.uint8:
        raise ValueError("update_activity: activity float32 [n] and layer uint8 [n] expected")
    rc = lib().gsr_update_activity(n, int(sh_degree), int(trainable) & 0xFFFFFFFF, _ptr(before["mean"]),
                                   _ptr(after["mean"]), _ptr(before["log_scale"]), _ptr(after["log_scale"]),
                                   _ptr(before["sh"]), _ptr(after["sh"]), _ptr(layer), _ptr(activity), _stream(stream))
    _check(rc, "gsr_update_activity")


ADAM_KEYS = ("mean", "log_scale", "quat", "opacity_logit", "sh")


def adam_step(params, grads, exp_avg, exp_avg_sq, lrs, layer, sh_degree, trainable, step, betas=(0.9, 0.999),
              eps=1e-15, activity=None, stream=None):
    """gsr_adam_step: one Adam step, in place, on the Gaussians of the
    trainable layers; dicts keyed by ADAM_KEYS of contiguous float32 device
    tensors ([3,n], [3,n], [4,n], [n], [(D+1)^2,3,n]); activity (optional
    [n]) accumulates the step's update-norm activity."""
    n = int(layer.shape[0])
    nc = (int(sh_degree) + 1) ** 2
    shapes = {"mean": (3, n), "log_scale": (3, n), "quat": (4, n), "opacity_logit": (n,), "sh": (nc, 3, n)}
    groups = (AdamGroup * 5)()
    for gi, k in enumerate(ADAM_KEYS):
        for t in (params[k], grads[k], exp_avg[k], exp_avg_sq[k]):
            if tuple(t.shape) != shapes[k] or t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"adam_step: {k} tensors must be contiguous CUDA float32 {shapes[k]}")
        groups[gi] = AdamGroup(params[k].data_ptr(), grads[k].data_ptr(), exp_avg[k].data_ptr(),
                               exp_avg_sq[k].data_ptr(), float(lrs[k]))
    if layer.dtype != torch.uint8:
        raise ValueError("adam_step: layer must be uint8")
    if activity is not None and (tuple(activity.shape) != (n,) or activity.dtype != torch.float32):
        raise ValueError("adam_step: activity must be float32 [n]")
    rc = lib().gsr_adam_step(n, int(sh_degree), int(trainable) & 0xFFFFFFFF, _ptr(layer), groups, float(betas[0]),
                             float(betas[1]), float(eps), int(step), _ptr(activity), _stream(stream))
    _check(rc, "gsr_adam_step")
