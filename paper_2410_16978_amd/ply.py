"""Layered splat assets as PLY files.

The paper keeps a trained multi-layer model as one PLY file whose vertices
are the Gaussians, with the layer of each Gaussian stored as an extra
per-vertex property (Sec. 3.2).  The vertex properties here are those
splat-training tools write, followed by the layer:

    x y z                      centre
    nx ny nz                   unused normals (written as 0)
    f_dc_0 f_dc_1 f_dc_2       SH degree-0 coefficient of r, g, b
    f_rest_0 ... f_rest_{3M-1} higher SH coefficients, channel-major:
                               f_rest_{ch * M + (k - 1)} is coefficient k of
                               channel ch, M = (D + 1)^2 - 1
    opacity                    logit of the opacity
    scale_0 scale_1 scale_2    log of the per-axis scale
    rot_0 rot_1 rot_2 rot_3    quaternion (w, x, y, z), not necessarily unit
    layer                      uchar layer id (absent: every Gaussian in 0)

All float properties are 32-bit; the file is binary little-endian.  Reading
accepts the properties in any order and ignores unknown ones.  The scene
dicts are those of scenes.py: planes `mean[3][n]`, `log_scale[3][n]`,
`quat[4][n]`, `opacity_logit[n]`, `sh[(D+1)^2][3][n]`, `layer[n]`, plus the
activated `scale` and `opacity`.
"""
from __future__ import annotations

import math

import numpy as np

from . import scenes

_PLY_TYPES = {
    "char": "i1", "int8": "i1", "uchar": "u1", "uint8": "u1", "short": "i2", "int16": "i2",
    "ushort": "u2", "uint16": "u2", "int": "i4", "int32": "i4", "uint": "u4", "uint32": "u4",
    "float": "f4", "float32": "f4", "double": "f8", "float64": "f8",
}


def _names(D):
    M = (D + 1) ** 2 - 1
    names = ["x", "y", "z", "nx", "ny", "nz", "f_dc_0", "f_dc_1", "f_dc_2"]
    names += [f"f_rest_{i}" for i in range(3 * M)]
    names += ["opacity", "scale_0", "scale_1", "scale_2", "rot_0", "rot_1", "rot_2", "rot_3"]
    return names


def write_ply(path, scene):
    """Write `scene` (raw parameters: log_scale, opacity_logit) as a binary
    little-endian layered PLY."""
    D = int(scene["sh_degree"])
    n = int(scene["mean"].shape[1])
    names = _names(D)
    M = (D + 1) ** 2 - 1
    dt = np.dtype([(nm, "<f4") for nm in names] + [("layer", "u1")])
    v = np.zeros(n, dt)
    for c, nm in enumerate("xyz"):
        v[nm] = scene["mean"][c]
    sh = np.asarray(scene["sh"], np.float32)
    for ch in range(3):
        v[f"f_dc_{ch}"] = sh[0, ch]
        for k in range(1, M + 1):
            v[f"f_rest_{ch * M + k - 1}"] = sh[k, ch]
    v["opacity"] = scene["opacity_logit"]
    for c in range(3):
        v[f"scale_{c}"] = scene["log_scale"][c]
    for c in range(4):
        v[f"rot_{c}"] = scene["quat"][c]
    v["layer"] = scene["layer"]
    header = ["ply", "format binary_little_endian 1.0", f"element vertex {n}"]
    header += [f"property float {nm}" for nm in names] + ["property uchar layer", "end_header"]
    with open(path, "wb") as f:
        f.write(("\n".join(header) + "\n").encode("ascii"))
        f.write(v.tobytes())


def read_ply(path):
    """Read a layered PLY into a scene dict (see the module docstring)."""
    with open(path, "rb") as f:
        if f.readline().strip() != b"ply":
            raise ValueError(f"{path}: not a PLY file")
        fmt, n, props, in_vertex, before = None, None, [], False, []
        while True:
            line = f.readline()
            if not line:
                raise ValueError(f"{path}: no end_header")
            tok = line.decode("ascii", "replace").split()
            if not tok or tok[0] == "comment" or tok[0] == "obj_info":
                continue
            if tok[0] == "end_header":
                break
            if tok[0] == "format":
                fmt = tok[1]
            elif tok[0] == "element":
                in_vertex = tok[1] == "vertex"
                if in_vertex:
                    n = int(tok[2])
                elif n is None:
                    before.append((tok[1], int(tok[2])))
            elif tok[0] == "property" and in_vertex:
                if tok[1] == "list":
                    raise ValueError(f"{path}: list properties on vertices are not supported")
                if tok[1] not in _PLY_TYPES:
                    raise ValueError(f"{path}: property type {tok[1]}")
                props.append((tok[2], "<" + _PLY_TYPES[tok[1]]))
        if fmt != "binary_little_endian":
            raise ValueError(f"{path}: format {fmt} (only binary_little_endian is read)")
        if n is None:
            raise ValueError(f"{path}: no vertex element")
        if before:
            raise ValueError(f"{path}: elements before the vertices are not supported")
        dt = np.dtype(props)
        v = np.frombuffer(f.read(dt.itemsize * n), dt, count=n)
    names = set(dt.names)
    n_rest = sum(1 for nm in names if nm.startswith("f_rest_"))
    if n_rest % 3:
        raise ValueError(f"{path}: {n_rest} f_rest properties is not a multiple of 3")
    M = n_rest // 3
    D = int(round(math.sqrt(M + 1))) - 1
    if (D + 1) ** 2 - 1 != M:
        raise ValueError(f"{path}: {M} higher SH coefficients per channel is no degree")
    need = [nm for nm in _names(D) if not nm.startswith("n")]
    missing = [nm for nm in need if nm not in names]
    if missing:
        raise ValueError(f"{path}: missing properties {missing}")
    mean = np.stack([v[c] for c in "xyz"]).astype(np.float32)
    sh = np.zeros(((D + 1) ** 2, 3, n), np.float32)
    for ch in range(3):
        sh[0, ch] = v[f"f_dc_{ch}"]
        for k in range(1, M + 1):
            sh[k, ch] = v[f"f_rest_{ch * M + k - 1}"]
    log_scale = np.stack([v[f"scale_{c}"] for c in range(3)]).astype(np.float32)
    quat = np.stack([v[f"rot_{c}"] for c in range(4)]).astype(np.float32)
    logit = np.asarray(v["opacity"], np.float32)
    layer = np.asarray(v["layer"], np.uint8) if "layer" in names else np.zeros(n, np.uint8)
    return scenes._finish(mean, log_scale, quat, logit, sh, layer)
