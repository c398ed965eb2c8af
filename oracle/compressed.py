"""Decoding of compressed attribute sets in plain numpy (test infrastructure
only: the tests use it; the product path never imports it).

The compression levels of Sec. 4.3: 16-bit floats for the point-cloud
parameters; the higher spherical-harmonic coefficients either as one word
per RGB triplet (codes q of 11, 11 and 10 bits, value lo + q step per
channel, the product rounded to float32 and then the sum) or as a 16-bit
index into a codebook of coefficient sets (stored as 16-bit floats, each
entry padded to a multiple of 8 halves).
decode() turns such a set back into the float32 scene that the oracle
renders; pack_codes() is the plain definition of the triplet codes, and
nearest() the plain definition of a codebook assignment.
"""
from __future__ import annotations

import numpy as np


def half_to_float(bits):
    """IEEE binary16 bit patterns -> the float32 values they denote."""
    return np.asarray(bits, np.uint16).view(np.float16).astype(np.float32)


def decode(comp):
    """Float32 scene (mean, scale, quat, opacity activated, sh, layer) of a
    compressed attribute set."""
    D = int(comp["sh_degree"])
    n = int(comp["n"])
    M = (D + 1) ** 2 - 1
    sh = np.zeros((M + 1, 3, n), np.float32)
    sh[0] = half_to_float(comp["sh_dc"])
    if M:
        if comp["format"] == "half_packed":
            w = np.asarray(comp["sh_packed"], np.uint32)
            for ch, (shift, bits) in enumerate(((0, 11), (11, 11), (22, 10))):
                q = ((w >> np.uint32(shift)) & np.uint32((1 << bits) - 1)).astype(np.float32)
                prod = (q * np.float32(comp["sh_step"][ch])).astype(np.float32)
                sh[1:, ch, :] = (np.float32(comp["sh_lo"][ch]) + prod).astype(np.float32)
        elif comp["format"] == "half_codebook":
            # entries of S halves, S = 3M rounded up to a multiple of 8; the
            # first 3M are the coefficients, [k][ch]
            S = (3 * M + 7) // 8 * 8
            idx = np.asarray(comp["sh_index"], np.int64)
            cb = half_to_float(comp["codebook"]).reshape(-1, S)[:, :3 * M].reshape(-1, M, 3)
            sh[1:] = cb[idx].transpose(1, 2, 0)
        else:
            raise ValueError(comp["format"])
    return {"mean": half_to_float(comp["mean"]).reshape(3, n), "scale": half_to_float(comp["scale"]).reshape(3, n),
            "quat": half_to_float(comp["quat"]).reshape(4, n), "opacity": half_to_float(comp["opacity"]).reshape(n),
            "sh": sh, "layer": np.asarray(comp["layer"], np.uint8), "sh_degree": D}


def pack_codes(x, lo, step, bits):
    """The nearest code of each value: round((x - lo) / step) clamped to
    [0, 2^bits - 1] (float64 arithmetic on the float32 inputs)."""
    q = np.rint((np.asarray(x, np.float64) - float(lo)) / float(step))
    return np.clip(q, 0, (1 << bits) - 1).astype(np.int64)


def nearest(x, centres):
    """Squared-distance to the nearest centre of every row of x (float64),
    and the distances to all centres."""
    d = ((np.asarray(x, np.float64)[:, None, :] - np.asarray(centres, np.float64)[None, :, :]) ** 2).sum(-1)
    return d.min(1), d
