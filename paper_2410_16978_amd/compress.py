"""Compressed attribute sets for rendering (the importer side).

Sec. 4.3 renders its models with two compression levels: "low" stores the
point-cloud parameters as 16-bit floats and the spherical-harmonic
coefficients as packed triplets; "clustered" (high) replaces each Gaussian's
higher SH coefficients by one of a fixed number of shared sets found with
K-means clustering across all layers (16k variants; Sec. 3.3 notes that
clustering across layers lets them share information and that volume
renderings use a limited palette).  The paper gives the triplet as 6 bytes
and as roughly 10.6 bits per colour channel; this module reads it as one
32-bit word per RGB triplet with 11, 11 and 10 bits (10.67 bits per channel),
each channel an unsigned code over that channel's range in the model.

compress() returns numpy arrays laid out as gsr_compressed (gsr.h) expects:
  mean, scale, quat, opacity, sh_dc   half bit patterns (uint16), activated
                                      scale and opacity
  "half_packed":   sh_packed uint32[M][n], sh_lo / sh_step float32[3]
  "half_codebook": sh_index uint16[n], codebook half bits [K][S], an
                   entry's M x 3 values ([k][ch]) padded to S = 3M rounded up
                   to 8 halves (16-byte entries)
with M = (D+1)^2 - 1.  rasterizer.to_device_compressed() uploads them.
This is offline import work on the host (numpy): rendering reads only the
arrays it produces.
"""
from __future__ import annotations

import numpy as np

PACK_BITS = (11, 11, 10)
PACK_SHIFT = (0, 11, 22)


def codebook_stride(D):
    """Halves per codebook entry: 3 ((D+1)^2 - 1) rounded up to 8 (16 bytes)."""
    return (3 * ((D + 1) ** 2 - 1) + 7) // 8 * 8


def half_bits(a):
    """IEEE binary16 bit patterns (round to nearest even) of float values."""
    return np.ascontiguousarray(np.asarray(a, np.float32).astype(np.float16).view(np.uint16))


def pack_sh(rest):
    """rest float32 [M, 3, n] -> (words uint32 [M, n], lo float32 [3],
    step float32 [3]).  Channel ch gets codes q in [0, 2^b - 1] (b = 11, 11,
    10) with value lo + q step, step = (max - min) / (2^b - 1) over every
    coefficient of that channel, q the nearest code."""
    rest = np.asarray(rest, np.float32)
    M, _, n = rest.shape
    lo = np.zeros(3, np.float32)
    step = np.zeros(3, np.float32)
    words = np.zeros((M, n), np.uint32)
    if M == 0 or n == 0:
        return words, lo, step
    for ch in range(3):
        levels = (1 << PACK_BITS[ch]) - 1
        x = rest[:, ch, :].astype(np.float64)
        lo[ch] = np.float32(x.min())
        hi = float(x.max())
        step[ch] = np.float32((hi - float(lo[ch])) / levels) if hi > float(lo[ch]) else np.float32(1.0)
        q = np.clip(np.rint((x - float(lo[ch])) / float(step[ch])), 0, levels).astype(np.uint32)
        words |= q << np.uint32(PACK_SHIFT[ch])
    return words, lo, step


def _nearest(x, c, c2, chunk=16384):
    """Index of the nearest row of c for every row of x (squared Euclidean
    distance, ties to the lower index)."""
    out = np.empty(len(x), np.int64)
    for a in range(0, len(x), chunk):
        xb = x[a:a + chunk]
        d = c2[None, :] - 2.0 * (xb @ c.T)  # |x|^2 is the same for every centre
        out[a:a + chunk] = np.argmin(d, axis=1)
    return out


def kmeans(x, k, iters=8, sample=131072, seed=0):
    """K-means (Lloyd) on a random sample of the rows of x float32 [n, d],
    started from k distinct sample rows; empty clusters keep their centre.
    Returns (centres float32 [k, d], index of every row's nearest centre)."""
    x = np.ascontiguousarray(x, np.float32)
    n = len(x)
    rng = np.random.default_rng(seed)
    k = int(min(k, n))
    smp = x[rng.choice(n, min(n, max(sample, k)), replace=False)]
    c = smp[rng.choice(len(smp), k, replace=False)].astype(np.float32)
    for _ in range(iters):
        a = _nearest(smp, c, (c.astype(np.float64) ** 2).sum(1).astype(np.float32))
        sums = np.zeros((k, x.shape[1]), np.float64)
        np.add.at(sums, a, smp)
        cnt = np.bincount(a, minlength=k)
        nz = cnt > 0
        c[nz] = (sums[nz] / cnt[nz, None]).astype(np.float32)
    idx = _nearest(x, c, (c.astype(np.float64) ** 2).sum(1).astype(np.float32))
    return c, idx


def compress(scene, sh_mode="packed", codebook_size=16384, iters=8, sample=131072, seed=0):
    """Compressed attribute arrays of `scene` (a scenes.py dict with
    activated scale and opacity).  sh_mode "packed" or "codebook"."""
    D = int(scene["sh_degree"])
    sh = np.asarray(scene["sh"], np.float32)
    n = sh.shape[2]
    M = (D + 1) ** 2 - 1
    out = {"sh_degree": D, "n": n, "layer": np.ascontiguousarray(scene["layer"], np.uint8),
           "mean": half_bits(scene["mean"]), "scale": half_bits(scene["scale"]), "quat": half_bits(scene["quat"]),
           "opacity": half_bits(scene["opacity"]), "sh_dc": half_bits(sh[0])}
    if sh_mode == "packed":
        out["format"] = "half_packed"
        out["sh_packed"], out["sh_lo"], out["sh_step"] = pack_sh(sh[1:])
    elif sh_mode == "codebook":
        out["format"] = "half_codebook"
        S = codebook_stride(D)
        if M == 0 or n == 0:
            out["sh_index"] = np.zeros(n, np.uint16)
            out["codebook"] = np.zeros((1, S), np.uint16)
        else:
            if codebook_size > 65536:
                raise ValueError("at most 65536 codebook entries (16-bit indices)")
            vec = np.ascontiguousarray(sh[1:].transpose(2, 0, 1).reshape(n, M * 3))  # [n][k][ch]
            c, idx = kmeans(vec, codebook_size, iters=iters, sample=sample, seed=seed)
            out["sh_index"] = idx.astype(np.uint16)
            cb = np.zeros((len(c), S), np.uint16)
            cb[:, :3 * M] = half_bits(c)
            out["codebook"] = cb
        out["codebook_size"] = int(out["codebook"].shape[0])
    else:
        raise ValueError(f"unknown sh_mode {sh_mode!r}")
    return out


def nbytes_per_gaussian(comp):
    """Device bytes per Gaussian of a compressed set (the codebook apart)."""
    n = max(int(comp["n"]), 1)
    keys = ("mean", "scale", "quat", "opacity", "sh_dc", "layer", "sh_packed", "sh_index")
    return sum(comp[k].nbytes for k in keys if k in comp) / n
