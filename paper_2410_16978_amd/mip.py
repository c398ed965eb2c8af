"""Mip-Splatting's 3D smoothing filter from a set of cameras (the
anti-aliasing the paper reports trying, Sec. 4.4; forward only here).

A Gaussian seen by a camera at depth d with focal length f is sampled at
f / d samples per unit length; the 3D filter limits its frequencies to the
highest rate any camera samples it at: an isotropic Gaussian of variance
k (d / f)^2 (k = 0.2), d / f the smallest over the cameras whose image,
widened by 15 % on every side, holds the centre.  Gaussians no camera sees
take the largest such value over the others.  The rasterizer applies it
(gsr_model.filter_3d) by widening each scale to sqrt(s^2 + f^2) and scaling
the opacity to keep the Gaussian's integral.
"""
from __future__ import annotations

import numpy as np


def filter_3d_variance(mean, cams, k=0.2, margin=0.15):
    """float32 [n] variances for the centres mean [3, n]."""
    mean = np.asarray(mean, np.float64)
    n = mean.shape[1]
    best = np.full(n, np.inf)
    for c in cams:
        R = np.asarray(c["R"], np.float64).reshape(3, 3)
        t = np.asarray(c["t"], np.float64)
        p = R @ mean + t[:, None]
        z = p[2]
        ok = z > float(c["znear"])
        zs = np.where(ok, z, 1.0)
        u = float(c["fx"]) * p[0] / zs + float(c["cx"])
        v = float(c["fy"]) * p[1] / zs + float(c["cy"])
        W, H = float(c["width"]), float(c["height"])
        ok &= (u >= -margin * W) & (u <= (1 + margin) * W) & (v >= -margin * H) & (v <= (1 + margin) * H)
        ratio = z / float(c["fx"])
        best = np.where(ok & (ratio < best), ratio, best)
    seen = np.isfinite(best)
    if not seen.all():
        best[~seen] = best[seen].max() if seen.any() else 0.0
    return (k * best * best).astype(np.float32)
