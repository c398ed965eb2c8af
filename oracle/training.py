"""Training-side statistics of the method in plain numpy float64 (test
infrastructure only: the tests use it; the product path never imports it).

update_activity: the inactive-pruning activity of one optimiser step
(Sec. 3.2.2 tracks the optimisation of each Gaussian's position, colour and
scale).  Under the update reading, a Gaussian's activity for a step is the
weighted sum of how far the step moved its parameters:
    2 |d mean| + 0.1 |d sh| + 0.1 |d log scale|,
each |.| the Euclidean norm over that parameter's values of the Gaussian;
Gaussians of frozen layers are not tracked (their activity stays).

densify_plan / split_child: the choices of adaptive density control in the
Gaussian-splatting optimisation the paper trains with (Sec. 4.3), on the
trainable layers: clone small Gaussians and split large ones whose mean
screen-space gradient statistic reaches a threshold; a split child is a
point of the parent Gaussian with the parent's scale divided by 0.8 times
the number of children.
"""
from __future__ import annotations

import numpy as np


def update_activity(before, after, layer, trainable, activity):
    """activity (float64 [n]) plus one step's activity.  before / after map
    "mean" [3, n], "log_scale" [3, n] and "sh" [(D+1)^2, 3, n] to arrays."""
    layer = np.asarray(layer, np.int64)
    n = layer.shape[0]
    out = np.array(activity, np.float64, copy=True)
    live = (layer < 32) & (((int(trainable) >> np.minimum(layer, 31)) & 1) == 1)
    for i in range(n):
        if not live[i]:
            continue
        norms = {}
        for k in ("mean", "log_scale", "sh"):
            d = np.asarray(after[k], np.float64)[..., i] - np.asarray(before[k], np.float64)[..., i]
            norms[k] = float(np.sqrt(np.sum(d * d)))
        out[i] += 2.0 * norms["mean"] + 0.1 * norms["sh"] + 0.1 * norms["log_scale"]
    return out


def quat_rotation(q):
    """Rotation matrix of the quaternion q = (w, x, y, z) (normalised first)."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def densify_plan(grad_sum, count, scale, layer, trainable, grad_threshold, percent_dense, extent, views_per_step):
    """Adaptive density control's choice per Gaussian: 'clone', 'split' or
    None.  A trainable Gaussian seen in at least one view whose mean
    statistic (times views_per_step, see the trainer) reaches the threshold
    is cloned when its largest scale is at most percent_dense * extent,
    split otherwise."""
    out = []
    for i in range(len(layer)):
        li = int(layer[i])
        if li >= 32 or not (int(trainable) >> li) & 1 or count[i] <= 0:
            out.append(None)
            continue
        if float(grad_sum[i]) / float(count[i]) * views_per_step < grad_threshold:
            out.append(None)
            continue
        out.append("clone" if max(float(s) for s in np.asarray(scale)[:, i]) <= percent_dense * extent else "split")
    return out


def split_child(mean, scale, quat, z, n_split):
    """One child of a split Gaussian: the point mean + R(q) diag(scale) z of
    the Gaussian (z a standard normal sample for a random child) and the
    scale divided by 0.8 n_split."""
    R = quat_rotation(quat)
    m = np.asarray(mean, np.float64) + R @ (np.asarray(scale, np.float64) * np.asarray(z, np.float64))
    return m, np.asarray(scale, np.float64) / (0.8 * n_split)
