"""Training-side statistics of the method in plain numpy float64 (test
infrastructure only: the tests use it; the product path never imports it).

update_activity: the inactive-pruning activity of one optimiser step
(Sec. 3.2.2 tracks the optimisation of each Gaussian's position, colour and
scale).  Under the update reading, a Gaussian's activity for a step is the
weighted sum of how far the step moved its parameters:
    2 |d mean| + 0.1 |d sh| + 0.1 |d log scale|,
each |.| the Euclidean norm over that parameter's values of the Gaussian;
Gaussians of frozen layers are not tracked (their activity stays).
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
