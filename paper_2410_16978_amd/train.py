"""Layered training with inactive-Gaussian pruning (Sec. 3.2).

Layers are trained consecutively: the Gaussians of earlier layers stay in
the scene and are rendered as background but receive no gradient (the
kernel zeroes them through `trainable_layers`), so the optimiser leaves
them untouched.  Every step renders a batch of views with a random
background colour and compares RGB and alpha with the target (alpha-channel
training, Sec. 3.2.1).

Inactive pruning (Sec. 3.2.2): the paper tracks how the optimisation moves
each Gaussian's position, colour and scale, compares that activity with a
threshold T (T0 = 0.015) at every densification interval (dR = 100 steps),
removes the trainable Gaussians at or below it and decays T by 0.975.  What
is measured is a reading; two are built:

* "update" (default): after each optimiser step, 2 |d mean| + 0.1 |d SH| +
  0.1 |d log scale| of the change the step made (gsr_update_activity),
  summed over the window and compared with T.  Adam's steps are about the
  learning rate in size whatever the gradient's scale, so a Gaussian the
  optimiser moves in most steps collects far more than T0 over a window and
  one it never moves collects exactly 0; the threshold then does not depend
  on the loss's scale.
* "gradient": the same weights on the L2 norms of the per-step gradients
  (fused into the backward kernel), averaged over the window.  Its scale is
  the loss's: at the 4M-Gaussian workload every trainable Gaussian's average
  is below T0.

Optionally, Gaussians whose largest alpha * T over the window stayed below
1/255 (they never visibly contributed) are removed as well; both criteria are
counted separately.
"""
from __future__ import annotations

import dataclasses
import io
import json

import numpy as np
import torch

from . import autograd as ag
from . import rasterizer as rz

PARAM_KEYS = ("mean", "log_scale", "quat", "opacity_logit", "sh")


@dataclasses.dataclass
class PruneConfig:
    interval: int = 100          # dR, the densification rate
    threshold: float = 0.015     # T0
    decay: float = 0.975
    use_max_contrib: bool = True
    min_contrib: float = 1.0 / 255.0
    use_activity: bool = True  # False: count the activity rule's decisions but prune by max_contrib only
    measure: str = "update"    # "update": optimiser-step norms, window sum; "gradient": gradient norms, window mean


class PruneState:
    """Window accumulation and the pruning decision (device-agnostic)."""

    def __init__(self, cfg: PruneConfig):
        self.cfg = cfg
        self.T = cfg.threshold
        self.steps_in_window = 0
        self.n_prunes = 0

    def schedule(self, k):
        """Threshold used at the k-th pruning step (k = 0, 1, ...)."""
        return self.cfg.threshold * self.cfg.decay ** k

    def due(self):
        return self.steps_in_window >= self.cfg.interval

    def decide(self, activity_sum, max_contrib, layer, trainable_layers):
        """Keep mask after a window; activity_sum is the window's sum.
        Returns keep (bool tensor) and per-criterion counts; decays T."""
        if self.cfg.measure == "update":
            score = activity_sum
        elif self.cfg.measure == "gradient":
            score = activity_sum / max(self.steps_in_window, 1)
        else:
            raise ValueError(f"unknown activity measure {self.cfg.measure!r}")
        trainable = ((int(trainable_layers) >> layer.to(torch.int64)) & 1).bool()
        inactive = trainable & (score <= self.T)
        invisible = trainable & (max_contrib < self.cfg.min_contrib) if self.cfg.use_max_contrib else \
            torch.zeros_like(inactive)
        keep = ~((inactive if self.cfg.use_activity else torch.zeros_like(inactive)) | invisible)
        counts = {"activity": int(inactive.sum()), "max_contrib": int(invisible.sum()),
                  "both": int((inactive & invisible).sum()), "pruned": int((~keep).sum()), "threshold": self.T}
        self.T *= self.cfg.decay
        self.n_prunes += 1
        self.steps_in_window = 0
        return keep, counts


class LayeredTrainer:
    """Adam on the trainable layers of a layered Gaussian scene."""

    def __init__(self, scene, cams, targets, trainable_layers, views_per_step=1, lrs=None, prune=None,
                 seed=0, device="cuda", sync=True):
        self.device = device
        self.params = {k: torch.tensor(np.ascontiguousarray(scene[k]), device=device, requires_grad=True)
                       for k in PARAM_KEYS}
        self.layer = torch.tensor(scene["layer"], device=device)
        self.sh_degree = int(scene["sh_degree"])
        self.cams = cams                              # pool of cameras (equal resolution)
        self.targets = targets                        # (rgb premultiplied [P,3,H,W], alpha [P,H,W]) tensors
        self.trainable = int(trainable_layers)
        self.views_per_step = views_per_step
        self.lrs = lrs or {"mean": 1.6e-4, "log_scale": 5e-3, "quat": 1e-3, "opacity_logit": 5e-2, "sh": 2.5e-3}
        self.opt = self._make_opt()
        self.prune = PruneState(prune or PruneConfig())
        self.rctx = ag.RenderContext(trainable_layers=self.trainable, track_activity=True, sync=sync,
                                     grad_activity=self.prune.cfg.measure == "gradient")
        self._before = None  # parameters before the optimiser step ("update" measure)
        self.rng = np.random.default_rng(seed)
        self.it = 0
        self.history = []

    def _make_opt(self, state=None):
        opt = torch.optim.Adam([{"params": [self.params[k]], "lr": self.lrs[k], "name": k} for k in PARAM_KEYS],
                               eps=1e-15)
        if state is not None:
            opt.load_state_dict(state)
        return opt

    @property
    def n(self):
        return int(self.layer.shape[0])

    def step(self):
        idx = self.rng.choice(len(self.cams), self.views_per_step, replace=False)
        bg = self.rng.uniform(0.0, 1.0, 3)
        cams = [self.cams[i] for i in idx]
        views = [{"layer_mask": 0xFFFFFFFF, "clips": [], "bg": tuple(bg)}] * len(cams)
        t_rgb = self.targets[0][idx].contiguous()
        t_alpha = self.targets[1][idx].contiguous()
        rgb, alpha = ag.render_params(self.params, self.layer, self.sh_degree, cams, views, self.rctx)
        loss = ag.l1_alpha_loss(rgb, alpha, t_rgb, t_alpha, [bg] * len(cams))
        self.opt.zero_grad(set_to_none=True)
        loss.backward()
        if self.prune.cfg.measure == "update":
            self._step_with_update_activity()
        else:
            self.opt.step()
        self.it += 1
        self.prune.steps_in_window += 1
        out = {"it": self.it, "loss": loss}
        if self.prune.due():
            out["prune"] = self.prune_now()
        return out

    def _step_with_update_activity(self):
        """The optimiser step, then the activity of the change it made."""
        keys = ("mean", "log_scale", "sh")
        if self._before is None or self._before["mean"].shape != self.params["mean"].shape:
            self._before = {k: torch.empty_like(self.params[k]) for k in keys}
        for k in keys:
            self._before[k].copy_(self.params[k].detach())
        self.opt.step()
        rz.update_activity(self._before, {k: self.params[k].detach() for k in keys}, self.layer, self.sh_degree,
                           self.trainable, self.rctx.activity)

    def prune_now(self):
        n = self.n
        if self.rctx.activity is None or self.rctx.activity.numel() != n:
            self.rctx.reset_accumulators(n, self.device)
        keep, counts = self.prune.decide(self.rctx.activity, self.rctx.max_contrib, self.layer, self.trainable)
        counts["before"] = n
        self.compact(keep)
        counts["after"] = self.n
        self.rctx.reset_accumulators(self.n, self.device)
        self.history.append(counts)
        return counts

    def compact(self, keep):
        """Remove Gaussians (params and Adam moments) where keep is False."""
        idx = torch.nonzero(keep, as_tuple=False).flatten()
        old_state = self.opt.state_dict()
        new_params = {}
        for k in PARAM_KEYS:
            new_params[k] = self.params[k].detach().index_select(-1, idx).contiguous().requires_grad_(True)
        for gi, k in enumerate(PARAM_KEYS):
            st = old_state["state"].get(gi)
            if st is not None:
                for m in ("exp_avg", "exp_avg_sq"):
                    st[m] = st[m].index_select(-1, idx).contiguous()
        self.params = new_params
        self.layer = self.layer.index_select(0, idx).contiguous()
        self.opt = self._make_opt(old_state)
        self.rctx.state = None

    # ---------------------------------------------------------- checkpoint
    def state_dict(self):
        return {"params": {k: v.detach().cpu().numpy() for k, v in self.params.items()},
                "layer": self.layer.cpu().numpy(), "opt": self.opt.state_dict(),
                "prune": {"T": self.prune.T, "steps_in_window": self.prune.steps_in_window,
                          "n_prunes": self.prune.n_prunes},
                "activity": None if self.rctx.activity is None else self.rctx.activity.cpu().numpy(),
                "max_contrib": None if self.rctx.max_contrib is None else self.rctx.max_contrib.cpu().numpy(),
                "rng": self.rng.bit_generator.state, "it": self.it}

    def save(self, path):
        sd = self.state_dict()
        buf = io.BytesIO()
        torch.save(sd["opt"], buf)
        arrays = {f"param_{k}": v for k, v in sd["params"].items()}
        arrays["layer"] = sd["layer"]
        if sd["activity"] is not None:
            arrays["activity"] = sd["activity"]
            arrays["max_contrib"] = sd["max_contrib"]
        arrays["opt"] = np.frombuffer(buf.getvalue(), dtype=np.uint8)
        meta = {"prune": sd["prune"], "rng": sd["rng"], "it": sd["it"], "trainable": self.trainable}
        arrays["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
        np.savez(path, **arrays)

    def export_ply(self, path):
        """The model as one layered PLY (the layer of each Gaussian a vertex
        property, Sec. 3.2; see ply.py)."""
        from . import ply, scenes
        p = {k: v.detach().cpu().numpy() for k, v in self.params.items()}
        sc = scenes._finish(p["mean"], p["log_scale"], p["quat"], p["opacity_logit"], p["sh"],
                            self.layer.cpu().numpy())
        ply.write_ply(path, sc)

    def load(self, path):
        z = np.load(path, allow_pickle=False)
        for k in PARAM_KEYS:
            self.params[k] = torch.tensor(z[f"param_{k}"], device=self.device, requires_grad=True)
        self.layer = torch.tensor(z["layer"], device=self.device)
        opt_state = torch.load(io.BytesIO(z["opt"].tobytes()), weights_only=True, map_location=self.device)
        self.opt = self._make_opt(opt_state)
        meta = json.loads(z["meta"].tobytes().decode())
        self.prune.T = meta["prune"]["T"]
        self.prune.steps_in_window = meta["prune"]["steps_in_window"]
        self.prune.n_prunes = meta["prune"]["n_prunes"]
        self.rng.bit_generator.state = meta["rng"]
        self.it = meta["it"]
        self.rctx.state = None
        if "activity" in z:
            self.rctx.activity = torch.tensor(z["activity"], device=self.device)
            self.rctx.max_contrib = torch.tensor(z["max_contrib"], device=self.device)
        else:
            self.rctx.activity = self.rctx.max_contrib = None
