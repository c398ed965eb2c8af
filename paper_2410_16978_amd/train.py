"""Layered training with inactive-Gaussian pruning (Sec. 3.2).

Layers are trained consecutively: the Gaussians of earlier layers stay in
the scene and are rendered as background but receive no gradient (the
kernel zeroes them through `trainable_layers`), so the optimiser leaves
them untouched.  Every step renders a batch of views with a random
background colour and compares RGB and alpha with the target (alpha-channel
training, Sec. 3.2.1).

Inactive pruning (Sec. 3.2.2): per trainable Gaussian the activity
2 p + 0.1 c + 0.1 s (position, colour and scale norms) is averaged over each
densification window of dR = 100 steps and compared with a threshold T
(T0 = 0.015): Gaussians at or below it are removed, then T decays by 0.975.
Which norms are meant is a reading; two are built:

* "update" (default): the norms of the change each optimiser step made to
  the Gaussian's mean, SH coefficients and log-scales (gsr_update_activity).
  A Gaussian the optimiser never moves scores exactly 0.
* "gradient": the norms of the per-step gradients (fused into the backward
  kernel), multiplied by views_per_step so that a step over V views, whose
  loss is the mean over them, scores like a step over one view.

T0 was tuned on the paper's data; the counts of every pruning step include
quantiles of the trainable Gaussians' averages so a threshold can be set for
other data.

Optionally, Gaussians whose largest alpha * T over the window stayed below
1/255 (they never visibly contributed) are removed as well; both criteria are
counted separately.

Adaptive density control (optional, DensifyConfig): the density control of
the Gaussian-splatting optimisation the paper trains with (Sec. 4.3: its
default settings or the HQ settings), on the trainable layers only.  The
backward kernel accumulates, per Gaussian and view in which it is visible,
the length of the loss gradient with respect to its projected centre in
normalised device coordinates; every interval, Gaussians whose mean of that
statistic reaches the threshold are cloned (small ones: largest scale at
most percent_dense times the scene extent) or split into n_split children
drawn from the Gaussian itself with scales divided by 0.8 n_split (large
ones); then Gaussians below the minimum opacity, and after the first opacity
reset those larger than max_world_size times the extent, are removed.  The
opacities are capped at reset_opacity every opacity_reset_interval steps.
Children and clones join the Gaussian's layer and start with zero Adam
moments.
"""
from __future__ import annotations

import dataclasses
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
    measure: str = "update"    # "update": norms of the optimiser's steps; "gradient": norms of the gradients


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
        if self.cfg.measure not in ("update", "gradient"):
            raise ValueError(f"unknown activity measure {self.cfg.measure!r}")
        avg = activity_sum / max(self.steps_in_window, 1)  # the window's average activity
        trainable = ((int(trainable_layers) >> layer.to(torch.int64)) & 1).bool()
        inactive = trainable & (avg <= self.T)
        invisible = trainable & (max_contrib < self.cfg.min_contrib) if self.cfg.use_max_contrib else \
            torch.zeros_like(inactive)
        keep = ~((inactive if self.cfg.use_activity else torch.zeros_like(inactive)) | invisible)
        counts = {"activity": int(inactive.sum()), "max_contrib": int(invisible.sum()),
                  "both": int((inactive & invisible).sum()), "pruned": int((~keep).sum()), "threshold": self.T}
        if bool(trainable.any()):
            qs = torch.quantile(avg[trainable].double().cpu(), torch.tensor([0.1, 0.5, 0.9, 0.99], dtype=torch.float64))
            counts["avg_quantiles"] = [float(x) for x in qs] + [float(avg[trainable].max())]
        self.T *= self.cfg.decay
        self.n_prunes += 1
        self.steps_in_window = 0
        return keep, counts


@dataclasses.dataclass
class DensifyConfig:
    """Adaptive density control (defaults: the Gaussian-splatting defaults the
    paper starts from; DensifyConfig.hq(): its HQ settings, Sec. 4.3)."""
    interval: int = 100
    start: int = 500
    until: int = 15_000
    grad_threshold: float = 2e-4
    percent_dense: float = 0.01
    min_opacity: float = 0.005
    max_world_size: float = 0.1
    opacity_reset_interval: int = 3000
    reset_opacity: float = 0.01
    n_split: int = 2

    @classmethod
    def hq(cls, **kw):
        kw.setdefault("grad_threshold", 1e-4)
        kw.setdefault("percent_dense", 0.005)
        return cls(**kw)


def trainable_mask(layer, trainable_layers):
    return ((int(trainable_layers) >> layer.to(torch.int64)) & 1).bool()


def densify_masks(grad_sum, count, log_scale, layer, trainable_layers, cfg, extent, views_per_step):
    """(clone, split) bool masks.  The statistic's mean over the views that saw
    the Gaussian, times views_per_step: a step's loss is the mean over its
    views, so each view's gradient is 1/views_per_step of that of its own
    mean loss."""
    live = trainable_mask(layer, trainable_layers)
    avg = grad_sum / torch.clamp(count, min=1.0) * float(views_per_step)
    cand = live & (count > 0) & (avg >= cfg.grad_threshold)
    smax = torch.exp(log_scale).amax(dim=0)
    small = smax <= cfg.percent_dense * extent
    return cand & small, cand & ~small


def split_children(mean, log_scale, quat, z, n_split):
    """Means and log-scales of the children of split Gaussians: child k of
    Gaussian i sits at mean_i + R(q_i) (s_i * z[k, :, i]) (a sample of the
    Gaussian itself for z ~ N(0, I)) with scale s_i / (0.8 n_split).
    mean, log_scale [3, m], quat [4, m] (w, x, y, z), z [n_split, 3, m].
    Returns (mean [3, n_split m], log_scale [3, n_split m]): the m first
    children, then the m second children, and so on."""
    q = quat / torch.linalg.vector_norm(quat, dim=0, keepdim=True)
    w, x, y, zq = q[0], q[1], q[2], q[3]
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y)]),
        torch.stack([2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x)]),
        torch.stack([2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)]),
    ])  # [3, 3, m]
    s = torch.exp(log_scale)
    means, scales = [], []
    for k in range(n_split):
        local = s * z[k]                                   # [3, m]
        means.append(mean + (R * local.unsqueeze(0)).sum(dim=1))
        scales.append(log_scale - float(np.log(0.8 * n_split)))
    return torch.cat(means, dim=1), torch.cat(scales, dim=1)


def camera_extent(cams):
    """Scene extent for density control: 1.1 times the largest distance of a
    camera centre from the centres' mean (1 for a single camera)."""
    cs = []
    for c in cams:
        R = np.asarray(c["R"], np.float64).reshape(3, 3)
        cs.append(-R.T @ np.asarray(c["t"], np.float64))
    cs = np.asarray(cs)
    d = np.linalg.norm(cs - cs.mean(0), axis=1).max() if len(cs) > 1 else 0.0
    return float(1.1 * d) if d > 0 else 1.0


class FusedAdam:
    """Adam (gsr_adam_step) over the parameter groups of a layered model:
    one kernel launch per step that skips the frozen layers' Gaussians and,
    given an activity buffer, adds the update-norm activity of the step.
    Moments are tensors shaped like the parameters; `t` counts the steps."""

    def __init__(self, params, lrs, betas=(0.9, 0.999), eps=1e-15):
        self.lrs = dict(lrs)
        self.betas = tuple(betas)
        self.eps = float(eps)
        self.t = 0
        self.m = {k: torch.zeros_like(params[k].detach()) for k in PARAM_KEYS}
        self.v = {k: torch.zeros_like(params[k].detach()) for k in PARAM_KEYS}

    def step(self, params, layer, sh_degree, trainable, activity=None):
        self.t += 1
        grads = {k: params[k].grad if params[k].grad is not None else torch.zeros_like(params[k].detach())
                 for k in PARAM_KEYS}
        rz.adam_step({k: params[k].detach() for k in PARAM_KEYS}, {k: g.contiguous() for k, g in grads.items()},
                     self.m, self.v, self.lrs, layer, sh_degree, trainable, self.t, self.betas, self.eps,
                     activity=activity)

    def remap(self, idx, m_new):
        """Keep the moments of Gaussians idx, then m_new zero columns."""
        for st in (self.m, self.v):
            for k in PARAM_KEYS:
                t = st[k].index_select(-1, idx)
                if m_new:
                    t = torch.cat([t, torch.zeros(t.shape[:-1] + (m_new,), dtype=t.dtype, device=t.device)], dim=-1)
                st[k] = t.contiguous()

    def arrays(self):
        out = {f"adam_m_{k}": v.cpu().numpy() for k, v in self.m.items()}
        out.update({f"adam_v_{k}": v.cpu().numpy() for k, v in self.v.items()})
        return out

    def load_arrays(self, z, t, device):
        self.t = int(t)
        self.m = {k: torch.tensor(z[f"adam_m_{k}"], device=device) for k in PARAM_KEYS}
        self.v = {k: torch.tensor(z[f"adam_v_{k}"], device=device) for k in PARAM_KEYS}


class LayeredTrainer:
    """Adam on the trainable layers of a layered Gaussian scene."""

    def __init__(self, scene, cams, targets, trainable_layers, views_per_step=1, lrs=None, prune=None,
                 seed=0, device="cuda", sync=True, densify=None, extent=None):
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
        self.densify = densify                        # DensifyConfig or None
        self.extent = camera_extent(cams) if extent is None else float(extent)
        self.dens = None                              # (grad_sum, count) accumulators
        if densify is not None:
            self._reset_densify_stats()
        self.rng = np.random.default_rng(seed)
        self.it = 0
        self.history = []

    def _make_opt(self):
        return FusedAdam(self.params, self.lrs)

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
        for k in PARAM_KEYS:
            self.params[k].grad = None
        loss.backward()
        act = self.rctx.activity if self.prune.cfg.measure == "update" else None
        self.opt.step(self.params, self.layer, self.sh_degree, self.trainable, activity=act)
        self.it += 1
        self.prune.steps_in_window += 1
        out = {"it": self.it, "loss": loss}
        if self.prune.due():
            out["prune"] = self.prune_now()
        d = self.densify
        if d is not None:
            if d.start <= self.it < d.until and self.it % d.interval == 0:
                out["densify"] = self.densify_now()
            if self.it % d.opacity_reset_interval == 0 and self.it < d.until:
                self.reset_opacity()
        return out

    # ---------------------------------------------------------- density control
    def _reset_densify_stats(self):
        n = self.n
        self.dens = (torch.zeros(n, dtype=torch.float32, device=self.device),
                     torch.zeros(n, dtype=torch.float32, device=self.device))
        self.rctx.densify_stats = self.dens

    def densify_now(self):
        """Clone, split, then prune by opacity (and size after the first
        opacity reset); returns the counts."""
        d = self.densify
        p = {k: v.detach() for k, v in self.params.items()}
        clone, split = densify_masks(self.dens[0], self.dens[1], p["log_scale"], self.layer, self.trainable, d,
                                     self.extent, self.views_per_step)
        ci = torch.nonzero(clone, as_tuple=False).flatten()
        si = torch.nonzero(split, as_tuple=False).flatten()
        n_before = self.n
        # children: all the originals' values, then the sampled means and scales
        gen = torch.Generator(device=self.device)
        gen.manual_seed(int(self.rng.integers(0, 2 ** 62)))
        z = torch.randn((d.n_split, 3, int(si.numel())), generator=gen, device=self.device)
        cm, cls_ = split_children(p["mean"][:, si], p["log_scale"][:, si], p["quat"][:, si], z, d.n_split)
        rep = si.repeat(d.n_split)
        extra = {k: torch.cat([p[k].index_select(-1, ci), p[k].index_select(-1, rep)], dim=-1) for k in PARAM_KEYS}
        extra["mean"][:, ci.numel():] = cm
        extra["log_scale"][:, ci.numel():] = cls_
        extra_layer = torch.cat([self.layer[ci], self.layer[rep]])
        keep = torch.ones(n_before, dtype=torch.bool, device=self.device)
        keep[si] = False
        self._rebuild(torch.nonzero(keep, as_tuple=False).flatten(), extra, extra_layer)
        # prune: too transparent, or (after the first opacity reset) too large
        live = trainable_mask(self.layer, self.trainable)
        op = torch.sigmoid(self.params["opacity_logit"].detach())
        bad = op < d.min_opacity
        if self.it > d.opacity_reset_interval:
            bad |= torch.exp(self.params["log_scale"].detach()).amax(dim=0) > d.max_world_size * self.extent
        bad &= live
        n_mid = self.n
        self._rebuild(torch.nonzero(~bad, as_tuple=False).flatten())
        self._reset_densify_stats()
        counts = {"it": self.it, "before": n_before, "cloned": int(ci.numel()), "split": int(si.numel()),
                  "pruned": int(n_mid - self.n), "after": self.n}
        self.history.append({"densify": counts})
        return counts

    def reset_opacity(self):
        """Cap the trainable Gaussians' opacities at reset_opacity and clear
        their Adam moments."""
        live = trainable_mask(self.layer, self.trainable)
        cap = float(np.log(self.densify.reset_opacity / (1.0 - self.densify.reset_opacity)))
        with torch.no_grad():
            lo = self.params["opacity_logit"]
            lo.copy_(torch.where(live, torch.clamp(lo, max=cap), lo))
        for st in (self.opt.m, self.opt.v):
            st["opacity_logit"][live] = 0.0

    def prune_now(self):
        n = self.n
        if self.rctx.activity is None or self.rctx.activity.numel() != n:
            self.rctx.reset_accumulators(n, self.device)
        act = self.rctx.activity
        if self.prune.cfg.measure == "gradient":
            act = act * float(self.views_per_step)
        keep, counts = self.prune.decide(act, self.rctx.max_contrib, self.layer, self.trainable)
        counts["before"] = n
        self.compact(keep)
        counts["after"] = self.n
        self.rctx.reset_accumulators(self.n, self.device)
        self.history.append(counts)
        return counts

    def compact(self, keep):
        """Remove Gaussians (params and Adam moments) where keep is False."""
        self._rebuild(torch.nonzero(keep, as_tuple=False).flatten())

    def _rebuild(self, idx, extra=None, extra_layer=None):
        """Keep the Gaussians idx (in that order), then append `extra`
        (parameters of new Gaussians, zero Adam moments).  Per-Gaussian
        accumulators follow (new Gaussians start at zero)."""
        m_new = 0 if extra is None else int(extra_layer.numel())
        new_params = {}
        for k in PARAM_KEYS:
            t = self.params[k].detach().index_select(-1, idx)
            if m_new:
                t = torch.cat([t, extra[k].to(t.dtype)], dim=-1)
            new_params[k] = t.contiguous().requires_grad_(True)
        self.opt.remap(idx, m_new)
        self.params = new_params
        lay = self.layer.index_select(0, idx)
        self.layer = (torch.cat([lay, extra_layer]) if m_new else lay).contiguous()
        self.rctx.state = None

        def remap(t):
            u = t.index_select(0, idx)
            return torch.cat([u, torch.zeros(m_new, dtype=u.dtype, device=u.device)]) if m_new else u.contiguous()

        if self.rctx.activity is not None and self.rctx.max_contrib is not None:
            self.rctx.activity = remap(self.rctx.activity)
            self.rctx.max_contrib = remap(self.rctx.max_contrib)
        if self.dens is not None:
            self.dens = (remap(self.dens[0]), remap(self.dens[1]))
            self.rctx.densify_stats = self.dens

    # ---------------------------------------------------------- checkpoint
    def state_dict(self):
        return {"params": {k: v.detach().cpu().numpy() for k, v in self.params.items()},
                "layer": self.layer.cpu().numpy(), "opt": self.opt.arrays(), "opt_t": self.opt.t,
                "prune": {"T": self.prune.T, "steps_in_window": self.prune.steps_in_window,
                          "n_prunes": self.prune.n_prunes},
                "activity": None if self.rctx.activity is None else self.rctx.activity.cpu().numpy(),
                "max_contrib": None if self.rctx.max_contrib is None else self.rctx.max_contrib.cpu().numpy(),
                "rng": self.rng.bit_generator.state, "it": self.it}

    def save(self, path):
        sd = self.state_dict()
        arrays = {f"param_{k}": v for k, v in sd["params"].items()}
        arrays.update(sd["opt"])
        arrays["layer"] = sd["layer"]
        if sd["activity"] is not None:
            arrays["activity"] = sd["activity"]
            arrays["max_contrib"] = sd["max_contrib"]
        if self.dens is not None:
            arrays["densify_grad"] = self.dens[0].cpu().numpy()
            arrays["densify_count"] = self.dens[1].cpu().numpy()
        meta = {"prune": sd["prune"], "rng": sd["rng"], "it": sd["it"], "trainable": self.trainable,
                "adam_t": sd["opt_t"]}
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
        meta = json.loads(z["meta"].tobytes().decode())
        self.opt = self._make_opt()
        self.opt.load_arrays(z, meta["adam_t"], self.device)
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
        if self.densify is not None:
            if "densify_grad" in z:
                self.dens = (torch.tensor(z["densify_grad"], device=self.device),
                             torch.tensor(z["densify_count"], device=self.device))
                self.rctx.densify_stats = self.dens
            else:
                self._reset_densify_stats()
