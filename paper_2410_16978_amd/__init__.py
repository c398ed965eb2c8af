"""Layered Gaussian-splat tile rasterizer for MI355X (gfx950).

The rasterizer itself lives in the HIP library built from csrc/ and is
reached through the C ABI declared in include/gsr.h; `rasterizer` holds the
thin Python binding, `autograd` the torch.autograd.Function around it,
`serve` the continuous-batching render server and `train` the layered
training loop with inactive-Gaussian pruning.  `scenes` draws the seeded
synthetic inputs.  Importing the package loads nothing native.
"""
__all__ = ["scenes"]
