"""torch.autograd.Function over the rasterizer and a fused Adam optimizer.

Both delegate every computation to libfastergs (HIP); torch only allocates.
"""
from __future__ import annotations

from typing import Dict, Optional

import torch

from . import binding as B

_ORDER = B.PARAM_NAMES  # means, log_scales, quats, opacity_logits, sh_dc, sh_rest


class RasterizeGaussians(torch.autograd.Function):
    """image, t_final, last = RasterizeGaussians.apply(means, log_scales, quats,
    opacity_logits, sh_dc, sh_rest, rasterizer).  t_final and last are not
    differentiable.  The backward pass needs the rasterizer's workspace as the
    forward left it, so keep one Rasterizer per in-flight graph."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh_dc, sh_rest, rasterizer: B.Rasterizer):
        params = dict(zip(_ORDER, (means, log_scales, quats, opacity_logits, sh_dc, sh_rest)))
        params = {k: v.detach().contiguous() for k, v in params.items()}
        image, t_final, last = rasterizer.forward(params)
        ctx.rasterizer = rasterizer
        ctx.save_for_backward(*[params[k] for k in _ORDER], image, last)
        ctx.mark_non_differentiable(t_final, last)
        return image, t_final, last

    @staticmethod
    def backward(ctx, d_image, d_t_final, d_last):
        *ps, image, last = ctx.saved_tensors
        params = dict(zip(_ORDER, ps))
        grads = ctx.rasterizer.backward(params, image, last, d_image.contiguous())
        return (*[grads[k] for k in _ORDER], None)


def rasterize(params: Dict[str, torch.Tensor], rasterizer: B.Rasterizer):
    return RasterizeGaussians.apply(*[params[k] for k in _ORDER], rasterizer)


class FusedAdam:
    """Adam over the six Gaussian parameter groups in one kernel launch
    (beta1 = 0.9, beta2 = 0.999, eps = 1e-15 by default).  Moments are float32
    tensors owned by this object; step(grads) updates params in place.
    Rasterizer.backward_adam(params, ..., optimizer) instead fuses the step
    into the backward pass (no gradient tensors)."""

    def __init__(self, params: Dict[str, torch.Tensor], lrs: Dict[str, float], betas=(0.9, 0.999),
                 eps: float = 1e-15, device_step: bool = False):
        self.params = params
        self.lrs = dict(lrs)
        self.betas = betas
        self.eps = eps
        # device_step: the step counter lives on the device (fgs_adam_step_device),
        # so a step captured into a graph advances it on every replay
        self.device_step = device_step
        dev = next(iter(params.values())).device
        self.state = torch.zeros(32, dtype=torch.int64, device=dev) if device_step else None
        # float32 moments also for bfloat16 parameters
        self.exp_avg = {k: torch.zeros_like(v, dtype=torch.float32) for k, v in params.items()}
        self.exp_avg_sq = {k: torch.zeros_like(v, dtype=torch.float32) for k, v in params.items()}
        self.t = 0

    def step(self, grads: Dict[str, torch.Tensor], stream=None) -> None:
        self.t += 1
        groups = [(self.params[k], grads[k], self.exp_avg[k], self.exp_avg_sq[k], self.lrs[k])
                  for k in self.params if k in self.lrs]
        if self.device_step:
            B.adam_step_device(groups, self.state, self.betas[0], self.betas[1], self.eps, stream=stream)
        else:
            B.adam_step(groups, self.t, self.betas[0], self.betas[1], self.eps, stream=stream)

    def state_dict(self) -> Dict[str, object]:
        return {"t": self.t, "exp_avg": self.exp_avg, "exp_avg_sq": self.exp_avg_sq, "lrs": self.lrs}

    def load_state_dict(self, sd: Dict[str, object]) -> None:
        self.t = int(sd["t"])
        for k in self.exp_avg:
            self.exp_avg[k].copy_(sd["exp_avg"][k])
            self.exp_avg_sq[k].copy_(sd["exp_avg_sq"][k])
        self.lrs = dict(sd["lrs"])


def train_step(params: Dict[str, torch.Tensor], rasterizer: B.Rasterizer, target: torch.Tensor,
               optimizer: FusedAdam, dl_dimage: Optional[torch.Tensor] = None,
               loss_out: Optional[torch.Tensor] = None, fused: bool = False) -> Dict[str, torch.Tensor]:
    """One training step without autograd bookkeeping: forward, L1 gradient,
    backward, Adam.  Returns the rendered image and (unless fused, where the
    Adam step runs inside the backward pass) the gradients."""
    image, t_final, last = rasterizer.forward(params)
    if dl_dimage is None:
        dl_dimage = torch.empty_like(image)
    B.l1_loss_backward(image, target, dl_dimage, loss_out)
    grads = None
    if fused:
        rasterizer.backward_adam(params, image, last, dl_dimage, optimizer)
    else:
        grads = rasterizer.backward(params, image, last, dl_dimage)
        optimizer.step(grads)
    return {"image": image, "t_final": t_final, "last": last, "grads": grads, "dl_dimage": dl_dimage}
