"""Adam in float64 (test infrastructure only; see ``oracle/__init__.py``).

Follows Adam (Kingma and Ba) as used by the paper: App. A gives
beta1 = 0.9, beta2 = 0.999, eps = 1e-15; Sec. 3.3 "Parameter Updates" requires
matching PyTorch's Adam (no weight decay, no amsgrad, bias correction with the
step counter t starting at 1), and "Fusing Backward and Optimizer" requires
updating every parameter, including those whose gradient is zero.
"""
from __future__ import annotations

import torch


def adam64(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
           step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
           eps: float = 1e-15):
    """One Adam step in float64.  Returns (new_param, new_m, new_v)."""
    p = param.to(torch.float64)
    g = grad.to(torch.float64)
    m = beta1 * m.to(torch.float64) + (1.0 - beta1) * g
    v = beta2 * v.to(torch.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return p - lr * m_hat / (torch.sqrt(v_hat) + eps), m, v
