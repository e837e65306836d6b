"""Conditional 4D Gaussians in float64 (test infrastructure only; see
``oracle/__init__.py``).

Sec. 3.4 ("Extension to Dynamic Scenes") renders 4D Gaussians at a timestep t
by conditioning each one on t: a 4D Gaussian has a 4D mean (x, y, z and a
time coordinate), a 4D scale (three spatial log-scales and a temporal one)
and a 4D rotation split into a left-isoclinic and a right-isoclinic part, one
quaternion each.  Its covariance is Sigma = R diag(s^2) R^T (as in Sec. 2.1),
and at time t it contributes the conditional 3D Gaussian

    mean_3D|t = mu_xyz + Sigma_xyz,t (t - mu_t) / Sigma_t,t
    cov_3D|t  = Sigma_xyz,xyz - Sigma_xyz,t Sigma_t,xyz / Sigma_t,t

whose alpha (Eq. (3)) is multiplied by the marginal p(t).  Readings adopted
where the paper is silent:

* Coordinates and rotation: the 4-vector (x, y, z, t) is the quaternion
  t + x i + y j + z k, and the 4D rotation maps v to q_l v q_r (Hamilton
  products) with the normalised left and right quaternions, both stored
  (w, x, y, z) like the 3D rotation.  With q_r the conjugate of q_l it is the
  3D rotation R(q_l) of the spatial part and leaves t alone, so a 4D Gaussian
  with that rotation is a static 3D Gaussian whose opacity fades with p(t).
* The marginal enters as exp(-(t - mu_t)^2 / (2 Sigma_t,t)), the Gaussian's
  value relative to its peak: a time-dependent opacity factor in [0, 1].  The
  normalised density would exceed 1 for Sigma_t,t < 1/(2 pi), and its excess
  would only be cut by the alpha cap.
* The degenerate-Gaussian guard of App. B.1 applies to both quaternions.

The functions are plain torch float64 and differentiable, so the oracle's
gradients of the raw 4D parameters come from autograd.
"""
from __future__ import annotations

from typing import Dict, Tuple

import torch

F64 = torch.float64


def hamilton(p: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
    """Quaternion product p q for [..., 4] tensors (w, x, y, z)."""
    p0, p1, p2, p3 = p.unbind(-1)
    q0, q1, q2, q3 = q.unbind(-1)
    return torch.stack([p0 * q0 - p1 * q1 - p2 * q2 - p3 * q3,
                        p0 * q1 + p1 * q0 + p2 * q3 - p3 * q2,
                        p0 * q2 - p1 * q3 + p2 * q0 + p3 * q1,
                        p0 * q3 + p1 * q2 - p2 * q1 + p3 * q0], dim=-1)


def rotation4(ql: torch.Tensor, qr: torch.Tensor) -> torch.Tensor:
    """[N, 4, 4] matrix of v -> ql v qr in coordinates (x, y, z, t) for unit
    quaternions ql, qr [N, 4]: column k is the image of the k-th basis vector
    (x = i, y = j, z = k, t = 1)."""
    n = ql.shape[0]
    basis = torch.tensor([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 1.0],
                          [1.0, 0.0, 0.0, 0.0]], dtype=F64)  # quaternions of x, y, z, t
    cols = []
    for k in range(4):
        e = basis[k].expand(n, 4)
        img = hamilton(hamilton(ql, e), qr)                 # (w, x, y, z) = (t, x, y, z)
        cols.append(torch.stack([img[:, 1], img[:, 2], img[:, 3], img[:, 0]], dim=-1))
    return torch.stack(cols, dim=-1)


def covariance4(log_scales4: torch.Tensor, ql: torch.Tensor, qr: torch.Tensor) -> torch.Tensor:
    """Sigma = R diag(s^2) R^T [N, 4, 4] from log-scales [N, 4] (x, y, z, t) and
    the raw quaternions [N, 4] (normalised here)."""
    qln = ql / torch.linalg.vector_norm(ql, dim=-1, keepdim=True)
    qrn = qr / torch.linalg.vector_norm(qr, dim=-1, keepdim=True)
    R = rotation4(qln, qrn)
    M = R * torch.exp(log_scales4)[:, None, :]
    return M @ M.transpose(-1, -2)


def condition(mean4: torch.Tensor, log_scales4: torch.Tensor, ql: torch.Tensor, qr: torch.Tensor,
              t: float) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """The conditional 3D Gaussian at time t and the marginal factor:
    (mean [N, 3], covariance [N, 3, 3], p(t) [N])."""
    S = covariance4(log_scales4, ql, qr)
    A, b, c = S[:, :3, :3], S[:, :3, 3], S[:, 3, 3]
    dt = t - mean4[:, 3]
    mean3 = mean4[:, :3] + b * (dt / c)[:, None]
    cov3 = A - b[:, :, None] * b[:, None, :] / c[:, None, None]
    p = torch.exp(-0.5 * dt * dt / c)
    return mean3, cov3, p


def rows4(rows: Dict[str, torch.Tensor]) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor, torch.Tensor]:
    """The 4D parameters from preprocess rows: mean4 [N, 4], log_scales4 [N, 4],
    ql [N, 4], qr [N, 4]."""
    mean4 = torch.cat([rows["means"], rows["mean_t"][:, None]], dim=1)
    ls4 = torch.cat([rows["log_scales"], rows["log_scale_t"][:, None]], dim=1)
    return mean4, ls4, rows["quats"], rows["quats_r"]


__all__ = ["hamilton", "rotation4", "covariance4", "condition", "rows4"]
