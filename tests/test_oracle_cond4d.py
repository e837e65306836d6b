"""Pins of the conditional 4D Gaussian oracle (``oracle/cond4d64.py``; Sec. 3.4
"Extension to Dynamic Scenes").

* The 4D rotation of two unit quaternions is orthogonal with determinant +1.
* With the right quaternion the conjugate of the left one it is the 3D
  rotation of the left quaternion on (x, y, z) and leaves t alone (the
  classical correspondence q v q* of 3D rotations).
* A rotation by theta in the (x, t) plane has a closed-form conditional
  Gaussian: Sigma_xt = sin cos (s_t^2 - s_x^2), Sigma_tt = sin^2 s_x^2 +
  cos^2 s_t^2, conditional variance s_x^2 s_t^2 / Sigma_tt (the determinant
  of the 2x2 block over Sigma_tt), mean moving with slope Sigma_xt / Sigma_tt.
* A 4D scene whose rotations leave t alone renders like the 3D scene whose
  opacities are multiplied by exp(-(t - mu_t)^2 / (2 s_t^2)).
* Autograd through the conditioning matches central finite differences on a
  tiny scene for every raw 4D parameter.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from oracle import cond4d64 as C
from oracle.render64 import DEFAULT_SETTINGS as ST

F64 = torch.float64


def rand_quats(n, seed):
    g = torch.Generator().manual_seed(seed)
    q = torch.randn(n, 4, generator=g, dtype=F64)
    return q / q.norm(dim=1, keepdim=True)


def test_rotation4_is_a_proper_rotation():
    ql, qr = rand_quats(64, 1), rand_quats(64, 2)
    R = C.rotation4(ql, qr)
    eye = torch.eye(4, dtype=F64).expand(64, 4, 4)
    assert float((R @ R.transpose(1, 2) - eye).abs().max()) <= 1e-14
    assert float((torch.linalg.det(R) - 1.0).abs().max()) <= 1e-13


def test_conjugate_pair_is_the_3d_rotation():
    q = rand_quats(32, 3)
    qc = q * torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=F64)
    R = C.rotation4(q, qc)
    R3 = O.quat_to_rotation64(q)
    assert float((R[:, :3, :3] - R3).abs().max()) <= 1e-14
    assert float(R[:, 3, :3].abs().max()) <= 1e-15 and float(R[:, :3, 3].abs().max()) <= 1e-15
    assert float((R[:, 3, 3] - 1.0).abs().max()) <= 1e-15


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, -0.7, math.pi / 2])
def test_xt_plane_rotation_closed_form(theta):
    q = torch.tensor([[math.cos(theta / 2), math.sin(theta / 2), 0.0, 0.0]], dtype=F64)
    sx, sy, sz, st = 0.3, 0.2, 0.25, 0.7
    ls4 = torch.log(torch.tensor([[sx, sy, sz, st]], dtype=F64))
    mean4 = torch.tensor([[0.1, -0.2, 3.0, 0.4]], dtype=F64)
    c, s = math.cos(theta), math.sin(theta)
    s_xt = s * c * (st * st - sx * sx)
    s_tt = s * s * sx * sx + c * c * st * st
    for t in (-0.5, 0.0, 0.4, 1.3):
        mean3, cov3, p = C.condition(mean4, ls4, q, q, t)
        assert abs(float(mean3[0, 0]) - (0.1 + s_xt / s_tt * (t - 0.4))) <= 1e-14
        assert abs(float(mean3[0, 1]) + 0.2) <= 1e-15 and abs(float(mean3[0, 2]) - 3.0) <= 1e-15
        assert abs(float(cov3[0, 0, 0]) - sx * sx * st * st / s_tt) <= 1e-14
        assert abs(float(cov3[0, 1, 1]) - sy * sy) <= 1e-15 and abs(float(cov3[0, 2, 2]) - sz * sz) <= 1e-15
        assert float(cov3[0, 0, 1:].abs().max()) <= 1e-15
        assert abs(float(p[0]) - math.exp(-0.5 * (t - 0.4) ** 2 / s_tt)) <= 1e-15


def scene4(n, seed, static=False):
    """Tiny 4D scene in front of an identity camera; static: right quaternion =
    conjugate of the left (time unmixed)."""
    g = torch.Generator().manual_seed(seed)
    sc = {
        "means": torch.stack([torch.rand(n, generator=g) * 1.0 - 0.5, torch.rand(n, generator=g) * 1.0 - 0.5,
                              torch.rand(n, generator=g) * 1.5 + 2.0]),
        "log_scales": torch.randn(3, n, generator=g) * 0.3 - 1.6,
        "quats": torch.randn(4, n, generator=g),
        "opacity_logits": torch.randn(n, generator=g) * 0.8,
        "sh_dc": torch.randn(3, n, generator=g) * 0.4,
        "sh_rest": torch.randn(45, n, generator=g) * 0.1,
        "mean_t": torch.rand(n, generator=g),
        "log_scale_t": torch.randn(n, generator=g) * 0.3 - 0.5,
        "quats_r": torch.randn(4, n, generator=g),
    }
    if static:
        sc["quats_r"] = sc["quats"] * torch.tensor([1.0, -1.0, -1.0, -1.0])[:, None]
    return {k: v.to(torch.float32).contiguous() for k, v in sc.items()}


def test_static_rotation_renders_like_3d_with_faded_opacity():
    n, t = 6, 0.35
    cam = S.identity_camera(40, 32, 45.0, bg=(0.1, 0.2, 0.3))
    sc = scene4(n, 5, static=True)
    r4 = O.render64(sc, cam, time=t, cull=False)
    s_t = torch.exp(sc["log_scale_t"].double())
    p = torch.exp(-0.5 * (t - sc["mean_t"].double()) ** 2 / (s_t * s_t))
    o = torch.sigmoid(sc["opacity_logits"].double()) * p
    # float64 scene of the 3D model: the opacity logit of o p(t)
    sc3 = {k: v.double() for k, v in sc.items() if k not in ("mean_t", "log_scale_t", "quats_r")}
    sc3["opacity_logits"] = torch.log(o / (1.0 - o))
    r3 = O.render64(sc3, cam, cull=False, order_keys=O.depth_key32(sc["means"], cam))
    assert float((r4["image"] - r3["image"]).abs().max()) <= 1e-12
    assert float((r4["t_final"] - r3["t_final"]).abs().max()) <= 1e-12


def _loss4(base, cam, gup, t):
    r = O.render64({k: v.clone() for k, v in base.items()}, cam, time=t, cull=False,
                   order_keys=np.arange(base["mean_t"].numel(), dtype=np.float32))
    return float((r["image"] * gup).sum()), bool(r["borderline"].any())


@pytest.mark.parametrize("seed", [0, 1])
def test_autograd_matches_central_finite_differences(seed):
    n, t = 3, 0.45
    cam = S.identity_camera(24, 20, 30.0, bg=(0.25, 0.5, 0.75))
    sc = scene4(n, 200 + seed)
    gup = S.make_dl_dimage(20, 24, seed=seed).to(F64)
    keys = np.arange(n, dtype=np.float32)  # a fixed order: the decisions of the depth sort are not differentiated
    r = O.render64(sc, cam, time=t, dl_dimage=gup, cull=False, order_keys=keys)
    assert not bool(r["borderline"].any())
    base = {k: v.to(F64).clone() for k, v in sc.items()}
    checked = 0
    for name, ad in r["grads"].items():
        flat_ad = ad.reshape(-1)
        scale = float(flat_ad.abs().max())
        p = base[name].reshape(-1)
        for j in range(flat_ad.numel()):
            h = 1e-5 * max(1.0, abs(float(p[j])))
            old = float(p[j])
            p[j] = old + h
            Lp, bp = _loss4(base, cam, gup, t)
            p[j] = old - h
            Lm, bm = _loss4(base, cam, gup, t)
            p[j] = old
            if bp or bm:
                continue
            fd = (Lp - Lm) / (2 * h)
            noise = 4 * np.finfo(np.float64).eps * (abs(Lp) + abs(Lm)) / (2 * h)
            tol = 1e-6 * max(abs(float(flat_ad[j])), 1e-3 * scale) + noise
            assert abs(fd - float(flat_ad[j])) <= tol, (name, j, fd, float(flat_ad[j]), tol)
            checked += 1
    assert set(r["grads"]) >= {"mean_t", "log_scale_t", "quats_r"}
    assert checked >= 65 * n - 4


def test_projection_form_equals_the_schur_complement():
    """The conditional covariance as the Gram matrix of the spatial rows of
    M = R diag(s) projected off the unit time row u (N = M_xyz (I - u u^T),
    Sigma_3|t = N N^T), the mean shift (M_xyz u) (t - mu_t) / |m_t| and the
    factor exp(-((t - mu_t) / |m_t|)^2 / 2) equal the Schur-complement
    definition: I - u u^T is idempotent, so N N^T = A - b b^T / c."""
    n = 48
    g = torch.Generator().manual_seed(11)
    ql, qr = rand_quats(n, 12), rand_quats(n, 13)
    ls4 = torch.randn(n, 4, generator=g, dtype=F64) * 0.8 - 1.0
    mean4 = torch.randn(n, 4, generator=g, dtype=F64)
    t = 0.3
    mean3, cov3, p = C.condition(mean4, ls4, ql, qr, t)
    M = C.rotation4(ql, qr) * torch.exp(ls4)[:, None, :]
    m = M[:, 3, :]
    norm = torch.linalg.vector_norm(m, dim=1)
    u = m / norm[:, None]
    along = (M[:, :3, :] * u[:, None, :]).sum(-1)
    N = M[:, :3, :] - along[:, :, None] * u[:, None, :]
    e = (t - mean4[:, 3]) / norm
    scale = cov3.abs().amax(dim=(1, 2)) + (M[:, :3, :] ** 2).sum(-1).amax(-1)
    assert float(((N @ N.transpose(1, 2) - cov3).abs().amax(dim=(1, 2)) / scale).max()) <= 1e-13
    assert float((mean4[:, :3] + along * e[:, None] - mean3).abs().max()) <= 1e-12
    assert float((torch.exp(-0.5 * e * e) - p).abs().max()) <= 1e-14
