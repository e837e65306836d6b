"""FP64 CPU oracle: preprocess, brute-force compositing, autograd gradients.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What is computed, and where the paper defines it (Faster-GS, Hahlbohm et al.):

* Activations (Sec. 2.1, "Activation Functions"): scale = exp(log-scale),
  opacity = sigmoid(logit), the rotation quaternion is normalised, the
  covariance is Sigma = R S S^T R^T, and the view-dependent colour is clipped
  to be non-negative.
* Mean projection, Eq. (1): mu2D = (fx x/z + cx, fy y/z + cy) with
  (x, y, z) = W (mu, 1)^T.
* Covariance projection, Eq. (2): Sigma2D = J W3 Sigma W3^T J^T with the
  affine Jacobian J of the perspective projection (no clamping of x/z, y/z).
* 2D dilation (App. C.2, the original 2D Gaussian filter): Sigma2D + 0.3 I.
* Degenerate-Gaussian guard (App. B.1): not rendered when |q| < 1e-4 or
  det(Sigma2D) < 1e-6 (the un-dilated matrix, as written there).
* Alpha, Eq. (3): alpha = o exp(-1/2 d^T Sigma2D^-1 d), evaluated with the
  dilated matrix, capped at 0.99 (App. B.1) and skipped when below
  tau_alpha = 1/255 (Sec. 3.2, "Splat Bounding").
* Front-to-back blending, Eq. (4), with early termination once the
  transmittance falls below 1e-4 (App. B.1).  Reading used: the fragment is
  blended first and the check follows; the background is weighted by the
  transmittance left after the last blended fragment.
* Degree-3 spherical harmonics (Sec. 2.1): real SH basis, 16 coefficients per
  channel, plus 0.5, clipped at 0.
* Gradients of the six raw parameter tensors: torch autograd in float64 over
  all of the above; the skip, cap and stop decisions are non-differentiable
  masks.

Pixel sample points are (i + 0.5, j + 0.5) in the coordinates of (cx, cy).
Per pixel, every candidate Gaussian is composited in the canonical order
(FP32 depth key, then Gaussian index); no tiles are involved.  For large
scenes candidates may be restricted, per block of pixels, to Gaussians whose
FP64 opacity-aware rectangle (Sec. 3.2), widened by one pixel, reaches the
block: outside that rectangle alpha < tau_alpha holds exactly, so the result
is unchanged (pinned by a test that compares culled and unculled output, and
by a certificate, over the whole 10k-Gaussian frame and the 3M-Gaussian
crops, that every dropped Gaussian stays below tau_alpha in the dropped
block: an eigenvalue bound, else brute force over the block's pixels).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import torch

from . import fp32err as E

F64 = torch.float64


def _f32(x: float) -> float:
    return float(np.float32(x))


@dataclasses.dataclass(frozen=True)
class Settings:
    """Thresholds, each the float32-rounded constant, used in float64."""

    tau_alpha: float = _f32(1.0 / 255.0)   # Sec. 3.2 Splat Bounding
    alpha_max: float = _f32(0.99)          # App. B.1
    t_min: float = _f32(1e-4)              # App. B.1
    dilation: float = _f32(0.3)            # App. C.2, 2D filter variance
    quat_min: float = _f32(1e-4)           # App. B.1
    det_min: float = _f32(1e-6)            # App. B.1
    tile: int = 16                         # Sec. 3.1 (16x16 tiles); unused by the blend


DEFAULT_SETTINGS = Settings()

# Borderline decisions (a threshold test whose float64 value lies within the
# float32 error of the compared quantity) are found with the float32 error
# model of ``fp32err``.


# ----------------------------------------------------------------------------
# Spherical harmonics (Sec. 2.1: degree three, 16 coefficients per channel).
# Real SH with the Condon-Shortley phase, ordered (l, m = -l..l); the
# normalisation constants are written as their closed forms.
# ----------------------------------------------------------------------------
def sh_basis64(d: torch.Tensor) -> torch.Tensor:
    """Real SH basis up to degree 3 at unit directions d [..., 3] -> [..., 16]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pi = math.pi
    k0 = 0.5 * math.sqrt(1.0 / pi)
    k1 = math.sqrt(3.0 / (4.0 * pi))
    k2a = 0.5 * math.sqrt(15.0 / pi)
    k2b = 0.25 * math.sqrt(5.0 / pi)
    k2c = 0.25 * math.sqrt(15.0 / pi)
    k3a = 0.25 * math.sqrt(35.0 / (2.0 * pi))
    k3b = 0.5 * math.sqrt(105.0 / pi)
    k3c = 0.25 * math.sqrt(21.0 / (2.0 * pi))
    k3d = 0.25 * math.sqrt(7.0 / pi)
    k3e = 0.25 * math.sqrt(105.0 / pi)
    xx, yy, zz = x * x, y * y, z * z
    one = torch.ones_like(x)
    return torch.stack([
        k0 * one,
        -k1 * y, k1 * z, -k1 * x,
        k2a * x * y, -k2a * y * z, k2b * (2 * zz - xx - yy), -k2a * x * z, k2c * (xx - yy),
        -k3a * y * (3 * xx - yy), k3b * x * y * z, -k3c * y * (4 * zz - xx - yy),
        k3d * z * (2 * zz - 3 * xx - 3 * yy), -k3c * x * (4 * zz - xx - yy),
        k3e * z * (xx - yy), -k3a * x * (xx - 3 * yy),
    ], dim=-1)


def quat_to_rotation64(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of unit quaternions q = (w, x, y, z) [..., 4] -> [..., 3, 3]."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    rows = [
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ]
    return torch.stack(rows, dim=-2)


def _camera64(cam):
    W = torch.as_tensor(np.asarray(cam.world_to_cam, dtype=np.float32), dtype=F64)
    return W[:3, :3], W[:3, 3]


def camera_center64(cam) -> torch.Tensor:
    W3, t = _camera64(cam)
    return -(W3.T @ t)


def _rows(scene: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
    """SoA float32 tensors [k, N] -> float64 row tensors [N, k] (copies)."""
    out = {}
    for name, v in scene.items():
        v = v.detach().to("cpu")
        out[name] = (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64).clone())
    return out


def preprocess64(p: Dict[str, torch.Tensor], cam, st: Settings = DEFAULT_SETTINGS,
                 sh_degree: int = 3, mca: bool = False, time: Optional[float] = None) -> Dict[str, torch.Tensor]:
    """Per-Gaussian projection in float64 (differentiable w.r.t. the row tensors in p).

    p holds row tensors: means [N,3], log_scales [N,3], quats [N,4],
    opacity_logits [N], sh_dc [N,3], sh_rest [N,45].  Conditional 4D
    Gaussians (Sec. 3.4; ``cond4d64``) also hold mean_t [N], log_scale_t [N]
    and quats_r [N,4] (quats is then the left quaternion); they are rendered
    at ``time`` as their conditional 3D Gaussians, the opacity times the
    marginal factor.
    Returns mean2d [N,2], cov2d [N,2,2] (un-dilated), cov2d_dil, conic [N,3]
    (a, b, c of the inverse dilated matrix [[a, b], [b, c]]), opacity [N],
    rgb [N,3], colour before the clip, camera-space position, the cull mask
    ``valid``, the opacity-aware rectangle half-extents, the borderline flags
    of the culls and the colour clip, and with ``mca`` the float32 deviation
    samples of ``fp32err.mca_deviations`` (key ``dev``).  Rows failing a
    cull test may hold non-finite values; callers select ``valid`` rows.
    """
    q = p["quats"]
    qn = torch.linalg.vector_norm(q, dim=-1)
    four_d = "quats_r" in p
    if four_d:
        if time is None:
            raise ValueError("conditional 4D Gaussians are rendered at a time")
        from .cond4d64 import condition, rows4
        # the guard of App. B.1 on both quaternions: the smaller norm decides
        qn = torch.minimum(qn, torch.linalg.vector_norm(p["quats_r"], dim=-1))
        mu, Sigma, p_t = condition(*rows4(p), float(time))
    else:
        mu = p["means"]
        s = torch.exp(p["log_scales"])
        qh = q / torch.where(qn > 0, qn, torch.ones_like(qn))[:, None]
        R = quat_to_rotation64(qh)
        M = R * s[:, None, :]
        Sigma = M @ M.transpose(-1, -2)

    W3, t = _camera64(cam)
    mh = mu @ W3.T + t
    x, y, z = mh[:, 0], mh[:, 1], mh[:, 2]
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    mean2d = torch.stack([fx * x / z + cx, fy * y / z + cy], dim=-1)

    zero = torch.zeros_like(z)
    J = torch.stack([
        torch.stack([fx / z, zero, -fx * x / (z * z)], -1),
        torch.stack([zero, fy / z, -fy * y / (z * z)], -1),
    ], dim=-2)
    Tm = J @ W3
    cov2d = Tm @ Sigma @ Tm.transpose(-1, -2)
    det2d = cov2d[:, 0, 0] * cov2d[:, 1, 1] - cov2d[:, 0, 1] * cov2d[:, 1, 0]
    eye2 = torch.eye(2, dtype=F64)
    cov2d_dil = cov2d + st.dilation * eye2
    det_dil = cov2d_dil[:, 0, 0] * cov2d_dil[:, 1, 1] - cov2d_dil[:, 0, 1] * cov2d_dil[:, 1, 0]
    safe_det = torch.where(det_dil > 0, det_dil, torch.ones_like(det_dil))
    conic = torch.stack([cov2d_dil[:, 1, 1] / safe_det,
                         -cov2d_dil[:, 0, 1] / safe_det,
                         cov2d_dil[:, 0, 0] / safe_det], dim=-1)

    opacity = torch.sigmoid(p["opacity_logits"])
    if four_d:
        opacity = opacity * p_t

    campos = camera_center64(cam)
    dvec = mu - campos
    dn = dvec / torch.linalg.vector_norm(dvec, dim=-1, keepdim=True)
    ncoef = (sh_degree + 1) ** 2
    Y = sh_basis64(dn)[:, :ncoef]                              # [N, K]
    n = mu.shape[0]
    coeffs = torch.cat([p["sh_dc"].reshape(n, 1, 3),
                        p["sh_rest"].reshape(n, 15, 3)[:, :ncoef - 1]], dim=1)  # [N, K, 3]
    colour = (Y[:, :, None] * coeffs).sum(dim=1) + 0.5
    rgb = torch.clamp(colour, min=0.0)

    with torch.no_grad():
        valid = ((qn >= st.quat_min) & (z >= float(cam.near)) & (det2d >= st.det_min)
                 & (opacity > st.tau_alpha) & torch.isfinite(det2d))
        thr = 2.0 * torch.log(torch.clamp(opacity, min=1e-300) / st.tau_alpha)
        thr = torch.where(valid, thr, torch.zeros_like(thr))
        ext = torch.sqrt(torch.clamp(thr[:, None] * torch.stack(
            [cov2d_dil[:, 0, 0], cov2d_dil[:, 1, 1]], -1), min=0.0))
        # float32 error model: the decisions of a culled Gaussian's guards,
        # and (mca=True) the per-Gaussian deviations the fragments' bands need
        lam = E.LAMBDA
        kappa = (torch.abs(cov2d[:, 0, 0] * cov2d[:, 1, 1]) + cov2d[:, 0, 1] ** 2) / torch.abs(det2d)
        near_cull = ((torch.abs(qn - st.quat_min) <= 1e-3 * st.quat_min)
                     | (torch.abs(z - float(cam.near)) <= 1e-3 * float(cam.near))
                     | (torch.abs(det2d - st.det_min) <= 1e3 * E.U32 * kappa * torch.abs(det2d))
                     | (torch.abs(opacity - st.tau_alpha) <= 1e-3 * st.tau_alpha))
        cull_border = torch.zeros_like(valid)
        idx = torch.nonzero(near_cull | ~torch.isfinite(kappa)).flatten()
        idx = idx[torch.isfinite(det2d[idx])]
        if len(idx):
            d = _mca(p, idx, cam, st, time)
            cull_border[idx] = ((torch.abs(qn[idx] - st.quat_min) <= lam * E.band_sigma(d["qn"]))
                                | (torch.abs(z[idx] - float(cam.near)) <= lam * E.band_sigma(d["z"]))
                                | (torch.abs(det2d[idx] - st.det_min) <= lam * E.band_sigma(d["det2d"]))
                                | (torch.abs(opacity[idx] - st.tau_alpha)
                                   <= lam * E.band_sigma(d["opacity_rel"]) * opacity[idx]))
        # colour clip at 0: a dot product of up to 16 basis terms, each a few roundings
        terms = Y[:, :, None] * coeffs
        col_sigma = E.U32 * torch.sqrt((4.0 * terms * terms).sum(dim=1) + colour * colour)
        clip_border = (torch.abs(colour) <= lam * col_sigma).any(dim=-1)
        dev = _mca(p, torch.arange(n), cam, st, time) if mca else None
    return {
        "mean2d": mean2d, "cov2d": cov2d, "cov2d_dil": cov2d_dil, "conic": conic,
        "opacity": opacity, "rgb": rgb, "colour": colour, "cam_pos": mh, "det2d": det2d,
        "valid": valid, "cull_border": cull_border, "clip_border": clip_border, "thr": thr, "extent": ext,
        "dev": dev,
    }


def _mca(p: Dict[str, torch.Tensor], idx: torch.Tensor, cam, st: Settings, time: Optional[float] = None,
         chunk: int = 32768):
    """fp32err.mca_deviations of rows idx (in chunks), detached from autograd."""
    W3, t = _camera64(cam)
    keys = ["means", "log_scales", "quats", "opacity_logits"]
    if "quats_r" in p:
        keys += ["mean_t", "log_scale_t", "quats_r"]
    outs = []
    for c0 in range(0, len(idx), chunk):
        sel = idx[c0:c0 + chunk]
        rows = {k: p[k].detach().index_select(0, sel) for k in keys}
        outs.append(E.mca_deviations(rows, W3, t, float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy),
                                     st.dilation, time=time))
    if not outs:
        return None
    return {k: torch.cat([o[k] for o in outs], dim=1) for k in outs[0]}


def composite64(px: torch.Tensor, py: torch.Tensor, mean2d: torch.Tensor,
                conic: torch.Tensor, opacity: torch.Tensor, rgb: torch.Tensor,
                bg: Sequence[float], st: Settings = DEFAULT_SETTINGS, block: int = 256,
                dev: Optional[Dict[str, torch.Tensor]] = None, stats: Optional[Dict[str, torch.Tensor]] = None):
    """Front-to-back compositing of candidates (already in canonical order).

    px, py [P]: pixel sample points.  Candidates: mean2d [G,2], conic [G,3],
    opacity [G], rgb [G,3]; dev: their float32 deviation samples
    (``fp32err.mca_deviations``, [K, G] each), which set the borderline bands
    (None: no bands).  Walks the candidates in blocks of ``block``, carrying
    the transmittance, and stops once no pixel can blend further (the rest
    would not be blended, so this changes nothing).
    Returns (C [P,3] differentiable, T_final [P], last [P] candidate index of
    the last blended fragment or -1, borderline [P] bool, blended count [P]).
    A pixel is borderline when one of its decisions lies within LAMBDA standard
    deviations of the float32 error of the compared quantity: the skip test of
    a walked fragment, the 0.99 cap of a blended one (which switches its
    gradient), or the stop test after a blended fragment.  stats (a dict, with
    dev): receives ``sigma_T`` [P], the relative standard deviation of the
    final transmittance under the float32 error model.
    """
    P = px.shape[0]
    G = mean2d.shape[0]
    lam = E.LAMBDA
    T_run = torch.ones(P, dtype=F64)
    C = torch.zeros(P, 3, dtype=F64)
    last = torch.full((P,), -1, dtype=torch.long)
    border = torch.zeros(P, dtype=torch.bool)
    nblend = torch.zeros(P, dtype=torch.long)
    # the transmittance's relative deviation per sample, and the variance of
    # its independent rounding part, carried along the walk
    K = dev["mean_x"].shape[0] if dev is not None else 0
    dT_run = torch.zeros(K, P, dtype=F64)
    vT_run = torch.zeros(P, dtype=F64)
    for s in range(0, G, block):
        if not bool((T_run.detach() >= st.t_min).any()):
            break
        e = min(G, s + block)
        dx = px[:, None] - mean2d[None, s:e, 0]
        dy = py[:, None] - mean2d[None, s:e, 1]
        a, b, c = conic[s:e, 0], conic[s:e, 1], conic[s:e, 2]
        quad = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
        gauss = torch.exp(-0.5 * quad)
        og = opacity[None, s:e] * gauss
        alpha = torch.clamp(og, max=st.alpha_max)
        use = (alpha >= st.tau_alpha).detach()
        a_eff = torch.where(use, alpha, torch.zeros_like(alpha))
        one_minus = 1.0 - a_eff
        cum = torch.cumprod(one_minus, dim=1)
        excl = torch.cat([torch.ones(P, 1, dtype=F64), cum[:, :-1]], dim=1)
        Tb = T_run[:, None] * excl
        keep = (Tb >= st.t_min).detach()
        w = torch.where(keep, a_eff * Tb, torch.zeros_like(Tb))
        C = C + w @ rgb[s:e]
        T_run = T_run * torch.prod(torch.where(keep, one_minus, torch.ones_like(one_minus)), dim=1)
        contrib = keep & use
        with torch.no_grad():
            k = e - s
            has = contrib.any(dim=1)
            rev_first = torch.argmax(torch.flip(contrib, dims=[1]).to(torch.int8), dim=1)
            last = torch.where(has, s + (k - 1 - rev_first), last)
            nblend += contrib.sum(dim=1)
            if dev is None:
                continue
            ddx, ddy = dx.detach(), dy.detach()
            ga, gb, gc = a.detach(), b.detach(), c.detach()
            dsub = {key: v[:, s:e] for key, v in dev.items()}
            d_ln = E.alpha_deviation(ddx, ddy, ga, gb, gc, dsub)            # [K, P, B]
            v_bl = E.blend_rounding_var(ddx, ddy, ga, gb, gc)               # [P, B]
            sig_a = torch.sqrt(torch.mean(d_ln * d_ln, dim=0) + v_bl)      # relative sigma of alpha (o G)
            al = alpha.detach()
            near_tau = torch.abs(al - st.tau_alpha) <= lam * sig_a * st.tau_alpha
            border |= (keep & near_tau).any(dim=1)
            near_cap = torch.abs(og.detach() - st.alpha_max) <= lam * sig_a * st.alpha_max
            border |= (contrib & near_cap).any(dim=1)
            # T (1 - alpha) as T - alpha T: the factor deviates by
            # -alpha / (1 - alpha) times alpha's relative deviation, plus two roundings
            ae = torch.where(contrib, a_eff.detach(), torch.zeros_like(al))
            ratio = ae / (1.0 - ae)
            dT = dT_run[:, :, None] - torch.cumsum(ratio[None] * d_ln, dim=2)
            vT = vT_run[:, None] + torch.cumsum(torch.where(
                contrib, ratio * ratio * v_bl + 2.0 * E.U32 * E.U32 / 3.0, torch.zeros_like(al)), dim=1)
            dT_run = dT[:, :, -1].clone()
            vT_run = vT[:, -1].clone()
            sig_T = torch.sqrt(torch.mean(dT * dT, dim=0) + vT)
            T_after = Tb.detach() * one_minus.detach()
            near_t = torch.abs(T_after - st.t_min) <= lam * sig_T * st.t_min
            border |= (contrib & near_t).any(dim=1)
    if stats is not None and dev is not None:
        stats["sigma_T"] = torch.sqrt(torch.mean(dT_run * dT_run, dim=0) + vT_run)
    bg_t = torch.as_tensor(list(bg), dtype=F64)
    C = C + T_run[:, None] * bg_t[None, :]
    return C, T_run, last, border, nblend


def _canonical_order(scene: Dict[str, torch.Tensor], cam, idx: np.ndarray,
                     keys: Optional[np.ndarray] = None) -> np.ndarray:
    """Indices ``idx`` ordered by (FP32 depth key, index), the canonical order.
    keys: the FP32 depth of every Gaussian when given (else computed from the
    means as the kernel does)."""
    from .keys32 import depth_key32  # same package; FP32 key spelled out there
    if keys is None:
        keys = depth_key32(scene["means"], cam)
    keys = np.asarray(keys, dtype=np.float32)[idx]
    return idx[np.lexsort((idx, keys))]


def rect_candidates64(mean2d: torch.Tensor, extent: torch.Tensor, box: Tuple[int, int, int, int]) -> torch.Tensor:
    """Mask of the Gaussians whose opacity-aware rectangle (Sec. 3.2, "Splat
    Bounding"; half-extents ``extent``), widened by one pixel, reaches the
    pixel centres of box = (x0, y0, x1, y1), a half-open pixel range.  The
    others have alpha < tau_alpha at every pixel of the box."""
    x0, y0, x1, y1 = box
    return ((mean2d[:, 0] + extent[:, 0] + 1.0 >= x0 + 0.5) & (mean2d[:, 0] - extent[:, 0] - 1.0 <= x1 - 0.5)
            & (mean2d[:, 1] + extent[:, 1] + 1.0 >= y0 + 0.5) & (mean2d[:, 1] - extent[:, 1] - 1.0 <= y1 - 0.5))


def render64(scene: Dict[str, torch.Tensor], cam, st: Settings = DEFAULT_SETTINGS, *,
             dl_dimage: Optional[torch.Tensor] = None, crop: Optional[Tuple[int, int, int, int]] = None,
             cull: bool = True, block_px: int = 16, sh_degree: int = 3,
             depth_block: int = 256, mask_borderline: bool = False, time: Optional[float] = None,
             order_keys: Optional[np.ndarray] = None) -> Dict[str, object]:
    """Render (and optionally differentiate) a scene in float64 on the CPU.

    scene: SoA float32 tensors (see ``synthetic``); cam: camera with
    world_to_cam, fx, fy, cx, cy, width, height, near, bg.
    crop: (x0, y0, x1, y1) pixel box, default the whole image.
    dl_dimage: optional upstream gradient [3, h, w] over the crop; when given,
    gradients of sum(dl_dimage * C) w.r.t. the six raw tensors are returned in
    the SoA layout of ``scene`` (float64).  mask_borderline: the upstream
    gradient is taken as zero on borderline pixels (whose decisions a float32
    evaluation may take either way); the gradient actually used is returned
    as ``dl_used``.
    cull: restrict each block's candidates to the Gaussians whose widened
    opacity-aware rectangle reaches it (exact: outside it alpha < tau_alpha,
    see the module docstring); False makes every Gaussian a candidate of every
    pixel.
    time: the timestep of conditional 4D Gaussians (``cond4d64``).
    order_keys: FP32 depth of every Gaussian for the canonical order (else the
    FP32 camera z of the means, as the kernel computes it; for conditional 4D
    Gaussians the float32 rounding of the float64 conditional depth).
    """
    x0, y0, x1, y1 = crop if crop is not None else (0, 0, int(cam.width), int(cam.height))
    h, w = y1 - y0, x1 - x0
    want_grad = dl_dimage is not None
    rows = _rows(scene)
    N = rows["means"].shape[0]

    with torch.no_grad():
        pre_all = preprocess64(rows, cam, st, sh_degree, time=time)
    valid_idx = torch.nonzero(pre_all["valid"]).flatten().numpy()
    if order_keys is None and "quats_r" in rows:
        order_keys = pre_all["cam_pos"][:, 2].numpy().astype(np.float32)
    order = _canonical_order(scene, cam, valid_idx, order_keys) if len(valid_idx) else valid_idx
    if cull and len(order):
        # Gaussians whose widened FP64 rectangle misses the crop have alpha < tau there.
        near = rect_candidates64(pre_all["mean2d"][order], pre_all["extent"][order], (x0, y0, x1, y1))
        order = order[near.numpy()]
    order_t = torch.as_tensor(order, dtype=torch.long)

    leaves = {}
    for k, v in rows.items():
        leaves[k] = v.clone().requires_grad_(want_grad)
    sub = {k: v.index_select(0, order_t) for k, v in leaves.items()}
    pre = preprocess64(sub, cam, st, sh_degree, mca=True, time=time)
    m2d, con, opa, rgb = pre["mean2d"], pre["conic"], pre["opacity"], pre["rgb"]
    lv = [t.detach().clone().requires_grad_(want_grad) for t in (m2d, con, opa, rgb)]
    devs = pre["dev"]

    image = torch.zeros(3, h, w, dtype=F64)
    tfin = torch.ones(h, w, dtype=F64)
    last_id = torch.full((h, w), -1, dtype=torch.long)
    border = torch.zeros(h, w, dtype=torch.bool)
    nblend = torch.zeros(h, w, dtype=torch.long)

    ext = pre_all["extent"][order_t] if len(order) else torch.zeros(0, 2, dtype=F64)
    m2d_d = m2d.detach()
    bgt = tuple(float(b) for b in cam.bg)

    # pixels touched by a Gaussian whose cull decision is borderline
    cb = torch.nonzero(pre_all["cull_border"]).flatten()
    for gi in cb.tolist():
        with torch.no_grad():
            one = preprocess64({k: v[gi:gi + 1] for k, v in rows.items()}, cam, st, sh_degree, time=time)
            e2 = torch.sqrt(torch.clamp(2.0 * math.log(max(float(one["opacity"][0]), 1e-300) / st.tau_alpha)
                                        * torch.stack([one["cov2d_dil"][0, 0, 0], one["cov2d_dil"][0, 1, 1]]),
                                        min=0.0))
            mx, my = one["mean2d"][0].tolist()
        if not (math.isfinite(mx) and math.isfinite(my)):
            continue
        xs = np.arange(x0, x1) + 0.5
        ys = np.arange(y0, y1) + 0.5
        mxk = np.abs(xs - mx) <= float(e2[0]) + 1.0
        myk = np.abs(ys - my) <= float(e2[1]) + 1.0
        border |= torch.as_tensor(myk[:, None] & mxk[None, :])

    dl_used = dl_dimage.to(F64).clone() if want_grad else None
    import time as _time
    t_blend0 = _time.perf_counter()
    for by in range(y0, y1, block_px):
        for bx in range(x0, x1, block_px):
            ex, ey = min(bx + block_px, x1), min(by + block_px, y1)
            ys, xs = torch.meshgrid(torch.arange(by, ey, dtype=F64), torch.arange(bx, ex, dtype=F64),
                                    indexing="ij")
            px = xs.flatten() + 0.5
            py = ys.flatten() + 0.5
            if cull and len(order):
                cand = torch.nonzero(rect_candidates64(m2d_d, ext, (bx, by, ex, ey))).flatten()
            else:
                cand = torch.arange(len(order))
            cm, cc, co, cr = (t.index_select(0, cand) for t in lv)
            cd = {key: v.index_select(1, cand) for key, v in devs.items()} if devs is not None else None
            Cc, Tc, lc, bc, nc = composite64(px, py, cm, cc, co, cr, bgt, st, block=depth_block, dev=cd)
            hh, ww = ey - by, ex - bx
            sl = (slice(by - y0, ey - y0), slice(bx - x0, ex - x0))
            image[:, sl[0], sl[1]] = Cc.detach().T.reshape(3, hh, ww)
            tfin[sl] = Tc.detach().reshape(hh, ww)
            gid = torch.where(lc >= 0, torch.as_tensor(order, dtype=torch.long)[cand][lc.clamp(min=0)]
                              if len(cand) else lc, torch.full_like(lc, -1))
            last_id[sl] = gid.reshape(hh, ww)
            border[sl] |= bc.reshape(hh, ww)
            nblend[sl] = nc.reshape(hh, ww)
            if want_grad:
                g = dl_dimage[:, by - y0:ey - y0, bx - x0:ex - x0].to(F64).reshape(3, -1).T
                if mask_borderline:
                    g = g * (~border[sl]).reshape(-1, 1).to(F64)
                    dl_used[:, sl[0], sl[1]] = g.T.reshape(3, hh, ww)
                if len(cand):
                    (Cc * g).sum().backward()

    t_blend = _time.perf_counter() - t_blend0
    out: Dict[str, object] = {
        "seconds_compositing": t_blend,
        "image": image, "t_final": tfin, "last_id": last_id, "borderline": border,
        "n_blended": nblend, "order": order, "n_valid": int(len(order)),
        "n_cull_border": int(cb.numel()),
        # Gaussians whose colour clip is borderline: the clip switches their
        # SH (and view-direction) gradients, which elementwise comparisons skip
        "clip_border": torch.as_tensor(order, dtype=torch.long)[pre["clip_border"]],
    }
    if want_grad:
        outs, grads = [], []
        for t, l in zip((m2d, con, opa, rgb), lv):
            if l.grad is not None:
                outs.append(t)
                grads.append(l.grad)
        if outs:
            torch.autograd.backward(outs, grads)
        gsoa = {}
        for k, v in leaves.items():
            g = v.grad if v.grad is not None else torch.zeros_like(v)
            gsoa[k] = g.T.contiguous() if g.dim() == 2 else g
        out["grads"] = gsoa
        out["dl_used"] = dl_used
        out["grads_2d"] = {"mean2d": lv[0].grad, "conic": lv[1].grad, "opacity": lv[2].grad,
                           "rgb": lv[3].grad, "order": order}
    return out


def l1_loss_grad64(image: torch.Tensor, target: torch.Tensor) -> Tuple[float, torch.Tensor]:
    """L1 loss, the mean of |C - target| over all pixels and channels, and its
    gradient sign(C - target) / (3P) with sign(0) = 0 (Sec. 2.1 loss, L1 term)."""
    d = image.to(F64) - target.to(F64)
    n = d.numel()
    return float(torch.abs(d).sum() / n), torch.sign(d) / n


__all__ = ["Settings", "DEFAULT_SETTINGS", "sh_basis64", "quat_to_rotation64", "preprocess64",
           "composite64", "rect_candidates64", "render64", "l1_loss_grad64", "camera_center64"]
