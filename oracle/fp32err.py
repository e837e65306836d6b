"""Float32 error model of the rasterizer's threshold decisions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The method makes hard decisions: a fragment is skipped when alpha falls below
tau_alpha (Sec. 3.2, "Splat Bounding"), alpha is capped at 0.99 and a pixel
stops once its transmittance falls below 1e-4 (App. B.1), and Gaussians are
culled by the guards of App. B.1 and the opacity test.  A float32 evaluation
of the same formulas can take such a decision the other way than the float64
oracle only where the float64 value lies within the float32 error of the
compared quantity; the comparison protocol exempts those decisions.

Width of each exemption band: LAMBDA standard deviations of that float32
error.  The standard deviation is estimated by Monte Carlo arithmetic
(D. S. Parker, "Monte Carlo Arithmetic", 1997): the per-Gaussian formulas
(Eq. (1), Eq. (2), the dilation, the 2x2 inverse, the activations) are
evaluated K times in float64 with the result of every operation multiplied by
(1 + m u xi), xi uniform in [-1, 1] and independent, u = 2^-24 the unit
roundoff of float32, m = 1 for the basic operations and 2 for exp and sqrt;
an operation whose exact result is a float32 number is left exact (a float32
operation returns it unrounded).  A round-to-nearest error lies within half
an ulp, at most u times the result, and is spread evenly there, so the model's
per-operation spread (u |x| / sqrt(3)) is at least the real one.  The sampled
deviations of mean2d, the conic and the opacity are carried to each fragment
to first order (``alpha_deviation``); the blend's own handful of operations
adds an independent term.  With LAMBDA = 6 a normally distributed error
exceeds its band with probability 2e-9.
"""
from __future__ import annotations

from typing import Dict, Optional

import torch

F64 = torch.float64
U32 = 2.0 ** -24
LAMBDA = 6.0
K_SAMPLES = 16


class _Perturb:
    """Rounding model of one Monte Carlo sample set: r(x) = x (1 + m u xi)."""

    def __init__(self, gen: torch.Generator, on: torch.Tensor):
        self.gen = gen
        self.on = on  # [K, 1] 1.0 for perturbed samples, 0.0 for the exact reference

    def __call__(self, x: torch.Tensor, m: float = 1.0) -> torch.Tensor:
        xi = torch.rand(x.shape, generator=self.gen, dtype=F64) * 2.0 - 1.0
        y = x * (1.0 + (m * U32) * xi * self.on)
        exact = x.to(torch.float32).to(F64) == x
        return torch.where(exact, x, y)


def mca_deviations(rows: Dict[str, torch.Tensor], W3: torch.Tensor, t: torch.Tensor, fx: float, fy: float,
                   cx: float, cy: float, dilation: float, K: int = K_SAMPLES, seed: int = 0,
                   time: Optional[float] = None) -> Dict[str, torch.Tensor]:
    """Deviations of K float32-rounding samples of the per-Gaussian quantities
    from their exact values (all float64).

    rows: the row tensors of ``render64.preprocess64`` (means [N,3],
    log_scales [N,3], quats [N,4], opacity_logits [N]); W3, t: the camera's
    rotation and translation; fx, fy, cx, cy: intrinsics; dilation: the 2D
    filter variance.  Conditional 4D Gaussians (rows with mean_t,
    log_scale_t, quats_r; Sec. 3.4) are conditioned on ``time`` first: the
    4D rotation from the two normalised quaternions, M = R diag(s), and the
    conditional mean, covariance and marginal factor in the projection form
    the kernel evaluates (the covariance as N N^T with N the spatial rows of
    M projected off the unit time row), one rounding per operation.  Returns [K, N] tensors: mean2d x and y, conic a, b, c, opacity
    (relative), quaternion norm (the smaller of two), camera z, det of the
    un-dilated Sigma2D.
    """
    N = rows["means"].shape[0]
    gen = torch.Generator().manual_seed(seed)
    on = torch.ones(K + 1, 1, dtype=F64)
    on[0] = 0.0  # sample 0 is the unperturbed evaluation of the same formulas
    r = _Perturb(gen, on)

    def ex(v: torch.Tensor) -> torch.Tensor:
        return v.unsqueeze(0).expand(K + 1, N).clone()

    mu = [ex(rows["means"][:, i]) for i in range(3)]
    four_d = time is not None and "quats_r" in rows

    def unit_quat(key):
        q = [ex(rows[key][:, i]) for i in range(4)]
        n2 = r(r(r(r(q[0] * q[0]) + r(q[1] * q[1])) + r(q[2] * q[2])) + r(q[3] * q[3]))
        qn = r(torch.sqrt(n2), 2.0)
        return [r(c / qn) for c in q], qn

    def dot(a, b):
        acc = r(a[0] * b[0])
        for k in range(1, len(a)):
            acc = r(acc + r(a[k] * b[k]))
        return acc

    if four_d:
        # 4D rotation v -> ql v qr as L(ql) R(qr) in (w, x, y, z), then (x, y, z, t) order
        a, qn_l = unit_quat("quats")
        b, qn_r = unit_quat("quats_r")
        Lm = [[a[0], -a[1], -a[2], -a[3]], [a[1], a[0], -a[3], a[2]], [a[2], a[3], a[0], -a[1]],
              [a[3], -a[2], a[1], a[0]]]
        Rq = [[b[0], -b[1], -b[2], -b[3]], [b[1], b[0], b[3], -b[2]], [b[2], -b[3], b[0], b[1]],
              [b[3], b[2], -b[1], b[0]]]
        P = [[dot(Lm[i], [Rq[k][j] for k in range(4)]) for j in range(4)] for i in range(4)]
        perm = [1, 2, 3, 0]
        R4 = [[P[perm[i]][perm[j]] for j in range(4)] for i in range(4)]
        s4 = [r(torch.exp(ex(rows["log_scales"][:, j])), 2.0) for j in range(3)]
        s4.append(r(torch.exp(ex(rows["log_scale_t"])), 2.0))
        M4 = [[r(R4[i][k] * s4[k]) for k in range(4)] for i in range(4)]
        # projection form: u = m_t / |m_t|, h = M_xyz u, e = dt / |m_t|,
        # N = M_xyz - h u^T; mean + h e, covariance N N^T, factor exp(-e^2 / 2)
        nt = r(torch.sqrt(dot(M4[3], M4[3])))
        inv = r(1.0 / nt)
        u = [r(M4[3][k] * inv) for k in range(4)]
        dt = r(float(time) - ex(rows["mean_t"]))
        e_t = r(dt * inv)
        h = [dot(M4[i], u) for i in range(3)]
        N4 = [[r(M4[i][k] - r(h[i] * u[k])) for k in range(4)] for i in range(3)]
        mu = [r(mu[i] + r(h[i] * e_t)) for i in range(3)]
        Sig4c = [[dot(N4[i], N4[j]) for j in range(3)] for i in range(3)]
        p_t = r(torch.exp(-r(0.5 * r(e_t * e_t))), 2.0)
    Wf = [[float(W3[i, j]) for j in range(3)] for i in range(3)]
    tf = [float(t[i]) for i in range(3)]

    # Eq. (1): camera-space position, then the projected mean
    cam = [r(r(r(r(Wf[i][0] * mu[0]) + r(Wf[i][1] * mu[1])) + r(Wf[i][2] * mu[2])) + tf[i]) for i in range(3)]
    X, Y, Z = cam
    xz, yz = r(X / Z), r(Y / Z)
    mx = r(r(fx * xz) + cx)
    my = r(r(fy * yz) + cy)

    def dot3(a, b):
        return r(r(r(a[0] * b[0]) + r(a[1] * b[1])) + r(a[2] * b[2]))

    if four_d:
        Sig = Sig4c
        qn = torch.minimum(qn_l, qn_r)
    else:
        # activations: normalised quaternion -> rotation, exp scales
        (w, x, y, z), qn = unit_quat("quats")
        xx, yy, zz = r(x * x), r(y * y), r(z * z)
        xy, xz_, yz_ = r(x * y), r(x * z), r(y * z)
        wx, wy, wz = r(w * x), r(w * y), r(w * z)
        Rm = [[r(1.0 - 2.0 * r(yy + zz)), 2.0 * r(xy - wz), 2.0 * r(xz_ + wy)],
              [2.0 * r(xy + wz), r(1.0 - 2.0 * r(xx + zz)), 2.0 * r(yz_ - wx)],
              [2.0 * r(xz_ - wy), 2.0 * r(yz_ + wx), r(1.0 - 2.0 * r(xx + yy))]]
        s = [r(torch.exp(ex(rows["log_scales"][:, j])), 2.0) for j in range(3)]
        M = [[r(Rm[i][j] * s[j]) for j in range(3)] for i in range(3)]
        Sig = [[dot3(M[i], M[j]) for j in range(3)] for i in range(3)]
    # Eq. (2): T = J W3 with J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]
    j00, j11 = r(fx / Z), r(fy / Z)
    j02, j12 = -r(j00 * xz), -r(j11 * yz)
    T = [[r(r(j00 * Wf[0][k]) + r(j02 * Wf[2][k])) for k in range(3)],
         [r(r(j11 * Wf[1][k]) + r(j12 * Wf[2][k])) for k in range(3)]]
    U = [[dot3(T[a], [Sig[j][k] for j in range(3)]) for k in range(3)] for a in range(2)]
    c00, c01, c11 = dot3(U[0], T[0]), dot3(U[0], T[1]), dot3(U[1], T[1])
    det2d = r(r(c00 * c11) - r(c01 * c01))
    h00, h11, h01 = r(c00 + dilation), r(c11 + dilation), c01
    deth = r(r(h00 * h11) - r(h01 * h01))
    ca, cb, cc = r(h11 / deth), -r(h01 / deth), r(h00 / deth)
    # opacity = sigmoid(logit)
    o = r(1.0 / r(1.0 + r(torch.exp(-ex(rows["opacity_logits"])), 2.0)))
    if four_d:
        o = r(o * p_t)

    def dev(v):
        return v[1:] - v[:1]

    return {"mean_x": dev(mx), "mean_y": dev(my), "conic_a": dev(ca), "conic_b": dev(cb), "conic_c": dev(cc),
            "opacity_rel": dev(o) / o[:1], "qn": dev(qn), "z": dev(Z), "det2d": dev(det2d)}


def band_sigma(d: torch.Tensor) -> torch.Tensor:
    """Standard deviation (root mean square over the samples, dim 0) of zero-mean deviations."""
    return torch.sqrt(torch.mean(d * d, dim=0))


def alpha_deviation(dx: torch.Tensor, dy: torch.Tensor, a: torch.Tensor, b: torch.Tensor, c: torch.Tensor,
                    dev: Dict[str, torch.Tensor]) -> torch.Tensor:
    """First-order deviation of ln(alpha) = ln(o) - 1/2 d^T conic d, d = x - mean2d,
    at fragments (pixel p, candidate g), per sample: [K, P, G].

    dx, dy [P, G]; a, b, c [G] (the conic); dev: ``mca_deviations`` of the
    candidates ([K, G] each)."""
    gx = a * dx + b * dy  # d ln(alpha) / d mean2d
    gy = b * dx + c * dy
    return (gx[None] * dev["mean_x"][:, None, :] + gy[None] * dev["mean_y"][:, None, :]
            - 0.5 * (dev["conic_a"][:, None, :] * (dx * dx)[None]
                     + 2.0 * dev["conic_b"][:, None, :] * (dx * dy)[None]
                     + dev["conic_c"][:, None, :] * (dy * dy)[None])
            + dev["opacity_rel"][:, None, :])


def blend_rounding_var(dx: torch.Tensor, dy: torch.Tensor, a: torch.Tensor, b: torch.Tensor,
                       c: torch.Tensor) -> torch.Tensor:
    """Variance of ln(alpha)'s error from the blend's own operations at each
    fragment [P, G]: the pixel offset (one rounding per axis), the quadratic
    form (six roundings of at most its absolute terms), exp (2u) and the
    product with the opacity; each rounding of x contributes u^2 x^2 / 3."""
    gx = a * dx + b * dy
    gy = b * dx + c * dy
    q = 0.5 * (torch.abs(a) * dx * dx + 2.0 * torch.abs(b * dx * dy) + torch.abs(c) * dy * dy)
    return (U32 * U32 / 3.0) * ((gx * dx) ** 2 + (gy * dy) ** 2 + 6.0 * q * q + 4.0 + 1.0)


__all__ = ["U32", "LAMBDA", "K_SAMPLES", "mca_deviations", "band_sigma", "alpha_deviation",
           "blend_rounding_var"]
