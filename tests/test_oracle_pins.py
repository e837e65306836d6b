"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one part of ``oracle.render64`` / ``oracle.adam64`` to
something other than the oracle itself: a closed form of a special case, an
invariant, central finite differences, quadrature, a library routine, a
literal sequential loop, or a value the paper prints (tests/golden).
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from oracle.render64 import DEFAULT_SETTINGS as ST, Settings

F64 = torch.float64
Y00 = 1.0 / (2.0 * math.sqrt(math.pi))  # the constant real SH function, 1/sqrt(4 pi)


def f32(x):
    return float(np.float32(x))


def make_gaussians(rows):
    """rows: list of dicts with mean, log_scale, quat, logit, dc, rest(optional)."""
    n = len(rows)
    sc = {
        "means": torch.tensor([r["mean"] for r in rows], dtype=torch.float32).T.contiguous(),
        "log_scales": torch.tensor([r["log_scale"] for r in rows], dtype=torch.float32).T.contiguous(),
        "quats": torch.tensor([r.get("quat", (1.0, 0.0, 0.0, 0.0)) for r in rows],
                              dtype=torch.float32).T.contiguous(),
        "opacity_logits": torch.tensor([r["logit"] for r in rows], dtype=torch.float32),
        "sh_dc": torch.tensor([r["dc"] for r in rows], dtype=torch.float32).T.contiguous(),
        "sh_rest": torch.zeros(45, n, dtype=torch.float32),
    }
    for i, r in enumerate(rows):
        if "rest" in r:
            sc["sh_rest"][:, i] = torch.tensor(r["rest"], dtype=torch.float32)
    return sc


def pixel_grid(w, h):
    ys, xs = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
    return xs, ys


def closed_form_alpha(xs, ys, mx, my, var_x, var_y, o, st=ST):
    G = np.exp(-0.5 * ((xs - mx) ** 2 / var_x + (ys - my) ** 2 / var_y))
    a = np.minimum(st.alpha_max, o * G)
    return np.where(a >= st.tau_alpha, a, 0.0), G


# --------------------------------------------------------------------------- P1
def test_p1_axis_aligned_single_gaussian_closed_form():
    """An axis-aligned Gaussian on the optical axis (W = I): mu2D = (cx, cy) and
    Sigma2D = diag((fx sx / z)^2, (fy sy / z)^2); the image is alpha*rgb + (1-alpha)*bg."""
    w, h, f = 40, 36, 50.0
    cam = S.identity_camera(w, h, f, bg=(0.1, 0.2, 0.3))
    z, ls, logit, dc = 3.0, (-2.6, -3.0, -2.0), 0.7, (0.4, -0.2, 0.9)
    sc = make_gaussians([dict(mean=(0.0, 0.0, z), log_scale=ls, logit=logit, dc=dc)])
    g_up = S.make_dl_dimage(h, w, seed=3).to(F64)
    r = O.render64(sc, cam, dl_dimage=g_up, cull=False)

    sx, sy = math.exp(f32(ls[0])), math.exp(f32(ls[1]))
    var_x = (f * sx / f32(z)) ** 2 + ST.dilation
    var_y = (f * sy / f32(z)) ** 2 + ST.dilation
    o = 1.0 / (1.0 + math.exp(-f32(logit)))
    xs, ys = pixel_grid(w, h)
    alpha, G = closed_form_alpha(xs, ys, w / 2, h / 2, var_x, var_y, o)
    rgb = np.maximum(np.array([Y00 * f32(c) + 0.5 for c in dc]), 0.0)
    bg = np.array(cam.bg)
    C = alpha[None] * rgb[:, None, None] + (1 - alpha[None]) * bg[:, None, None]
    assert np.abs(r["image"].numpy() - C).max() <= 1e-12
    assert np.abs(r["t_final"].numpy() - (1 - alpha)).max() <= 1e-12
    assert np.array_equal(r["last_id"].numpy(), np.where(alpha > 0, 0, -1))

    # analytic gradients: dC/do = G (rgb - bg) where uncapped; dC/drgb = alpha
    gu = g_up.numpy()
    uncapped = (o * G <= ST.alpha_max) & (alpha > 0)
    dL_do = np.sum(gu * np.where(uncapped, G, 0.0)[None] * (rgb - bg)[:, None, None])
    dL_dlogit = dL_do * o * (1 - o)
    assert abs(float(r["grads"]["opacity_logits"][0]) - dL_dlogit) <= 1e-12 * max(1, abs(dL_dlogit))
    dL_ddc = np.sum(gu * alpha[None], axis=(1, 2)) * Y00
    assert np.abs(r["grads"]["sh_dc"][:, 0].numpy() - dL_ddc).max() <= 1e-11


def test_p1_off_axis_isotropic_closed_form():
    """Off-axis isotropic Gaussian: Sigma = s^2 I for any rotation, so
    Sigma2D = s^2 J J^T; this pins the -f x / z^2 column of Eq. (2)'s Jacobian
    and the projection of Eq. (1)."""
    w, h, f = 48, 40, 60.0
    cam = S.identity_camera(w, h, f, bg=(0.0, 0.5, 1.0), cx=20.0, cy=22.0)
    x0, y0, z = 0.3, -0.25, 2.5
    q = np.array([0.3, -0.5, 0.7, 0.2])
    q /= np.linalg.norm(q)
    sc = make_gaussians([dict(mean=(x0, y0, z), log_scale=(-2.2, -2.2, -2.2), quat=tuple(q),
                              logit=1.5, dc=(0.2, 0.1, -0.3))])
    r = O.render64(sc, cam, cull=False)
    x0, y0, z = f32(x0), f32(y0), f32(z)
    s = math.exp(f32(-2.2))
    qq = np.array([f32(v) for v in q])
    s2 = s * s * float(np.dot(qq, qq))  # R(q/|q|) is a rotation; |q|^2 enters via float32 rounding only
    s2 = s * s
    jx = np.array([f / z, 0.0, -f * x0 / z ** 2])
    jy = np.array([0.0, f / z, -f * y0 / z ** 2])
    cxx = s2 * jx @ jx + ST.dilation
    cyy = s2 * jy @ jy + ST.dilation
    cxy = s2 * jx @ jy
    mx, my = f * x0 / z + 20.0, f * y0 / z + 22.0
    det = cxx * cyy - cxy * cxy
    xs, ys = pixel_grid(w, h)
    dx, dy = xs - mx, ys - my
    quad = (cyy * dx * dx - 2 * cxy * dx * dy + cxx * dy * dy) / det
    o = 1.0 / (1.0 + math.exp(-f32(1.5)))
    a = np.minimum(ST.alpha_max, o * np.exp(-0.5 * quad))
    a = np.where(a >= ST.tau_alpha, a, 0.0)
    rgb = np.maximum(np.array([Y00 * f32(c) + 0.5 for c in (0.2, 0.1, -0.3)]), 0)
    bg = np.array(cam.bg)
    C = a[None] * rgb[:, None, None] + (1 - a[None]) * bg[:, None, None]
    # the quaternion is normalised in float64 from float32 inputs: rotation exact up to 1e-15
    assert np.abs(r["image"].numpy() - C).max() <= 1e-12


# --------------------------------------------------------------------------- P2
def test_p2_weights_plus_transmittance_is_one():
    """With rgb = 1 and c_bg = 0, Eq. (4) gives C = sum_i w_i and C + T_final = 1."""
    rng = np.random.default_rng(5)
    G = 300
    m2d = torch.tensor(rng.uniform(0, 64, (G, 2)), dtype=F64)
    A = rng.normal(size=(G, 2, 2)) * rng.uniform(1, 7, (G, 1, 1))
    m2d[: G // 2, 0] *= 0.5  # dense left half terminates, sparse right half does not
    cov = torch.tensor(A @ A.transpose(0, 2, 1) + 0.3 * np.eye(2), dtype=F64)
    inv = torch.linalg.inv(cov)
    conic = torch.stack([inv[:, 0, 0], inv[:, 0, 1], inv[:, 1, 1]], -1)
    opa = torch.tensor(rng.uniform(0.05, 1.0, G), dtype=F64)
    xs, ys = pixel_grid(64, 64)
    px, py = torch.tensor(xs.ravel()), torch.tensor(ys.ravel())
    C, T, last, border, nb = O.composite64(px, py, m2d, conic, opa, torch.ones(G, 3, dtype=F64),
                                           (0.0, 0.0, 0.0), block=37)
    assert (C[:, 0] + T - 1).abs().max() <= 1e-12
    assert (T < ST.t_min).any() and (T > ST.t_min).any()  # both regimes exercised


# --------------------------------------------------------------------------- literal loop
def sequential_blend(px, py, m2d, conic, opa, rgb, bg, st=ST):
    """App. B.1 + Eq. (4) read literally: walk fragments front to back, skip
    alpha < tau, blend, then stop once T < t_min."""
    T, C, last = 1.0, np.zeros(3), -1
    for i in range(len(opa)):
        dx, dy = px - m2d[i, 0], py - m2d[i, 1]
        a, b, c = conic[i]
        alpha = min(st.alpha_max, opa[i] * math.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)))
        if alpha < st.tau_alpha:
            continue
        C += alpha * T * rgb[i]
        T *= 1.0 - alpha
        last = i
        if T < st.t_min:
            break
    return C + T * np.asarray(bg), T, last


def test_composite_matches_literal_sequential_loop():
    rng = np.random.default_rng(11)
    G = 24
    m2d = rng.uniform(0, 12, (G, 2))
    m2d[:8] = [6.1, 5.2]  # a stack of nearly opaque splats forces early termination
    A = rng.normal(size=(G, 2, 2)) * 1.5
    cov = A @ A.transpose(0, 2, 1) + 0.3 * np.eye(2)
    inv = np.linalg.inv(cov)
    conic = np.stack([inv[:, 0, 0], inv[:, 0, 1], inv[:, 1, 1]], -1)
    opa = rng.uniform(0.02, 0.95, G)
    opa[:8] = 0.93
    cov[:8] = np.diag([40.0, 40.0])
    conic[:8] = [1 / 40.0, 0.0, 1 / 40.0]
    rgb = rng.uniform(0, 1.5, (G, 3))
    bg = (0.3, 0.6, 0.9)
    xs, ys = pixel_grid(12, 10)
    C, T, last, border, _ = O.composite64(torch.tensor(xs.ravel()), torch.tensor(ys.ravel()),
                                          torch.tensor(m2d), torch.tensor(conic), torch.tensor(opa),
                                          torch.tensor(rgb), bg, block=5)
    stopped = 0
    for k, (x, y) in enumerate(zip(xs.ravel(), ys.ravel())):
        c_ref, t_ref, l_ref = sequential_blend(x, y, m2d, conic, opa, rgb, bg)
        assert np.abs(C[k].detach().numpy() - c_ref).max() <= 1e-13
        assert abs(float(T[k]) - t_ref) <= 1e-15
        assert int(last[k]) == l_ref
        stopped += t_ref < ST.t_min
    assert stopped > 0


# --------------------------------------------------------------------------- P3
@pytest.mark.parametrize("front_first", [True, False])
def test_p3_two_gaussians_depth_order(front_first):
    """Two overlapping splats: C = a1 c1 + (1-a1) a2 c2 + (1-a1)(1-a2) bg with 1 the nearer one."""
    w, h, f = 30, 30, 40.0
    cam = S.identity_camera(w, h, f, bg=(0.2, 0.2, 0.2))
    zA, zB = (2.0, 3.0) if front_first else (3.0, 2.0)
    ga = dict(mean=(0.0, 0.0, zA), log_scale=(-2.0, -2.0, -2.0), logit=0.3, dc=(1.0, -1.0, 0.0))
    gb = dict(mean=(0.0, 0.0, zB), log_scale=(-1.8, -1.8, -1.8), logit=1.1, dc=(-1.0, 1.0, 0.5))
    sc = make_gaussians([ga, gb])
    r = O.render64(sc, cam, cull=False)
    xs, ys = pixel_grid(w, h)

    def alpha_rgb(g):
        s = math.exp(f32(g["log_scale"][0]))
        var = (f * s / f32(g["mean"][2])) ** 2 + ST.dilation
        o = 1 / (1 + math.exp(-f32(g["logit"])))
        a, _ = closed_form_alpha(xs, ys, w / 2, h / 2, var, var, o)
        return a, np.maximum(np.array([Y00 * f32(c) + 0.5 for c in g["dc"]]), 0)

    (a1, c1), (a2, c2) = (alpha_rgb(ga), alpha_rgb(gb)) if front_first else (alpha_rgb(gb), alpha_rgb(ga))
    bg = np.array(cam.bg)[:, None, None]
    C = a1 * c1[:, None, None] + (1 - a1) * a2 * c2[:, None, None] + (1 - a1) * (1 - a2) * bg
    assert np.abs(r["image"].numpy() - C).max() <= 1e-12


def test_p3_equal_depth_ties_broken_by_index():
    """Equal FP32 depth keys: the lower Gaussian index is composited first."""
    w, h, f = 20, 20, 30.0
    cam = S.identity_camera(w, h, f)
    g0 = dict(mean=(0.0, 0.0, 2.5), log_scale=(-2.0,) * 3, logit=2.0, dc=(2.0, 0.0, 0.0))
    g1 = dict(mean=(0.01, 0.0, 2.5), log_scale=(-1.9,) * 3, logit=2.0, dc=(0.0, 2.0, 0.0))
    r01 = O.render64(make_gaussians([g0, g1]), cam, cull=False)
    r10 = O.render64(make_gaussians([g1, g0]), cam, cull=False)
    c = r01["image"][:, 10, 10]
    assert c[0] > c[1]          # red (index 0) in front
    c = r10["image"][:, 10, 10]
    assert c[1] > c[0]          # now green has index 0 and is in front


# --------------------------------------------------------------------------- P4
def tiny_scene(seed, n):
    g = torch.Generator().manual_seed(seed)
    sc = {
        "means": torch.stack([torch.rand(n, generator=g) * 1.2 - 0.6, torch.rand(n, generator=g) * 1.2 - 0.6,
                              torch.rand(n, generator=g) * 1.5 + 2.0]),
        "log_scales": torch.randn(3, n, generator=g) * 0.3 - 1.6,
        "quats": torch.randn(4, n, generator=g),
        "opacity_logits": torch.randn(n, generator=g) * 0.8,
        "sh_dc": torch.randn(3, n, generator=g) * 0.4,
        "sh_rest": torch.randn(45, n, generator=g) * 0.1,
    }
    return {k: v.to(torch.float32).contiguous() for k, v in sc.items()}


def _loss64(sc64_rows, cam, gup, st=ST):
    """L = sum(gup * C) in float64 from float64 SoA params (used for finite differences)."""
    sc = {k: v for k, v in sc64_rows.items()}
    rows = {k: (v.T.contiguous() if v.dim() == 2 else v) for k, v in sc.items()}
    pre = O.preprocess64(rows, cam, st)
    valid = pre["valid"]
    idx = torch.nonzero(valid).flatten()
    z = pre["cam_pos"][idx, 2]
    # canonical order by depth then index (distinct depths here)
    order = idx[torch.argsort(z, stable=True)]
    xs, ys = pixel_grid(cam.width, cam.height)
    C, T, last, border, _ = O.composite64(torch.tensor(xs.ravel()), torch.tensor(ys.ravel()),
                                          pre["mean2d"][order], pre["conic"][order], pre["opacity"][order],
                                          pre["rgb"][order], cam.bg, st)
    return float((C.T.reshape(3, cam.height, cam.width) * gup).sum()), bool(border.any())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p4_autograd_matches_central_finite_differences(seed):
    n = 3 + seed
    cam = S.identity_camera(24, 20, 30.0, bg=(0.25, 0.5, 0.75))
    sc = tiny_scene(100 + seed, n)
    gup = S.make_dl_dimage(20, 24, seed=seed).to(F64)
    r = O.render64(sc, cam, dl_dimage=gup, cull=False)
    assert not bool(r["borderline"].any())
    pre = O.preprocess64({k: (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64))
                          for k, v in sc.items()}, cam)
    # kinks: the 0.99 cap and the colour clip; keep draws away from them
    assert bool((pre["colour"].abs() > 1e-3).all())
    base = {k: v.to(F64).clone() for k, v in sc.items()}
    L0, _ = _loss64(base, cam, gup)
    checked = 0
    for name, ad in r["grads"].items():
        flat_ad = ad.reshape(-1)
        scale = float(flat_ad.abs().max())
        for j in range(flat_ad.numel()):
            p = base[name].reshape(-1)
            h = 1e-5 * max(1.0, abs(float(p[j])))
            old = float(p[j])
            p[j] = old + h
            Lp, bp = _loss64(base, cam, gup)
            p[j] = old - h
            Lm, bm = _loss64(base, cam, gup)
            p[j] = old
            if bp or bm:
                continue
            fd = (Lp - Lm) / (2 * h)
            noise = 4 * np.finfo(np.float64).eps * (abs(Lp) + abs(Lm)) / (2 * h)  # rounding floor of the difference
            tol = 1e-6 * max(abs(float(flat_ad[j])), 1e-3 * scale) + noise
            assert abs(fd - float(flat_ad[j])) <= tol, (name, j, fd, float(flat_ad[j]), tol)
            checked += 1
    assert checked >= 59 * n - 4


# --------------------------------------------------------------------------- P5
def test_p5_sh_basis_orthonormal_by_quadrature():
    """Integral over the sphere of Y_i Y_j = delta_ij (Gauss-Legendre in cos(theta),
    uniform in phi; exact for the degree-6 products involved)."""
    ct, wt = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    st_ = np.sqrt(1 - ct ** 2)
    d = np.stack([st_[:, None] * np.cos(phi)[None], st_[:, None] * np.sin(phi)[None],
                  np.broadcast_to(ct[:, None], (24, nphi))], -1).reshape(-1, 3)
    w = np.broadcast_to(wt[:, None] * (2 * np.pi / nphi), (24, nphi)).reshape(-1)
    Y = O.sh_basis64(torch.tensor(d)).numpy()
    gram = (Y * w[:, None]).T @ Y
    assert np.abs(gram - np.eye(16)).max() <= 1e-12


def test_p5_degree_zero_reduction():
    """Degree-0 colour is Y00 * dc + 0.5 (then clipped at 0)."""
    sc = tiny_scene(7, 5)
    cam = S.identity_camera(16, 16, 20.0)
    rows = {k: (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64)) for k, v in sc.items()}
    pre = O.preprocess64(rows, cam, sh_degree=0)
    ref = np.maximum(Y00 * sc["sh_dc"].double().numpy().T + 0.5, 0)
    assert np.abs(pre["rgb"].detach().numpy() - ref).max() <= 1e-15


# --------------------------------------------------------------------------- P6
def test_p6_truncation_constants_printed_in_paper(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "paper_truncation.json")))
    cam = S.identity_camera(64, 64, 64.0)
    sc = make_gaussians([dict(mean=(0.0, 0.0, 4.0), log_scale=(-1.5,) * 3, logit=60.0, dc=(0, 0, 0))])
    rows = {k: (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64)) for k, v in sc.items()}
    for e in gold["entries"]:
        st = Settings(tau_alpha=e["tau_alpha"])
        pre = O.preprocess64(rows, cam, st)
        sigma = math.sqrt(float(pre["cov2d_dil"][0, 0, 0]))
        ratio = float(pre["extent"][0, 0]) / sigma
        assert round(ratio, e["digits"]) == e["sigmas"], (e, ratio)
    # alpha one (dilated) standard deviation from the centre with o -> 1: exp(-1/2)
    pre = O.preprocess64(rows, cam)
    sig = math.sqrt(float(pre["cov2d_dil"][0, 0, 0]))
    C, T, *_ = O.composite64(torch.tensor([32.0 + sig]), torch.tensor([32.0]), pre["mean2d"].detach(),
                             pre["conic"].detach(), pre["opacity"].detach(), torch.ones(1, 3, dtype=F64),
                             (0.0, 0.0, 0.0))
    g = gold["one_sigma_min_opacity"]
    assert round(float(C[0, 0]), g["digits"]) == g["value"]


# --------------------------------------------------------------------------- P7
def test_p7_adam64_matches_torch_adam_and_first_step_closed_form():
    rng = np.random.default_rng(3)
    p0 = torch.tensor(rng.normal(size=500))
    grads = [torch.tensor(rng.normal(size=500)) for _ in range(6)]
    grads[2][::7] = 0.0  # zero-gradient entries still move (the paper updates them)
    lr = 5e-3
    pt = p0.clone().requires_grad_(True)
    opt = torch.optim.Adam([pt], lr=lr, betas=(0.9, 0.999), eps=1e-15, foreach=False, fused=False)
    p, m, v = p0.clone(), torch.zeros(500, dtype=F64), torch.zeros(500, dtype=F64)
    for t, g in enumerate(grads, start=1):
        pt.grad = g.clone()
        opt.step()
        p, m, v = O.adam64(p, g, m, v, t, lr)
        assert ((p - pt.detach()).abs() / pt.detach().abs().clamp_min(1e-300)).max() <= 1e-14
    # first step from zero moments: delta = -lr g / (|g| + eps)
    g = grads[0]
    p1, _, _ = O.adam64(p0, g, torch.zeros_like(g), torch.zeros_like(g), 1, lr)
    err = ((p1 - p0) - (-lr * g / (g.abs() + 1e-15))).abs()
    assert bool((err <= 4 * np.finfo(np.float64).eps * p0.abs()).all())  # p1 - p0 is exact to an ulp of p


# --------------------------------------------------------------------------- P9
def test_p9_alpha_below_threshold_outside_opacity_aware_rectangle():
    sc = S.make_scene(400, seed=9)
    cam = S.workload_camera("c1")
    rows = {k: (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64)) for k, v in sc.items()}
    pre = {k: (v.detach() if torch.is_tensor(v) else v) for k, v in O.preprocess64(rows, cam).items()}
    rng = np.random.default_rng(0)
    vi = torch.nonzero(pre["valid"]).flatten()
    m, e, c, o = pre["mean2d"][vi], pre["extent"][vi], pre["conic"][vi], pre["opacity"][vi]
    for side in range(4):
        u = torch.tensor(rng.uniform(0, 1, len(vi)))
        t = torch.tensor(rng.uniform(-3, 3, len(vi)))
        sgn = 1 if side % 2 == 0 else -1
        if side < 2:   # beyond the x half-extent, anywhere in y
            dx = sgn * e[:, 0] * (1 + 1e-9 + u)
            dy = t * e[:, 1]
        else:
            dy = sgn * e[:, 1] * (1 + 1e-9 + u)
            dx = t * e[:, 0]
        q = c[:, 0] * dx * dx + 2 * c[:, 1] * dx * dy + c[:, 2] * dy * dy
        alpha = o * torch.exp(-0.5 * q)
        assert bool((alpha < ST.tau_alpha).all())


# --------------------------------------------------------------------------- P10
def test_p10_transparent_scene_shows_background():
    sc = S.make_scene(200, seed=1)
    sc["opacity_logits"][:] = -30.0
    cam = S.workload_camera("c1", bg=(0.3, 0.1, 0.7))
    r = O.render64(sc, cam)
    assert r["n_valid"] == 0
    assert torch.allclose(r["image"], torch.tensor(cam.bg, dtype=F64)[:, None, None].expand(3, 256, 256), atol=0)
    assert bool((r["t_final"] == 1).all())


# --------------------------------------------------------------------------- P11
def test_p11_isotropic_rotation_invariance_and_quaternion_scale():
    cam = S.identity_camera(32, 32, 40.0, bg=(0.1, 0.1, 0.1))
    base = dict(mean=(0.1, -0.05, 2.5), log_scale=(-2.0, -2.0, -2.0), logit=0.5, dc=(0.3, 0.2, 0.1))
    r0 = O.render64(make_gaussians([dict(base, quat=(1.0, 0.0, 0.0, 0.0))]), cam, cull=False)
    r1 = O.render64(make_gaussians([dict(base, quat=(0.2, 0.7, -0.1, 0.4))]), cam, cull=False)
    assert (r0["image"] - r1["image"]).abs().max() <= 1e-12
    # anisotropic: scaling q by lambda > 0 leaves the image unchanged and dL/dq is orthogonal to q
    aniso = dict(base, log_scale=(-1.8, -2.4, -2.1), quat=(0.5, 0.5, -0.25, 0.125))
    gup = S.make_dl_dimage(32, 32, seed=4)
    ra = O.render64(make_gaussians([aniso]), cam, dl_dimage=gup, cull=False)
    rb = O.render64(make_gaussians([dict(aniso, quat=(1.5, 1.5, -0.75, 0.375))]), cam, cull=False)  # exact x3
    assert (ra["image"] - rb["image"]).abs().max() <= 1e-12
    q = torch.tensor(aniso["quat"], dtype=torch.float32).double()
    gq = ra["grads"]["quats"][:, 0]
    assert abs(float(gq @ q)) <= 1e-12 * float(gq.norm()) + 1e-15


# --------------------------------------------------------------------------- P12
def test_p12_mean_projection_hand_values():
    """Eq. (1) with a non-trivial W: rotate 90 degrees about z and translate."""
    W = np.array([[0, -1, 0, 0.5], [1, 0, 0, -0.25], [0, 0, 1, 1.0], [0, 0, 0, 1]], dtype=np.float32)
    cam = S.Camera(W, 100.0, 80.0, 50.0, 40.0, 100, 80)
    sc = make_gaussians([dict(mean=(0.5, 1.0, 3.0), log_scale=(-3,) * 3, logit=0, dc=(0, 0, 0)),
                         dict(mean=(-1.0, 0.25, 1.0), log_scale=(-3,) * 3, logit=0, dc=(0, 0, 0))])
    rows = {k: (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64)) for k, v in sc.items()}
    pre = O.preprocess64(rows, cam)
    # camera coords: (-y + 0.5, x - 0.25, z + 1)
    # G0: (-0.5, 0.25, 4.0) -> (100*-0.5/4 + 50, 80*0.25/4 + 40) = (37.5, 45.0)
    # G1: (0.25, -1.25, 2.0) -> (62.5, -10.0)
    assert np.allclose(pre["mean2d"].detach().numpy(), [[37.5, 45.0], [62.5, -10.0]], atol=1e-12, rtol=0)
    assert np.allclose(pre["cam_pos"][:, 2].detach().numpy(), [4.0, 2.0], atol=0)
    # camera centre -W3^T t: the point that maps to camera (0,0,0)
    c = O.camera_center64(cam).numpy()
    assert np.allclose(W[:3, :3].astype(np.float64) @ c + W[:3, 3], 0, atol=1e-12)


# --------------------------------------------------------------------------- culling exactness
def test_candidate_culling_does_not_change_the_result():
    sc = S.make_scene(1500, seed=4)
    cam = S.workload_camera("c1", bg=(0.2, 0.4, 0.6))
    gup = S.make_dl_dimage(64, 64, seed=2)
    crop = (96, 80, 160, 144)
    a = O.render64(sc, cam, crop=crop, dl_dimage=gup, cull=True)
    b = O.render64(sc, cam, crop=crop, dl_dimage=gup, cull=False)
    assert (a["image"] - b["image"]).abs().max() <= 1e-13
    assert torch.equal(a["last_id"], b["last_id"])
    for k in a["grads"]:
        assert (a["grads"][k] - b["grads"][k]).abs().max() <= 1e-11 * max(1.0, float(b["grads"][k].abs().max()))


def _certify_dropped(pre, keep, box, tau):
    """Every valid Gaussian outside ``keep`` stays below tau_alpha at every
    pixel centre of box = (x0, y0, x1, y1): proved for most of them by the
    smallest eigenvalue of the conic and the distance from the mean to the
    box (alpha <= o exp(-lambda_min dist^2 / 2)), and by brute force over the
    box's pixel centres for the rest.  Returns (dropped, brute-forced)."""
    x0, y0, x1, y1 = box
    idx = torch.nonzero(pre["valid"] & ~keep).flatten()
    m = pre["mean2d"][idx].detach()
    a, b, c = (pre["conic"][idx, k].detach() for k in range(3))
    o = pre["opacity"][idx].detach()
    lam_min = 0.5 * (a + c) - torch.sqrt((0.5 * (a - c)) ** 2 + b * b)
    assert bool((lam_min > 0).all())
    dx = torch.clamp(torch.maximum(x0 + 0.5 - m[:, 0], m[:, 0] - (x1 - 0.5)), min=0.0)
    dy = torch.clamp(torch.maximum(y0 + 0.5 - m[:, 1], m[:, 1] - (y1 - 0.5)), min=0.0)
    bound = o * torch.exp(-0.5 * lam_min * (dx * dx + dy * dy))
    rest = torch.nonzero(bound >= tau).flatten()
    if len(rest):
        ys, xs = torch.meshgrid(torch.arange(y0, y1, dtype=F64) + 0.5, torch.arange(x0, x1, dtype=F64) + 0.5,
                                indexing="ij")
        ddx = xs.flatten()[None, :] - m[rest, 0:1]
        ddy = ys.flatten()[None, :] - m[rest, 1:2]
        q = a[rest, None] * ddx * ddx + 2.0 * b[rest, None] * ddx * ddy + c[rest, None] * ddy * ddy
        alpha = o[rest, None] * torch.exp(-0.5 * q)
        assert float(alpha.max()) < tau, "a dropped candidate reaches tau_alpha"
    return len(idx), len(rest)


def _check_block_culling(scene, cam, box, block=16):
    """The two-level candidate culling of render64 (the box, then each block
    of it) drops only Gaussians that never reach tau_alpha there."""
    rows = {k: (v.to(F64).T.contiguous() if v.dim() == 2 else v.to(F64)) for k, v in scene.items()}
    with torch.no_grad():
        pre = O.preprocess64(rows, cam, sh_degree=0)  # colour plays no part in the selection
    tau = O.DEFAULT_SETTINGS.tau_alpha
    x0, y0, x1, y1 = box
    keep_box = O.rect_candidates64(pre["mean2d"], pre["extent"], box)
    _certify_dropped(pre, keep_box, box, tau)
    dropped = 0
    for by in range(y0, y1, block):
        for bx in range(x0, x1, block):
            blk = (bx, by, min(bx + block, x1), min(by + block, y1))
            keep = keep_box & O.rect_candidates64(pre["mean2d"], pre["extent"], blk)
            dropped += _certify_dropped(pre, keep, blk, tau)[0]
    assert dropped > 0


def test_candidate_culling_is_exact_on_the_small_workload_frame():
    """Candidate culling over the whole 10k-Gaussian 256x256 frame, block by block."""
    _check_block_culling(S.make_scene(10_000, seed=0), S.workload_camera("c1"), (0, 0, 256, 256))


@pytest.mark.parametrize("box", [(768, 498, 832, 562), (1336, 996, 1400, 1060), (0, 0, 64, 64)],
                         ids=["centre", "edge", "corner"])
def test_candidate_culling_is_exact_on_the_3m_crops(box):
    """Candidate culling at the 64x64 crops of the 3M-Gaussian 1600x1060 frame."""
    _check_block_culling(S.make_scene(3_000_000, seed=0), S.workload_camera("c3"), box)


def test_degenerate_gaussians_are_not_rendered():
    """App. B.1: |q| < 1e-4 or det(Sigma2D) < 1e-6 -> not rendered; also behind the near plane."""
    cam = S.identity_camera(32, 32, 40.0)
    good = dict(mean=(0.0, 0.0, 3.0), log_scale=(-2.0,) * 3, logit=2.0, dc=(1.0, 1.0, 1.0))
    bad_q = dict(good, quat=(5e-5, 0.0, 0.0, 0.0))
    tiny = dict(good, log_scale=(-12.0, -12.0, -12.0))
    behind = dict(good, mean=(0.0, 0.0, 0.1))
    r = O.render64(make_gaussians([bad_q, tiny, behind]), cam, cull=False)
    assert r["n_valid"] == 0
    r = O.render64(make_gaussians([good, bad_q]), cam, cull=False)
    assert r["n_valid"] == 1
