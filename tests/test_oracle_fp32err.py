"""Pins of the float32 error model that sets the oracle's borderline bands
(oracle/fp32err.py).

The bands must not be narrower than the float32 error they stand for.  They
are checked against an actual float32 evaluation of the same formulas,
written here on its own in numpy float32 (one rounding per operation, no
fused operations): Eq. (1)-(2), the dilation, the 2x2 inverse, the
activations, alpha of Eq. (3) and the front-to-back transmittance of Eq. (4).
On the small workload, at every fragment whose alpha lies near tau_alpha the
float32 alpha must lie within the model's band, and along every pixel's walk
the float32 transmittance must lie within the model's transmittance band;
the model's standard deviation must not fall below the observed spread.  A
dropped term, a wrong sign or a missing factor in the model shrinks some band
below the float32 error and fails these tests.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from oracle import fp32err as E
from oracle.render64 import _rows

F32 = np.float32


def hamilton32(p, q):
    """Quaternion product of float32 component lists (w, x, y, z)."""
    return [p[0] * q[0] - p[1] * q[1] - p[2] * q[2] - p[3] * q[3],
            p[0] * q[1] + p[1] * q[0] + p[2] * q[3] - p[3] * q[2],
            p[0] * q[2] - p[1] * q[3] + p[2] * q[0] + p[3] * q[1],
            p[0] * q[3] + p[1] * q[2] - p[2] * q[1] + p[3] * q[0]]


def condition32(sc, t):
    """Conditional 4D Gaussians at time t in numpy float32: the mean, the 3x3
    covariance and the marginal factor (Sec. 3.4), written on its own with
    quaternion products applied to the basis vectors, and the covariance as
    the Gram matrix of the spatial rows of M = R diag(s) with their
    components along the time row removed (the form the kernel evaluates)."""
    def unit(q):
        qn = np.sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3])
        return [q[k] / qn for k in range(4)]
    ql = unit(sc["quats"].numpy().astype(F32))
    qr = unit(sc["quats_r"].numpy().astype(F32))
    n = ql[0].shape[0]
    z, o = np.zeros(n, F32), np.ones(n, F32)
    basis = [[z, o, z, z], [z, z, o, z], [z, z, z, o], [o, z, z, z]]  # x, y, z, t as quaternions
    cols = []
    for e in basis:
        im = hamilton32(hamilton32(ql, e), qr)
        cols.append([im[1], im[2], im[3], im[0]])
    R = [[cols[c][r] for c in range(4)] for r in range(4)]
    s = [np.exp(v) for v in sc["log_scales"].numpy().astype(F32)] + [np.exp(sc["log_scale_t"].numpy().astype(F32))]
    M = [[R[i][k] * s[k] for k in range(4)] for i in range(4)]
    # the time row m of M: Sigma_tt = |m|^2; the spatial rows minus their
    # components along m give the conditional covariance as a Gram matrix
    m = M[3]
    mm = ((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2]) + m[3] * m[3]
    norm = np.sqrt(mm)
    unit = [m[k] / norm for k in range(4)]
    along = [((M[i][0] * unit[0] + M[i][1] * unit[1]) + M[i][2] * unit[2]) + M[i][3] * unit[3] for i in range(3)]
    perp = [[M[i][k] - along[i] * unit[k] for k in range(4)] for i in range(3)]
    dt = F32(t) - sc["mean_t"].numpy().astype(F32)
    mu = sc["means"].numpy().astype(F32)
    mean = [mu[i] + along[i] * (dt / norm) for i in range(3)]
    cov = [[((perp[i][0] * perp[j][0] + perp[i][1] * perp[j][1]) + perp[i][2] * perp[j][2]) + perp[i][3] * perp[j][3]
            for j in range(3)] for i in range(3)]
    p = np.exp(F32(-0.5) * (dt / norm) * (dt / norm))
    return np.stack(mean), cov, p


def preprocess32(sc, cam, time=None):
    """mean2d, conic (a, b, c), opacity in numpy float32, operation by operation
    (conditional 4D Gaussians at ``time`` when the scene has them)."""
    W = np.asarray(cam.world_to_cam, dtype=F32)
    mu = sc["means"].numpy().astype(F32)
    four_d = "quats_r" in sc
    if four_d:
        mu, cov4, p4 = condition32(sc, time)
    X = [(W[r, 0] * mu[0] + W[r, 1] * mu[1]) + W[r, 2] * mu[2] + W[r, 3] for r in range(3)]
    x, y, z = X
    mx = F32(cam.fx) * (x / z) + F32(cam.cx)
    my = F32(cam.fy) * (y / z) + F32(cam.cy)
    q = sc["quats"].numpy().astype(F32)
    qn = np.sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3])
    w, qx, qy, qz = (q[k] / qn for k in range(4))
    one, two = F32(1), F32(2)
    R = [[one - two * (qy * qy + qz * qz), two * (qx * qy - w * qz), two * (qx * qz + w * qy)],
         [two * (qx * qy + w * qz), one - two * (qx * qx + qz * qz), two * (qy * qz - w * qx)],
         [two * (qx * qz - w * qy), two * (qy * qz + w * qx), one - two * (qx * qx + qy * qy)]]
    s = np.exp(sc["log_scales"].numpy().astype(F32))
    M = [[R[i][j] * s[j] for j in range(3)] for i in range(3)]
    Sig = [[(M[i][0] * M[j][0] + M[i][1] * M[j][1]) + M[i][2] * M[j][2] for j in range(3)] for i in range(3)]
    if four_d:
        Sig = cov4
    fx, fy = F32(cam.fx), F32(cam.fy)
    J = [[fx / z, np.zeros_like(z), -(fx / z) * (x / z)], [np.zeros_like(z), fy / z, -(fy / z) * (y / z)]]
    T = [[(J[a][0] * W[0, k] + J[a][1] * W[1, k]) + J[a][2] * W[2, k] for k in range(3)] for a in range(2)]
    U = [[(T[a][0] * Sig[0][k] + T[a][1] * Sig[1][k]) + T[a][2] * Sig[2][k] for k in range(3)] for a in range(2)]
    cov = [[(U[a][0] * T[b][0] + U[a][1] * T[b][1]) + U[a][2] * T[b][2] for b in range(2)] for a in range(2)]
    h00, h11, h01 = cov[0][0] + F32(0.3), cov[1][1] + F32(0.3), cov[0][1]
    det = h00 * h11 - h01 * h01
    o = one / (one + np.exp(-sc["opacity_logits"].numpy().astype(F32)))
    if four_d:
        o = o * p4
    return mx, my, h11 / det, -h01 / det, h00 / det, o


@pytest.fixture(scope="module")
def small():
    sc, cam = S.make_scene(4_000, 7), S.identity_camera(128, 112, 130.0, cx=50.0, cy=70.0)
    rows = _rows(sc)
    with torch.no_grad():
        pre = O.preprocess64(rows, cam, mca=True)
    return sc, cam, pre, preprocess32(sc, cam)


def test_perturbation_switch_and_exact_results():
    gen = torch.Generator().manual_seed(0)
    off = E._Perturb(gen, torch.zeros(2, 1, dtype=torch.float64))
    on = E._Perturb(gen, torch.ones(2, 1, dtype=torch.float64))
    x = torch.rand(2, 50, dtype=torch.float64, generator=gen) + 1.0
    assert torch.equal(off(x), x)  # the reference sample is never perturbed
    y = on(x)
    assert bool((y != x).all()) and float(((y - x) / x).abs().max()) <= E.U32
    f32 = x.float().double()  # float32 numbers are results a float32 operation returns exactly
    assert torch.equal(on(f32), f32)
    assert float(((on(x, 2.0) - x) / x).abs().max()) <= 2 * E.U32


def test_model_deviations_have_the_oracle_shape(small):
    sc, cam, pre, _ = small
    dev = pre["dev"]
    assert set(dev) >= {"mean_x", "mean_y", "conic_a", "conic_b", "conic_c", "opacity_rel"}
    for v in dev.values():
        assert v.shape == (E.K_SAMPLES, S.count(sc))
    assert float(dev["mean_x"][:, pre["valid"]].abs().max()) > 0


def test_mean2d_deviation_matches_its_roundings():
    # identity camera, z = 1: X, Y, Z are exact, so mean_x = fx (x / z) + cx
    # takes three roundings (division, product, sum); the model's spread is
    # sqrt(|x/z|^2 fx^2 + |fx x/z|^2 + |mean_x|^2) u / sqrt(3)
    n = 20_000
    g = torch.Generator().manual_seed(3)
    mu = torch.stack([torch.rand(n, generator=g) * 0.8 + 0.1, torch.zeros(n), torch.ones(n)]).float()
    rows = {"means": mu.double().T.contiguous(), "log_scales": torch.full((n, 3), -3.0, dtype=torch.float64),
            "quats": torch.tensor([[1.0, 0, 0, 0]], dtype=torch.float64).expand(n, 4).contiguous(),
            "opacity_logits": torch.zeros(n, dtype=torch.float64)}
    fx, cx = 300.0, 17.0
    d = E.mca_deviations(rows, torch.eye(3, dtype=torch.float64), torch.zeros(3, dtype=torch.float64),
                         fx, fx, cx, cx, 0.3, K=64)
    x = rows["means"][:, 0]  # x / 1 is exact; the product and the sum are rounded
    prod_exact = (fx * x).float().double() == fx * x
    want = E.U32 / np.sqrt(3.0) * torch.sqrt(torch.where(prod_exact, 0.0, 1.0) * (fx * x) ** 2
                                               + (fx * x + cx) ** 2)
    got = E.band_sigma(d["mean_x"])
    # with 64 samples the estimate scatters by about 1 / sqrt(128)
    ratio = got / want
    assert float(ratio.median()) == pytest.approx(1.0, rel=0.1)
    assert float(ratio.max()) < 1.6


def scene4d(n, seed):
    """The workload's draws plus conditional 4D parameters: time means in [0, 1],
    temporal log-scales N(-1, 0.3), right quaternions near the left ones'
    conjugates (small mixing of space and time)."""
    sc = S.make_scene(n, seed)
    g = torch.Generator().manual_seed(seed + 11)
    sc["mean_t"] = torch.rand(n, generator=g)
    sc["log_scale_t"] = (torch.randn(n, generator=g) * 0.3 - 1.0)
    conj = sc["quats"] * torch.tensor([1.0, -1.0, -1.0, -1.0])[:, None]
    sc["quats_r"] = conj + 0.3 * torch.randn(4, n, generator=g)
    return {k: v.float().contiguous() for k, v in sc.items()}


@pytest.fixture(scope="module")
def small4d():
    sc, cam, t = scene4d(4_000, 8), S.identity_camera(128, 112, 130.0, cx=50.0, cy=70.0), 0.37
    with torch.no_grad():
        pre = O.preprocess64(_rows(sc), cam, mca=True, time=t)
    return sc, cam, pre, preprocess32(sc, cam, time=t)


def test_alpha_band_covers_float32_alpha(small):
    _check_alpha_band(*small)


def test_alpha_band_covers_float32_alpha_conditional_4d(small4d):
    """The same for conditional 4D Gaussians (Sec. 3.4): the model's bands
    include the float32 error of the conditioning."""
    _check_alpha_band(*small4d)


def _check_alpha_band(sc, cam, pre, f32vals):
    mx, my, ca, cb, cc, o32 = f32vals
    v = pre["valid"].numpy()
    idx = np.nonzero(v)[0]
    m64 = pre["mean2d"].numpy()
    con = pre["conic"].numpy()
    op = pre["opacity"].numpy()
    dev = pre["dev"]
    tau = O.DEFAULT_SETTINGS.tau_alpha
    ratios = []
    for i in idx[:1500]:
        ext = np.sqrt(max(pre["thr"][i].item(), 0.0) * max(pre["cov2d_dil"][i, 0, 0].item(),
                                                            pre["cov2d_dil"][i, 1, 1].item())) + 2
        xs = np.arange(max(0, int(m64[i, 0] - ext)), min(cam.width, int(m64[i, 0] + ext) + 1))
        ys = np.arange(max(0, int(m64[i, 1] - ext)), min(cam.height, int(m64[i, 1] + ext) + 1))
        if len(xs) == 0 or len(ys) == 0:
            continue
        PX, PY = np.meshgrid(xs, ys, indexing="xy")
        px64, py64 = PX.ravel() + 0.5, PY.ravel() + 0.5
        dx, dy = px64 - m64[i, 0], py64 - m64[i, 1]
        a64 = op[i] * np.exp(-0.5 * (con[i, 0] * dx * dx + 2 * con[i, 1] * dx * dy + con[i, 2] * dy * dy))
        dx32 = (PX.ravel().astype(F32) + F32(0.5)) - mx[i]
        dy32 = (PY.ravel().astype(F32) + F32(0.5)) - my[i]
        q32 = (ca[i] * dx32 * dx32 + F32(2) * cb[i] * dx32 * dy32) + cc[i] * dy32 * dy32
        a32 = o32[i] * np.exp(F32(-0.5) * q32)
        sel = (a64 > tau / 4) & (a64 < 4 * tau)
        if not sel.any():
            continue
        tdx = torch.as_tensor(dx[sel])[:, None]
        tdy = torch.as_tensor(dy[sel])[:, None]
        di = {k: t[:, i:i + 1] for k, t in dev.items()}
        a, b, c = (torch.as_tensor(con[i:i + 1, j]) for j in range(3))
        d_ln = E.alpha_deviation(tdx, tdy, a, b, c, di)
        sig = torch.sqrt(torch.mean(d_ln * d_ln, dim=0) + E.blend_rounding_var(tdx, tdy, a, b, c))[:, 0].numpy()
        ratios.append(np.abs(a32[sel].astype(np.float64) - a64[sel]) / (a64[sel] * sig))
    r = np.concatenate(ratios)
    print(f"fragments {r.size}: |alpha32 - alpha64| / (alpha sigma) rms {np.sqrt((r ** 2).mean()):.3f} "
          f"p99.9 {np.quantile(r, 0.999):.2f} max {r.max():.2f}")
    assert r.size > 20_000
    assert r.max() <= E.LAMBDA
    assert np.sqrt((r ** 2).mean()) <= 1.0  # the model's sigma is not below the observed spread


def test_transmittance_band_covers_float32_walk(small):
    sc, cam, pre, (mx, my, ca, cb, cc, o32) = small
    ref = O.render64(sc, cam)
    order = ref["order"]
    st = O.DEFAULT_SETTINGS
    tau, amax, tmin = F32(st.tau_alpha), F32(st.alpha_max), F32(st.t_min)
    # the float32 front-to-back walk of Eq. (4) over every candidate, blend then stop
    H, Wd = cam.height, cam.width
    PY, PX = np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij")
    px, py = PX.ravel().astype(F32) + F32(0.5), PY.ravel().astype(F32) + F32(0.5)
    T = np.ones(px.size, F32)
    live = np.ones(px.size, bool)
    for i in order:
        dx, dy = px - mx[i], py - my[i]
        q = (ca[i] * dx * dx + F32(2) * cb[i] * dx * dy) + cc[i] * dy * dy
        al = np.minimum(o32[i] * np.exp(F32(-0.5) * q), amax)
        blend = live & (al >= tau)
        T = np.where(blend, T - al * T, T)
        live &= ~(T < tmin)
    # the model's band of the final transmittance (per pixel, relative)
    rows = _rows(sc)
    sub = {k: v.index_select(0, torch.as_tensor(order)) for k, v in rows.items()}
    with torch.no_grad():
        p2 = O.preprocess64(sub, cam, mca=True)
    stats = {}
    with torch.no_grad():
        _, T64, _, border, _ = O.composite64(torch.as_tensor(px.astype(np.float64)), torch.as_tensor(
            py.astype(np.float64)), p2["mean2d"], p2["conic"], p2["opacity"], p2["rgb"], (0, 0, 0),
            dev=p2["dev"], stats=stats)
    ok = ~border.numpy()
    T64 = T64.numpy()
    diff = np.abs(T.astype(np.float64) - T64)[ok]
    band = T64[ok] * stats["sigma_T"].numpy()[ok]
    assert np.all((band > 0) | (diff == 0))  # no blended fragment: T = 1 on both sides
    r = np.where(diff > 0, diff / np.maximum(band, 1e-300), 0.0)
    print(f"pixels {ok.sum()}: |T32 - T64| / (T sigma_T) rms {np.sqrt((r ** 2).mean()):.3f} max {r.max():.2f}")
    assert r.max() <= E.LAMBDA
    assert np.sqrt((r ** 2).mean()) <= 1.0
    # the culled oracle (candidates by rectangle) gives the same transmittance
    assert np.allclose(T64, ref["t_final"].numpy().ravel(), rtol=1e-12, atol=0)
