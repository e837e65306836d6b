"""Shared helpers for the GPU parity tests (not a test module)."""
from __future__ import annotations

import sys
from typing import Dict, Optional

import numpy as np
import torch

import oracle as O
import synthetic as S
from paper_2602_09999_amd import binding as B


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


# Comparison protocol against the FP64 oracle.
IMG_TOL = 1e-5        # image and final transmittance, absolute, off borderline pixels
GRAD_TOL = 1e-3       # gradients: per-group relative L2 and the elementwise bound below
# Borderline pixels (a decision within the float32 error band of oracle/fp32err.py,
# 6 standard deviations of the modelled float32 error) may make up at most this
# fraction of a comparison's pixels.  The fraction grows with the fragments whose
# alpha ring or stop crosses a pixel centre inside a band: measured 0.03 % at the
# small workload, 0.2-0.25 % at the 64x64 crops of the 3M one and up to 0.41 % at
# the bottom-edge window of the dynamic workload (few, large, far off-axis
# Gaussians).  The cap bounds a band model gone wide; it is not the tolerance.
EXEMPT_FRAC = 0.005


def exempt_cap(npix: int) -> int:
    return max(2, int(EXEMPT_FRAC * npix))


def check_image(label: str, image, ref, t_final=None, last_ids_gpu=None) -> np.ndarray:
    """Image (and T, last contributor) against render64's output on the pixels
    without a borderline decision; returns that pixel mask.  Logs the exempt
    count and the max abs, max relative and RMS error."""
    ok = ~ref["borderline"].numpy()
    img = image.detach().cpu().double().numpy()
    r = ref["image"].numpy()
    d = np.abs(img - r)
    dm = d.max(0)
    n_ex = int((~ok).sum())
    rel = (d / np.maximum(np.abs(r), 1e-3)).max(0)
    flips = int((dm[~ok] > IMG_TOL).sum())  # exempt pixels where a decision did go the other way
    say(f"  {label}: exempt {n_ex} of {ok.size} (cap {exempt_cap(ok.size)}; {flips} of them off by more than "
        f"{IMG_TOL:g}); image max abs {dm[ok].max():.2e} max rel {rel[ok].max():.2e} "
        f"rms {np.sqrt((d[:, ok] ** 2).mean()):.2e}")
    assert n_ex <= exempt_cap(ok.size), (label, n_ex)
    assert dm[ok].max() <= IMG_TOL, (label, float(dm[ok].max()))
    if t_final is not None:
        te = np.abs(t_final.detach().cpu().double().numpy() - ref["t_final"].numpy())
        say(f"  {label}: T max abs {te[ok].max():.2e}")
        assert te[ok].max() <= IMG_TOL, (label, float(te[ok].max()))
    if last_ids_gpu is not None:
        assert np.array_equal(last_ids_gpu[ok], ref["last_id"].numpy()[ok]), label
    return ok


def _gaussian_axis_rows(t: torch.Tensor) -> torch.Tensor:
    """[k, n] or [n] -> [n, k]: one row per Gaussian."""
    return t.T if t.dim() == 2 else t[:, None]


def grad_errors(got: torch.Tensor, ref: torch.Tensor, tol: float = GRAD_TOL,
                exempt: Optional[np.ndarray] = None, bf16: bool = False) -> Dict[str, float]:
    """Errors of one gradient group against the FP64 oracle, with the
    elementwise bound |g - g_ref| <= tol * max(|g_ref|, rms) (rms: root mean
    square of g_ref over the Gaussians that receive a gradient).  bf16: g is
    the bfloat16 rounding of a float32 value, which may lie half a bfloat16
    ulp further.  exempt: Gaussian indices left out of the elementwise check."""
    g = _gaussian_axis_rows(got.detach().float().cpu().double())
    r = _gaussian_axis_rows(ref.detach().cpu().double())
    live = (r != 0).any(dim=1)
    rms = float(torch.sqrt((r[live] ** 2).mean())) if bool(live.any()) else 0.0
    d = (g - r).abs()
    bound = tol * torch.clamp(r.abs(), min=rms)
    if bf16:
        # half an ulp of bfloat16 (8 significant bits) at the value's binade
        e = torch.floor(torch.log2(torch.clamp(r.abs() * (1 + tol), min=1e-38)))
        bound = bound + torch.pow(2.0, e - 8)
    mask = torch.ones_like(d, dtype=torch.bool)
    if exempt is not None and len(exempt):
        mask[torch.as_tensor(np.asarray(exempt), dtype=torch.long)] = False
    over = (d > bound) & mask
    big = (r.abs() >= rms) & mask
    return {
        "rel_l2": float((g - r).norm()) / max(float(r.norm()), 1e-300),
        "max_abs": float(d.max()) if d.numel() else 0.0,
        "max_rel": float((d[big] / r.abs()[big]).max()) if bool(big.any()) else 0.0,
        "rms": float(torch.sqrt((d ** 2).mean())) if d.numel() else 0.0,
        "worst_ratio": float((d / torch.clamp(bound, min=1e-300))[mask].max()) if bool(mask.any()) else 0.0,
        "n_over": int(over.sum()),
        "n_gaussians": int(live.sum()),
    }


def check_grads(label: str, got: Dict[str, torch.Tensor], ref: Dict[str, torch.Tensor], names=None,
                tol: float = GRAD_TOL, exempt: Optional[np.ndarray] = None, bf16_groups=(),
                rel_tol: Optional[Dict[str, float]] = None) -> Dict[str, Dict[str, float]]:
    """Every gradient group: relative L2 <= tol (or rel_tol[group]) and the
    elementwise bound of grad_errors; logs max abs, max relative and RMS error."""
    out = {}
    for k in names or B.PARAM_NAMES:
        e = grad_errors(got[k], ref[k], tol, exempt, bf16=k in bf16_groups)
        lim = (rel_tol or {}).get(k, tol)
        say(f"  {label} {k:15s} rel L2 {e['rel_l2']:.2e} max abs {e['max_abs']:.2e} max rel {e['max_rel']:.2e} "
            f"rms {e['rms']:.2e} worst/bound {e['worst_ratio']:.2e} over {e['n_over']} "
            f"({e['n_gaussians']} Gaussians)")
        assert e["rel_l2"] <= lim, (label, k, e)
        assert e["n_over"] == 0, (label, k, e)
        out[k] = e
    return out


def to_gpu(scene: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
    return {k: v.to("cuda").contiguous() for k, v in scene.items()}


def forward(scene, cam, capacity: Optional[int] = None, settings=None):
    rz = B.Rasterizer(cam, settings=settings)
    params = to_gpu(scene)
    if capacity is not None:
        rz._ensure(int(params["opacity_logits"].shape[0]), capacity)
    image, t_final, last = rz.forward(params)
    torch.cuda.synchronize()
    return rz, params, image, t_final, last


def sorted_instances(rz: B.Rasterizer):
    lay = rz.layout()
    I = rz.last_stats["n_instances"]
    kdt = torch.int16 if lay.inst_key_bytes == 2 else torch.int32
    keys = rz.view("inst_keys", I, dtype=kdt, index=lay.inst_final).cpu().numpy()
    keys = keys.view(np.uint16 if lay.inst_key_bytes == 2 else np.uint32).astype(np.uint32)
    vals = rz.view("inst_vals", I, index=lay.inst_final).cpu().numpy().view(np.uint32)
    tiles = int(lay.total_tiles)
    ranges = rz.view("ranges", 2 * tiles).cpu().numpy().view(np.uint32).reshape(tiles, 2)
    return keys, vals, ranges


def record(rz: B.Rasterizer, n: int) -> np.ndarray:
    """The first three float4 of each 64-byte record: mu2D, o, thr | a, b, c, z | rgb, flags."""
    return rz.view("rec", 16 * n, dtype=torch.float32).cpu().numpy().reshape(n, 16)[:, :12]


def last_ids(rz: B.Rasterizer, last: torch.Tensor) -> np.ndarray:
    """Gaussian index of each pixel's last blended fragment (-1 if none)."""
    keys, vals, ranges = sorted_instances(rz)
    lay = rz.layout()
    h, w = last.shape
    t = int(rz.settings.tile)
    ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    tile = (ys // t) * lay.tiles_x + xs // t
    lp = last.cpu().numpy().astype(np.int64)
    pos = ranges[tile, 0].astype(np.int64) + lp - 1
    out = np.full((h, w), -1, np.int64)
    ok = lp > 0
    out[ok] = vals[pos[ok]]
    return out


def compare_lists(keys, vals, ranges, ref, border_pairs, depth=None):
    """Bit-exact comparison of sorted instances with the FP32 key reference,
    allowing only the borderline (tile, gaussian) pairs to differ.
    Returns the number of borderline pairs on which the two disagree."""
    tiles = ranges.shape[0]
    assert ref["ranges"].shape[0] == tiles
    flips = 0
    if not border_pairs:
        assert np.array_equal(keys, ref["keys"]), "tile keys differ"
        assert np.array_equal(vals, ref["vals"]), "values differ"
        assert np.array_equal(ranges, ref["ranges"]), "tile ranges differ"
        return 0
    by_tile = {}
    for t, g in border_pairs:
        by_tile.setdefault(t, set()).add(g)
    for t in range(tiles):
        s, e = ranges[t]
        rs, re_ = ref["ranges"][t]
        a = vals[s:e].tolist()
        b = ref["vals"][rs:re_].tolist()
        if a == b:
            continue
        bt = by_tile.get(t, set())
        a2 = [g for g in a if g not in bt]
        b2 = [g for g in b if g not in bt]
        assert a2 == b2, f"tile {t}: lists differ outside the borderline band"
        flips += len(set(a) ^ set(b))
    # keys must be the tile id of each slot, lists in (depth key, index) order
    dbits = None if depth is None else np.asarray(depth, np.float32).view(np.uint32).astype(np.int64)
    for t in range(tiles):
        s, e = ranges[t]
        assert np.all(keys[s:e] == t)
        if dbits is not None and e - s > 1:
            v = vals[s:e].astype(np.int64)
            comp = dbits[v] * (1 << 32) + v
            assert np.all(np.diff(comp) > 0), f"tile {t} not in (depth, index) order"
    return flips


CROPS = {
    # 64x64 comparison windows of the full-size workloads: the image centre,
    # and the bottom edge where the projected means are largest (the last tile
    # row of the 1060-pixel frame is partial: 1060 = 66 * 16 + 4)
    "c2": {"centre": (608, 328, 672, 392), "edge": (1076, 656, 1140, 720)},
    "c3": {"centre": (768, 498, 832, 562), "edge": (1336, 996, 1400, 1060)},
}


def half_bf16_ulp(x: torch.Tensor) -> torch.Tensor:
    """Half the spacing of bfloat16 numbers (8 significant bits) at |x|."""
    e = torch.floor(torch.log2(torch.clamp(x.abs(), min=1e-38)))
    return torch.pow(2.0, e - 8)


def check_adam(label: str, name: str, p0, p, m, v, g_ref, m0, v0, step: int, lr: float, beta1: float = 0.9,
               beta2: float = 0.999, eps: float = 1e-15, tol: float = GRAD_TOL, bf16: bool = False,
               chunk: int = 1 << 20) -> None:
    """One Adam step of the HIP path, (p, m, v) from (p0, m0, v0), against
    adam64 with the oracle gradient g_ref, elementwise.  The bound carries the
    gradient tolerance of the comparison protocol (|g - g_ref| <= tol
    max(|g_ref|, rms)) through the step to first order, plus four float32
    roundings of each moment and eight of the update.  bf16: the parameter is
    stored in bfloat16 and its gradient is rounded to bfloat16 before the
    update (half an ulp each).  Gaussians are compared in chunks of ``chunk``."""
    rows = _gaussian_axis_rows(g_ref.detach().cpu().double())
    live = (rows != 0).any(dim=1)
    rms = float(torch.sqrt((rows[live] ** 2).mean())) if bool(live.any()) else 0.0
    u = 2.0 ** -24
    bc1, bc2 = 1.0 - beta1 ** step, 1.0 - beta2 ** step
    n = rows.shape[0]
    worst = {"p": [0.0, 0.0, 0], "m": [0.0, 0.0, 0], "v": [0.0, 0.0, 0]}
    moved = 0
    for c0 in range(0, n, chunk):
        sl = slice(c0, min(n, c0 + chunk))
        P0, G, M0, V0, Pg, Mg, Vg = (t.detach()[..., sl].float().cpu().double()
                                     for t in (p0, g_ref, m0, v0, p, m, v))
        pr, mr, vr = O.adam64(P0, G, M0, V0, step, lr, beta1, beta2, eps)
        dg = tol * torch.clamp(G.abs(), min=rms)
        if bf16:
            dg = dg + half_bf16_ulp(G)
        mh, vh = mr / bc1, vr / bc2
        D = torch.sqrt(vh) + eps
        dm = (1.0 - beta1) * dg
        dv = (1.0 - beta2) * (2.0 * G.abs() * dg + dg * dg)
        dD = dv / (bc2 * 2.0 * torch.clamp(torch.sqrt(vh), min=1e-300))
        dstep = lr * (dm / (bc1 * D) + mh.abs() * dD / (D * D))
        bm = dm + 4 * u * (mr.abs() + M0.abs() + (1.0 - beta1) * G.abs())
        bv = dv + 4 * u * (vr.abs() + V0.abs() + (1.0 - beta2) * G * G)
        bp = dstep + 8 * u * (pr - P0).abs() + u * pr.abs()
        if bf16:
            bp = bp + half_bf16_ulp(pr)
        for what, got, ref, bound in (("p", Pg, pr, bp), ("m", Mg, mr, bm), ("v", Vg, vr, bv)):
            d = (got - ref).abs()
            if d.numel() == 0:
                continue
            w = worst[what]
            w[0] = max(w[0], float(d.max()))
            w[1] = max(w[1], float((d / torch.clamp(bound, min=1e-300)).max()))
            w[2] += int((d > bound).sum())
        moved += int((Pg != P0).sum())
    say(f"  {label} adam {name:15s} " + " ".join(f"{k}: max abs {a:.2e} worst/bound {r:.2e}"
                                                  for k, (a, r, _) in worst.items())
        + f"; parameters moved {moved / max(1, p.numel()):.3f}")
    for k, (_, _, n_over) in worst.items():
        assert n_over == 0, (label, name, k, worst)
