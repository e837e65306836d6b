"""FP32 reference for instance keys, the two-stage sort order and tile ranges.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Definition followed (Faster-GS, Sec. 3.2 "Splat Bounding", "Tile-based
Culling", "Sorting"; App. B.2 "Separate Sorting"):

* A Gaussian is bounded by the opacity-aware rectangle centred at mu2D with
  half-extents sqrt(2 ln(o / tau_alpha) * Sigma_ii) of the dilated 2D
  covariance (the extent where alpha can reach tau_alpha).
* Each 16x16 tile inside the rectangle is kept only if the Gaussian reaches
  tau_alpha somewhere in it: the minimum of d^T Sigma^-1 d over the tile's
  pixel-centre hull (restricted to pixels inside the image) is compared with
  2 ln(o / tau_alpha).  The minimum is 0 when mu2D lies in the hull, else it
  is found on the hull edges that face mu2D (a clamped 1-D quadratic each,
  whose minimiser -(b d) / c is formed with the reciprocal of c, or of a,
  rounded once).
* Every kept (tile, Gaussian) pair is an instance.  The per-tile lists are
  ordered by depth: the paper sorts visible Gaussians by a 32-bit depth key
  and then stably by tile, which yields the lexicographic order
  (tile, depth key, Gaussian index) -- the index breaks depth ties.
* Tile ranges are [start, end) offsets of each tile's list.

These integer decisions are taken in FP32, the precision of the kernel, one
operation at a time with no fused multiply-add, in the order written below.
Transcendental functions (exp, log) may differ by an ulp between this numpy
code and the GPU, so ``keys_ref_banded`` also returns the instances that flip
when the thresholds move by a relative ``delta``: pairs outside that band
must match exactly; pairs inside it may go either way.

The depth key is the FP32 camera-space z computed as
((W20*x + W21*y) + W22*z) + W23 -- no transcendental, so it is exact.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np
import torch

f32 = np.float32

TAU_ALPHA = f32(1.0 / 255.0)
ALPHA_MAX = f32(0.99)
T_MIN = f32(1e-4)
DILATION = f32(0.3)
QUAT_MIN = f32(1e-4)
DET_MIN = f32(1e-6)


def _np32(t) -> np.ndarray:
    if isinstance(t, torch.Tensor):
        t = t.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(t, dtype=np.float32))


def depth_key32(means, cam) -> np.ndarray:
    """FP32 camera-space depth ((W20*x + W21*y) + W22*z) + W23 per Gaussian."""
    m = _np32(means)
    W = np.asarray(cam.world_to_cam, dtype=np.float32)
    with np.errstate(all="ignore"):
        return ((W[2, 0] * m[0] + W[2, 1] * m[1]) + W[2, 2] * m[2]) + W[2, 3]


def cond_inputs32(scene: Dict[str, torch.Tensor], time: float) -> Dict[str, np.ndarray]:
    """Conditional 4D Gaussians (Sec. 3.4) at ``time``: the conditional mean
    [3, N], covariance entries and marginal factor [N] computed in float64 by
    the oracle (``cond4d64``) and rounded to float32, as inputs of
    ``record32``.  The kernel conditions in float32; the differences (a few
    ulps) move decisions only inside the borderline band."""
    from .cond4d64 import condition, rows4
    rows = {k: (v.detach().to(torch.float64).T.contiguous() if v.dim() == 2 else v.detach().to(torch.float64))
            for k, v in scene.items()}
    with torch.no_grad():
        mean3, cov3, p = condition(*rows4(rows), float(time))
    return {"means": mean3.T.numpy().astype(np.float32),
            "cov": {(i, j): cov3[:, i, j].numpy().astype(np.float32) for i in range(3) for j in range(3)},
            "p": p.numpy().astype(np.float32),
            "qn_r": np.sqrt((rows["quats_r"] ** 2).sum(1)).numpy().astype(np.float32)}


def record32(scene: Dict[str, torch.Tensor], cam, *, thr_scale: float = 1.0,
             cull_slack: float = 0.0, dilation=DILATION, tau=TAU_ALPHA,
             det_min=DET_MIN, quat_min=QUAT_MIN, fp64_conic: bool = False,
             cond: Optional[Dict[str, np.ndarray]] = None) -> Dict[str, np.ndarray]:
    """FP32 per-Gaussian quantities that decide the instance keys.

    thr_scale multiplies the truncation threshold (used for the borderline
    band); cull_slack > 0 loosens, < 0 tightens each cull comparison by that
    relative amount.  fp64_conic: the precision form's determinant and 2x2
    inverse in float64 from the float32 entries (products exact, one rounding
    per subtraction and per division), the conic rounded to float32.
    cond: ``cond_inputs32`` of conditional 4D Gaussians, whose mean and 3D
    covariance replace those of the raw parameters and whose marginal factor
    multiplies the opacity.
    """
    with np.errstate(all="ignore"):
        mu = _np32(scene["means"]) if cond is None else cond["means"]
        ls = _np32(scene["log_scales"])
        q = _np32(scene["quats"])
        logit = _np32(scene["opacity_logits"])
        W = np.asarray(cam.world_to_cam, dtype=np.float32)
        fx, fy, cx, cy = f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy)
        near = f32(cam.near)

        s0, s1, s2 = np.exp(ls[0]), np.exp(ls[1]), np.exp(ls[2])
        n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]
        qn = np.sqrt(n2)
        w, x, y, z = q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn
        xx, yy, zz = x * x, y * y, z * z
        xy, xz, yz = x * y, x * z, y * z
        wx, wy, wz = w * x, w * y, w * z
        one, two = f32(1.0), f32(2.0)
        r = [[one - two * (yy + zz), two * (xy - wz), two * (xz + wy)],
             [two * (xy + wz), one - two * (xx + zz), two * (yz - wx)],
             [two * (xz - wy), two * (yz + wx), one - two * (xx + yy)]]
        s = (s0, s1, s2)
        m = [[r[i][j] * s[j] for j in range(3)] for i in range(3)]

        def sig(i, j):
            return (m[i][0] * m[j][0] + m[i][1] * m[j][1]) + m[i][2] * m[j][2]
        S = {(0, 0): sig(0, 0), (0, 1): sig(0, 1), (0, 2): sig(0, 2),
             (1, 1): sig(1, 1), (1, 2): sig(1, 2), (2, 2): sig(2, 2)}
        S[(1, 0)], S[(2, 0)], S[(2, 1)] = S[(0, 1)], S[(0, 2)], S[(1, 2)]
        if cond is not None:
            S = dict(cond["cov"])
            qn = np.minimum(qn, cond["qn_r"])

        X = ((W[0, 0] * mu[0] + W[0, 1] * mu[1]) + W[0, 2] * mu[2]) + W[0, 3]
        Y = ((W[1, 0] * mu[0] + W[1, 1] * mu[1]) + W[1, 2] * mu[2]) + W[1, 3]
        Z = ((W[2, 0] * mu[0] + W[2, 1] * mu[1]) + W[2, 2] * mu[2]) + W[2, 3]
        iz = one / Z
        u, v = X * iz, Y * iz
        mx = fx * u + cx
        my = fy * v + cy
        j00, j11 = fx * iz, fy * iz
        j02, j12 = -(j00 * u), -(j11 * v)
        T0 = [j00 * W[0, k] + j02 * W[2, k] for k in range(3)]
        T1 = [j11 * W[1, k] + j12 * W[2, k] for k in range(3)]
        U0 = [(T0[0] * S[(0, k)] + T0[1] * S[(1, k)]) + T0[2] * S[(2, k)] for k in range(3)]
        U1 = [(T1[0] * S[(0, k)] + T1[1] * S[(1, k)]) + T1[2] * S[(2, k)] for k in range(3)]
        c00 = (U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2]
        c01 = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2]
        c11 = (U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2]
        det = c00 * c11 - c01 * c01
        h00 = c00 + dilation
        h11 = c11 + dilation
        h01 = c01
        if fp64_conic:
            d = np.float64
            det_d = c00.astype(d) * c11.astype(d) - c01.astype(d) * c01.astype(d)
            deth_d = h00.astype(d) * h11.astype(d) - h01.astype(d) * h01.astype(d)
            ca = (h11.astype(d) / deth_d).astype(np.float32)
            cb = (-h01.astype(d) / deth_d).astype(np.float32)
            cc = (h00.astype(d) / deth_d).astype(np.float32)
        else:
            deth = h00 * h11 - h01 * h01
            ca = h11 / deth
            cb = -h01 / deth
            cc = h00 / deth
        o = one / (one + np.exp(-logit))
        if cond is not None:
            o = o * cond["p"]

        lo, hi = f32(1.0 - cull_slack), f32(1.0 + cull_slack)
        det_ok = (det_d >= np.float64(det_min * lo)) if fp64_conic else (det >= det_min * lo)
        valid = ((qn >= quat_min * lo) & (Z >= near * lo) & det_ok & (o > tau * lo))
        thr = (two * np.log(o / tau)) * f32(thr_scale)
        ext_x = np.sqrt(thr * h00)
        ext_y = np.sqrt(thr * h11)
        valid &= (ext_x >= 0) & (ext_y >= 0) & np.isfinite(mx) & np.isfinite(my)
        valid &= np.isfinite(ca) & np.isfinite(cb) & np.isfinite(cc)
        del hi
    return {"mx": mx, "my": my, "a": ca, "b": cb, "c": cc, "thr": thr, "ext_x": ext_x,
            "ext_y": ext_y, "depth": Z, "valid": valid, "opacity": o, "det": det,
            "h00": h00, "h11": h11}


def tile_rect(rec: Dict[str, np.ndarray], width: int, height: int, tile: int):
    """Inclusive tile bounds (tx0, ty0, tx1, ty1) of the opacity-aware rectangle,
    from the pixel-centre index range [ceil(m - e - 0.5), floor(m + e - 0.5)]
    clipped to the image; ``nonempty`` is False when it misses the image."""
    with np.errstate(all="ignore"):
        half = f32(0.5)
        lx = (rec["mx"] - rec["ext_x"]) - half
        hx = (rec["mx"] + rec["ext_x"]) - half
        ly = (rec["my"] - rec["ext_y"]) - half
        hy = (rec["my"] + rec["ext_y"]) - half
        wm1, hm1 = f32(width - 1), f32(height - 1)
        nonempty = rec["valid"] & (hx >= 0) & (lx <= wm1) & (hy >= 0) & (ly <= hm1)
        i0 = np.where(lx <= 0, 0, np.ceil(np.where(nonempty, lx, 0))).astype(np.int64)
        i1 = np.where(hx >= wm1, width - 1, np.floor(np.where(nonempty, hx, 0))).astype(np.int64)
        j0 = np.where(ly <= 0, 0, np.ceil(np.where(nonempty, ly, 0))).astype(np.int64)
        j1 = np.where(hy >= hm1, height - 1, np.floor(np.where(nonempty, hy, 0))).astype(np.int64)
    nonempty &= (i0 <= i1) & (j0 <= j1)
    return i0 // tile, j0 // tile, i1 // tile, j1 // tile, nonempty


def _edge_q(a, b, c, dfix, m_other, lo, hi, first_is_x: bool):
    """Minimum of the quadratic form along one hull edge (FP32, fixed order).

    The unconstrained minimiser along the edge is -(b d) / c (vertical edge)
    or -(b d) / a (horizontal edge); it is taken as -(b d) times the
    reciprocal 1/c (1/a), the reciprocal rounded once per Gaussian."""
    one = np.float32(1.0)
    if first_is_x:
        t = -(b * dfix) * (one / c)
    else:
        t = -(b * dfix) * (one / a)
    p = np.minimum(np.maximum(m_other + t, lo), hi)
    dvar = p - m_other
    if first_is_x:
        dx, dy = dfix, dvar
    else:
        dx, dy = dvar, dfix
    return ((a * dx) * dx + ((b + b) * dx) * dy) + (c * dy) * dy


def tile_min_q(mx, my, a, b, c, tx, ty, width: int, height: int, tile: int) -> np.ndarray:
    """Min over the tile's pixel-centre hull of d^T [[a,b],[b,c]] d (FP32)."""
    with np.errstate(all="ignore"):
        half = f32(0.5)
        x0 = (tx * tile).astype(np.float32) + half
        x1 = np.minimum(tx * tile + tile - 1, width - 1).astype(np.float32) + half
        y0 = (ty * tile).astype(np.float32) + half
        y1 = np.minimum(ty * tile + tile - 1, height - 1).astype(np.float32) + half
        inf = np.full_like(mx, np.inf)
        q = inf.copy()
        left, right = mx < x0, mx > x1
        top, bottom = my < y0, my > y1
        qe = _edge_q(a, b, c, x0 - mx, my, y0, y1, True)
        q = np.where(left, np.minimum(q, qe), q)
        qe = _edge_q(a, b, c, x1 - mx, my, y0, y1, True)
        q = np.where(right, np.minimum(q, qe), q)
        qe = _edge_q(a, b, c, y0 - my, mx, x0, x1, False)
        q = np.where(top, np.minimum(q, qe), q)
        qe = _edge_q(a, b, c, y1 - my, mx, x0, x1, False)
        q = np.where(bottom, np.minimum(q, qe), q)
        inside = ~(left | right | top | bottom)
        q = np.where(inside, np.float32(0.0), q)
    return q.astype(np.float32)


def _instances(rec, width, height, tile, ext_scale: float = 1.0, chunk: int = 1 << 22):
    """All kept (gaussian, tile) pairs in Gaussian order, row-major tiles within each."""
    r = dict(rec)
    if ext_scale != 1.0:
        r["ext_x"] = rec["ext_x"] * f32(ext_scale)
        r["ext_y"] = rec["ext_y"] * f32(ext_scale)
    tx0, ty0, tx1, ty1, ne = tile_rect(r, width, height, tile)
    tiles_x = (width + tile - 1) // tile
    wt = np.where(ne, tx1 - tx0 + 1, 0)
    ht = np.where(ne, ty1 - ty0 + 1, 0)
    cnt = wt * ht
    gids, tids = [], []
    ids = np.nonzero(cnt)[0]
    # chunk over Gaussians so that the pair arrays stay bounded
    start = 0
    csum = np.cumsum(cnt[ids])
    while start < len(ids):
        base = csum[start - 1] if start else 0
        stop = int(np.searchsorted(csum, base + chunk, side="right"))
        stop = max(stop, start + 1)
        sel = ids[start:stop]
        c = cnt[sel]
        g = np.repeat(sel, c)
        off = np.repeat(np.cumsum(c) - c, c)
        local = np.arange(int(c.sum()), dtype=np.int64) - off
        tx = tx0[g] + local % wt[g]
        ty = ty0[g] + local // wt[g]
        qmin = tile_min_q(rec["mx"][g], rec["my"][g], rec["a"][g], rec["b"][g], rec["c"][g],
                          tx, ty, width, height, tile)
        keep = qmin <= rec["thr"][g]
        gids.append(g[keep])
        tids.append((ty * tiles_x + tx)[keep])
        start = stop
    if gids:
        return np.concatenate(gids).astype(np.int64), np.concatenate(tids).astype(np.int64)
    return np.zeros(0, np.int64), np.zeros(0, np.int64)


def _sort_instances(gid, tid, depth, n_tiles_total):
    dbits = depth.view(np.uint32).astype(np.int64)
    order = np.lexsort((gid, dbits[gid], tid))
    keys = tid[order].astype(np.uint32)
    vals = gid[order].astype(np.uint32)
    ranges = np.zeros((n_tiles_total, 2), np.uint32)
    if len(keys):
        bounds = np.flatnonzero(np.diff(keys.astype(np.int64))) + 1
        starts = np.concatenate([[0], bounds])
        ends = np.concatenate([bounds, [len(keys)]])
        ranges[keys[starts], 0] = starts
        ranges[keys[starts], 1] = ends
    return keys, vals, ranges


def keys_ref(scene: Dict[str, torch.Tensor], cam, tile: int = 16, thr_scale: float = 1.0,
             cull_slack: float = 0.0, fp64_conic: bool = False, time: Optional[float] = None,
             depth: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Sorted instance keys (tile id), values (Gaussian index), tile ranges [tiles, 2],
    per-Gaussian tile counts and the FP32 record they were derived from.
    time: conditional 4D Gaussians at that time; depth: FP32 depth keys for
    the order (else the record's)."""
    rec = record32(scene, cam, thr_scale=thr_scale, cull_slack=cull_slack, fp64_conic=fp64_conic,
                   cond=cond_inputs32(scene, time) if "quats_r" in scene else None)
    if depth is not None:
        rec = dict(rec, depth=np.asarray(depth, dtype=np.float32))
    w, h = int(cam.width), int(cam.height)
    gid, tid = _instances(rec, w, h, tile)  # the extents already carry thr_scale
    tiles = ((w + tile - 1) // tile) * ((h + tile - 1) // tile)
    keys, vals, ranges = _sort_instances(gid, tid, rec["depth"], tiles)
    n = rec["mx"].shape[0]
    n_tiles = np.bincount(gid, minlength=n).astype(np.uint32) if len(gid) else np.zeros(n, np.uint32)
    return {"keys": keys, "vals": vals, "ranges": ranges, "n_tiles": n_tiles, "record": rec,
            "depth": rec["depth"], "tiles_x": (w + tile - 1) // tile,
            "tiles_y": (h + tile - 1) // tile}


def keys_ref_banded(scene, cam, tile: int = 16, delta: float = 1e-3, fp64_conic: bool = False,
                    time: Optional[float] = None, depth: Optional[np.ndarray] = None):
    """Nominal instances plus the borderline pairs: those present with every
    threshold loosened by ``delta`` (relative) but absent with every threshold
    tightened by ``delta``.  Returns (nominal, borderline_pairs) where
    borderline_pairs is a set of (tile, gaussian) tuples."""
    kw = dict(fp64_conic=fp64_conic, time=time, depth=depth)
    nom = keys_ref(scene, cam, tile, **kw)
    loose = keys_ref(scene, cam, tile, thr_scale=1.0 + delta, cull_slack=delta, **kw)
    tight = keys_ref(scene, cam, tile, thr_scale=1.0 - delta, cull_slack=-delta, **kw)
    lo_pairs = set(zip(tight["keys"].tolist(), tight["vals"].tolist()))
    hi_pairs = set(zip(loose["keys"].tolist(), loose["vals"].tolist()))
    return nom, hi_pairs - lo_pairs


def tile_lists_for(scene, cam, tiles, tile: int = 16, delta: Optional[float] = None, time: Optional[float] = None,
                   depth: Optional[np.ndarray] = None):
    """Reference list of Gaussian indices (canonical order) for a few tile ids,
    without materialising every instance -- for full-size spot checks.
    With ``delta`` also returns the borderline Gaussians of each tile.
    time: conditional 4D Gaussians at that time; depth: FP32 depth keys for
    the order (else the record's)."""
    rec = record32(scene, cam, cond=cond_inputs32(scene, time) if "quats_r" in scene else None)
    if depth is not None:
        rec = dict(rec, depth=np.asarray(depth, dtype=np.float32))
    w, h = int(cam.width), int(cam.height)
    tiles_x = (w + tile - 1) // tile
    tx0, ty0, tx1, ty1, ne = tile_rect(rec, w, h, tile)
    out = {}
    for t in tiles:
        tx, ty = int(t) % tiles_x, int(t) // tiles_x
        cand = np.nonzero(ne & (tx0 <= tx) & (tx <= tx1) & (ty0 <= ty) & (ty <= ty1))[0]
        q = tile_min_q(rec["mx"][cand], rec["my"][cand], rec["a"][cand], rec["b"][cand],
                       rec["c"][cand], np.full(len(cand), tx), np.full(len(cand), ty), w, h, tile)
        keep = cand[q <= rec["thr"][cand]]
        dbits = rec["depth"].view(np.uint32).astype(np.int64)
        lst = keep[np.lexsort((keep, dbits[keep]))]
        if delta is None:
            out[int(t)] = lst
        else:
            thr = rec["thr"][cand].astype(np.float64)
            band = np.abs(q.astype(np.float64) - thr) <= delta * np.maximum(np.abs(thr), 1e-6)
            out[int(t)] = (lst, set(cand[band].tolist()))
    return out
