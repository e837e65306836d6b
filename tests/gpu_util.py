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
