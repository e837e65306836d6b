"""Autotuner over the rasterizer's tiling, scheduling and blocking: the tile
size (8, 16 or 32 pixels), the blend schedule (one workgroup per tile, or
persistent waves taking tiles from per-XCD queues, FGS_FLAG_BLEND_QUEUE) and
the tile sort's block (4096 or 8192 pairs, FGS_FLAG_SORT_LARGE_BLOCKS),
chosen for a workload by timing rasterizer steps and cached per
(Gaussian-count bucket, pixel-count bucket, view count).

The timing runs the library's forward and backward passes (HIP events on the
current stream).  The search is coordinate-wise: every tile size with the
default schedule and block, then the other schedules at the fastest tile
size, then the other sort blocks at the fastest (tile, schedule).  No choice
changes the result: every tile size gives the same image up to the float32
rounding of borderline fragments, both schedules run the same per-tile code
(the backward's gradient sums differ only in the order of their float
atomics), and both blockings sort stably to the same order.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, Optional, Sequence, Tuple

import torch

from . import _lib as L
from . import binding as B

CANDIDATES = (8, 16, 32)
SCHEDULES = ("grid", "queue")
SORT_BLOCKS = (4096, 8192)


def bucket(n: int, cameras: Sequence) -> Tuple[int, int, int]:
    """(round(log2 N), round(log2 total pixels), views): workloads in one bucket
    share a configuration."""
    pixels = sum(int(c.width) * int(c.height) for c in cameras)
    return (int(round(math.log2(max(n, 1)))), int(round(math.log2(max(pixels, 1)))), len(cameras))


def settings_for(config: Dict[str, object], base=None) -> L.Settings:
    """Settings with the configuration's tile size, blend schedule and sort
    block (other fields from ``base``, else the defaults)."""
    st = B.default_settings() if base is None else base
    st = B.default_settings(**{f: getattr(st, f) for f, _ in st._fields_})
    st.tile = int(config["tile"])
    if config.get("schedule", "grid") == "queue":
        st.flags |= L.FGS_FLAG_BLEND_QUEUE
    else:
        st.flags &= ~L.FGS_FLAG_BLEND_QUEUE
    if int(config.get("sort_block", SORT_BLOCKS[0])) == 8192:
        st.flags |= L.FGS_FLAG_SORT_LARGE_BLOCKS
    else:
        st.flags &= ~L.FGS_FLAG_SORT_LARGE_BLOCKS
    return st


class Autotuner:
    """choose(params, cameras) -> {"tile": t, "schedule": s, "sort_block": b}.
    ``measure(config) -> ms`` may be given to replace the timed steps (tests);
    ``cache_path`` persists choices as JSON."""

    def __init__(self, candidates: Iterable[int] = CANDIDATES, schedules: Iterable[str] = SCHEDULES,
                 sort_blocks: Iterable[int] = SORT_BLOCKS, reps: int = 3, cache_path: Optional[str] = None):
        self.candidates = tuple(int(t) for t in candidates)
        for t in self.candidates:
            if t not in CANDIDATES:
                raise ValueError(f"tile {t} not in {CANDIDATES}")
        self.schedules = tuple(schedules)
        for s in self.schedules:
            if s not in SCHEDULES:
                raise ValueError(f"schedule {s!r} not in {SCHEDULES}")
        if "grid" not in self.schedules:
            raise ValueError("the one-workgroup-per-tile schedule ('grid') is the search's starting point")
        self.sort_blocks = tuple(int(b) for b in sort_blocks)
        for b in self.sort_blocks:
            if b not in SORT_BLOCKS:
                raise ValueError(f"sort block {b} not in {SORT_BLOCKS}")
        if SORT_BLOCKS[0] not in self.sort_blocks:
            raise ValueError(f"the default sort block ({SORT_BLOCKS[0]}) is the search's starting point")
        self.reps = int(reps)
        self.cache_path = cache_path
        self.cache: Dict[str, Dict[str, object]] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    @staticmethod
    def _key(k: Tuple[int, int, int]) -> str:
        return f"{k[0]}:{k[1]}:{k[2]}"

    @staticmethod
    def _name(config: Dict[str, object]) -> str:
        return f"{config['tile']}/{config['schedule']}/{config['sort_block']}"

    def time_steps(self, params: Dict[str, torch.Tensor], cameras: Sequence, config: Dict[str, object],
                   times: Optional[Sequence[float]] = None, settings=None) -> float:
        """Mean ms of a forward + backward pass over the views in this configuration."""
        br = B.BatchRasterizer(cameras, settings=settings_for(config, settings), times=times)
        npix = sum(B.view_pixels(cameras))
        dl = torch.full((3 * npix,), 1e-3, device=br.device)
        grads = {k: torch.empty_like(v) for k, v in params.items()}
        br.forward(params)
        br.backward(params, dl, grads)  # warm-up (and workspace sizing)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(self.reps):
            br.forward(params)
            br.backward(params, dl, grads)
        stop.record()
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / self.reps

    def choose(self, params: Dict[str, torch.Tensor], cameras: Sequence, times: Optional[Sequence[float]] = None,
               settings=None, measure: Optional[Callable[[Dict[str, object]], float]] = None) -> Dict[str, object]:
        n = int(params["opacity_logits"].shape[0])
        key = self._key(bucket(n, cameras))
        if key in self.cache:
            c = self.cache[key]
            return {"tile": int(c["tile"]), "schedule": str(c["schedule"]), "sort_block": int(c["sort_block"])}
        timings: Dict[str, float] = {}

        def run(config):
            ms = float(measure(config) if measure is not None
                       else self.time_steps(params, cameras, config, times, settings))
            timings[self._name(config)] = ms
            return ms

        # tile sizes with one workgroup per tile and the default sort block;
        # equal times: the smaller tile
        b0 = SORT_BLOCKS[0]
        tile_ms = {t: run({"tile": t, "schedule": "grid", "sort_block": b0}) for t in self.candidates}
        best = {"tile": min(tile_ms, key=lambda t: (tile_ms[t], t)), "schedule": "grid", "sort_block": b0}
        best_ms = tile_ms[best["tile"]]
        # the other schedules at that tile size, then the other sort blocks
        # (each kept only when faster)
        for s in self.schedules:
            if s == "grid":
                continue
            config = dict(best, schedule=s)
            ms = run(config)
            if ms < best_ms:
                best, best_ms = config, ms
        for b in self.sort_blocks:
            if b == b0:
                continue
            config = dict(best, sort_block=b)
            ms = run(config)
            if ms < best_ms:
                best, best_ms = config, ms
        self.cache[key] = dict(best, ms=timings)
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return dict(best)


# the tile-size-only name of earlier releases
TileAutotuner = Autotuner
