"""Tile-size autotuner: picks 8, 16 or 32 pixel tiles for a workload by timing
rasterizer steps, and caches the choice per (Gaussian-count bucket,
pixel-count bucket, view count).

The timing runs the library's forward and backward passes (HIP events on the
current stream); the choice only changes how the image is cut into tiles, not
the result (every tile size gives the same image up to the float32 rounding
of borderline fragments).
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, Optional, Sequence, Tuple

import torch

from . import binding as B

CANDIDATES = (8, 16, 32)


def bucket(n: int, cameras: Sequence) -> Tuple[int, int, int]:
    """(round(log2 N), round(log2 total pixels), views): workloads in one bucket
    share a tile size."""
    pixels = sum(int(c.width) * int(c.height) for c in cameras)
    return (int(round(math.log2(max(n, 1)))), int(round(math.log2(max(pixels, 1)))), len(cameras))


class TileAutotuner:
    """choose(params, cameras) -> tile size.  ``measure(tile) -> ms`` may be
    given to replace the timed steps (tests); ``cache_path`` persists choices
    as JSON."""

    def __init__(self, candidates: Iterable[int] = CANDIDATES, reps: int = 3, cache_path: Optional[str] = None):
        self.candidates = tuple(int(t) for t in candidates)
        for t in self.candidates:
            if t not in CANDIDATES:
                raise ValueError(f"tile {t} not in {CANDIDATES}")
        self.reps = int(reps)
        self.cache_path = cache_path
        self.cache: Dict[str, Dict[str, object]] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    @staticmethod
    def _key(k: Tuple[int, int, int]) -> str:
        return f"{k[0]}:{k[1]}:{k[2]}"

    def time_steps(self, params: Dict[str, torch.Tensor], cameras: Sequence, tile: int,
                   times: Optional[Sequence[float]] = None, settings=None) -> float:
        """Mean ms of a forward + backward pass over the views at this tile size."""
        st = B.default_settings() if settings is None else settings
        st = B.default_settings(**{f: getattr(st, f) for f, _ in st._fields_})
        st.tile = int(tile)
        br = B.BatchRasterizer(cameras, settings=st, times=times)
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
               settings=None, measure: Optional[Callable[[int], float]] = None) -> int:
        n = int(params["opacity_logits"].shape[0])
        key = self._key(bucket(n, cameras))
        if key in self.cache:
            return int(self.cache[key]["tile"])
        timings = {}
        for t in self.candidates:
            timings[t] = float(measure(t) if measure is not None
                               else self.time_steps(params, cameras, t, times, settings))
        best = min(timings, key=lambda t: (timings[t], t))
        self.cache[key] = {"tile": best, "ms": {str(t): v for t, v in timings.items()}}
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return best
