"""Host logic of the tile-size autotuner: buckets, choice, cache (no GPU: the
timing function is replaced by a table)."""
import json

import pytest
import torch

import synthetic as S
from paper_2602_09999_amd.autotune import CANDIDATES, TileAutotuner, bucket


def test_buckets_group_similar_workloads():
    cams = [S.identity_camera(1280, 720, 1000.0)] * 2
    assert bucket(1_000_000, cams) == bucket(1_100_000, cams)
    assert bucket(1_000_000, cams) != bucket(4_000_000, cams)
    assert bucket(1_000_000, cams) != bucket(1_000_000, cams[:1])
    assert bucket(1_000_000, cams)[2] == 2


def test_choice_is_the_fastest_and_is_cached(tmp_path):
    params = {"opacity_logits": torch.zeros(5000)}
    cams = [S.identity_camera(640, 480, 500.0)]
    calls = []

    def measure(t):
        calls.append(t)
        return {8: 3.0, 16: 1.5, 32: 2.0}[t]

    path = tmp_path / "tiles.json"
    tuner = TileAutotuner(cache_path=str(path))
    assert tuner.choose(params, cams, measure=measure) == 16
    assert sorted(calls) == sorted(CANDIDATES)
    assert tuner.choose(params, cams, measure=measure) == 16 and len(calls) == 3  # cached
    saved = json.loads(path.read_text())
    assert list(saved.values())[0]["tile"] == 16
    again = TileAutotuner(cache_path=str(path))
    assert again.choose(params, cams, measure=lambda t: 1 / 0) == 16  # loaded, not re-measured
    ties = TileAutotuner()
    assert ties.choose(params, cams, measure=lambda t: 1.0) == 8  # equal times: the smallest tile


def test_rejects_unknown_tile_sizes():
    with pytest.raises(ValueError):
        TileAutotuner(candidates=(8, 12))
