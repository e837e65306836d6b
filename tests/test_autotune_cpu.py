"""Host logic of the autotuner over tile size, blend schedule and sort block:
buckets, the coordinate search, cache, settings (no GPU: the timing function
is replaced by a table)."""
import json

import pytest
import torch

import synthetic as S
from paper_2602_09999_amd import _lib as L
from paper_2602_09999_amd.autotune import CANDIDATES, SCHEDULES, SORT_BLOCKS, Autotuner, bucket, settings_for


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
    # only the best tile tries a queue, and only the best (tile, schedule) the large sort block
    table = {(8, "grid", 4096): 3.0, (16, "grid", 4096): 1.5, (32, "grid", 4096): 2.0, (16, "queue", 4096): 1.2,
             (16, "queue", 8192): 1.1, (8, "queue", 4096): 0.1, (32, "queue", 4096): 0.1, (16, "grid", 8192): 0.1}

    def measure(c):
        calls.append((c["tile"], c["schedule"], c["sort_block"]))
        return table[calls[-1]]

    path = tmp_path / "tiles.json"
    tuner = Autotuner(cache_path=str(path))
    best = {"tile": 16, "schedule": "queue", "sort_block": 8192}
    assert tuner.choose(params, cams, measure=measure) == best
    assert sorted(calls) == sorted([(t, "grid", 4096) for t in CANDIDATES] + [(16, "queue", 4096),
                                                                               (16, "queue", 8192)])
    assert tuner.choose(params, cams, measure=measure) == best and len(calls) == 5  # cached
    saved = json.loads(path.read_text())
    entry = list(saved.values())[0]
    assert entry["tile"] == 16 and entry["schedule"] == "queue" and entry["ms"]["16/queue/4096"] == 1.2
    again = Autotuner(cache_path=str(path))
    assert again.choose(params, cams, measure=lambda c: 1 / 0) == best  # loaded, not re-measured
    # equal times: the smallest tile, the queue and the large block only when strictly faster
    assert Autotuner().choose(params, cams, measure=lambda c: 1.0) == {"tile": 8, "schedule": "grid",
                                                                       "sort_block": 4096}
    assert Autotuner(schedules=("grid",), sort_blocks=(4096,)).choose(params, cams, measure=measure) == {
        "tile": 16, "schedule": "grid", "sort_block": 4096}


def test_settings_carry_tile_schedule_and_sort_block():
    st = settings_for({"tile": 32, "schedule": "queue", "sort_block": 8192})
    assert st.tile == 32 and st.flags & L.FGS_FLAG_BLEND_QUEUE and st.flags & L.FGS_FLAG_SORT_LARGE_BLOCKS
    base = settings_for({"tile": 8, "schedule": "queue", "sort_block": 8192})
    base.flags |= L.FGS_FLAG_FP64_CONIC
    st = settings_for({"tile": 16, "schedule": "grid", "sort_block": 4096}, base)
    assert st.tile == 16 and st.flags == L.FGS_FLAG_FP64_CONIC
    assert base.tile == 8  # the base is not modified


def test_rejects_unknown_candidates():
    with pytest.raises(ValueError):
        Autotuner(candidates=(8, 12))
    with pytest.raises(ValueError):
        Autotuner(schedules=("grid", "stealing"))
    with pytest.raises(ValueError):
        Autotuner(schedules=("queue",))
    with pytest.raises(ValueError):
        Autotuner(sort_blocks=(4096, 2048))
    with pytest.raises(ValueError):
        Autotuner(sort_blocks=(8192,))
    assert SCHEDULES == ("grid", "queue") and SORT_BLOCKS == (4096, 8192)
