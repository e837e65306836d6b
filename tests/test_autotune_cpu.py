"""Host logic of the autotuner over tile size and blend schedule: buckets, the
coordinate search, cache, settings (no GPU: the timing function is replaced
by a table)."""
import json

import pytest
import torch

import synthetic as S
from paper_2602_09999_amd import _lib as L
from paper_2602_09999_amd.autotune import CANDIDATES, SCHEDULES, Autotuner, bucket, settings_for


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
    table = {(8, "grid"): 3.0, (16, "grid"): 1.5, (32, "grid"): 2.0, (16, "queue"): 1.2,
             (8, "queue"): 0.1, (32, "queue"): 0.1}  # never measured: only the best tile tries a queue

    def measure(c):
        calls.append((c["tile"], c["schedule"]))
        return table[(c["tile"], c["schedule"])]

    path = tmp_path / "tiles.json"
    tuner = Autotuner(cache_path=str(path))
    assert tuner.choose(params, cams, measure=measure) == {"tile": 16, "schedule": "queue"}
    assert sorted(calls) == sorted([(t, "grid") for t in CANDIDATES] + [(16, "queue")])
    assert tuner.choose(params, cams, measure=measure)["tile"] == 16 and len(calls) == 4  # cached
    saved = json.loads(path.read_text())
    entry = list(saved.values())[0]
    assert entry["tile"] == 16 and entry["schedule"] == "queue" and entry["ms"]["16/queue"] == 1.2
    again = Autotuner(cache_path=str(path))
    assert again.choose(params, cams, measure=lambda c: 1 / 0)["schedule"] == "queue"  # loaded, not re-measured
    # equal times: the smallest tile, and the queue only when strictly faster
    assert Autotuner().choose(params, cams, measure=lambda c: 1.0) == {"tile": 8, "schedule": "grid"}
    assert Autotuner(schedules=("grid",)).choose(params, cams, measure=measure) == {"tile": 16, "schedule": "grid"}


def test_settings_carry_tile_and_schedule():
    st = settings_for({"tile": 32, "schedule": "queue"})
    assert st.tile == 32 and st.flags & L.FGS_FLAG_BLEND_QUEUE
    base = settings_for({"tile": 8, "schedule": "queue"})
    base.flags |= L.FGS_FLAG_FP64_CONIC
    st = settings_for({"tile": 16, "schedule": "grid"}, base)
    assert st.tile == 16 and not st.flags & L.FGS_FLAG_BLEND_QUEUE and st.flags & L.FGS_FLAG_FP64_CONIC
    assert base.tile == 8  # the base is not modified


def test_rejects_unknown_candidates():
    with pytest.raises(ValueError):
        Autotuner(candidates=(8, 12))
    with pytest.raises(ValueError):
        Autotuner(schedules=("grid", "stealing"))
    with pytest.raises(ValueError):
        Autotuner(schedules=("queue",))
    assert SCHEDULES == ("grid", "queue")
