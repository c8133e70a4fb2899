"""Host logic of the window autotuner: cache keys and a cache hit that needs no GPU."""
import json

import paper_2503_01109_amd as F
from paper_2503_01109_amd import autotune
import synth


def test_cache_key_rounds_gaussian_count_up_to_a_power_of_two():
    assert autotune._key("dev", 640, 480, 300_000) == "dev|640x480|n<=524288"
    assert autotune._key("dev", 640, 480, 524_288) == "dev|640x480|n<=524288"
    assert autotune._key("dev", 640, 480, 0) == "dev|640x480|n<=1"


def test_cache_hit_returns_stored_shapes(tmp_path):
    cams = [synth.camera_tum(), synth.camera_replica(), synth.camera_tum()]
    n = 500_000
    db = {autotune._key("fake", 640, 480, n): {"tile": [32, 8]},
          autotune._key("fake", 1200, 680, n): {"tile": [8, 32]},
          autotune._key("fake", 0, 0, n) + "|640x480,1200x680|views=3": {"blocks_per_cu": 8}}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps(db))
    r = autotune.tune_window(F, None, cams, None, n, [None] * 3, cache=str(path), verify=False, device="fake")
    assert r["from_cache"] and r["blocks_per_cu"] == 8
    assert r["tiles"] == [(32, 8), (8, 32), (32, 8)]
