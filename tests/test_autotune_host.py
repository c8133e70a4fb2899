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


def _fake_results(monkeypatch, g_default, g_tuned, l_default=1.0, l_tuned=1.0):
    import torch
    calls = iter([(torch.tensor([l_default]), g_default), (torch.tensor([l_tuned]), g_tuned)])
    monkeypatch.setattr(autotune, "_window_result", lambda *a, **k: next(calls))


def test_check_against_default_bounds(monkeypatch):
    """Appearance rows are held tightly, geometric rows only to fault-sized bounds, losses to 1e-5."""
    import pytest
    import torch
    gen = torch.Generator().manual_seed(0)
    g0 = torch.randn(14, 1000, generator=gen, dtype=torch.float64)

    def run(g1, l1=1.0):
        _fake_results(monkeypatch, g0.float(), g1.float(), 1.0, l1)
        autotune.check_against_default(F, None, [], [], 0, None, 1000, [], None)

    geo_noise = g0.clone()
    geo_noise[:10] += 5e-4 * torch.randn(10, 1000, generator=gen, dtype=torch.float64)  # summation-order size
    run(geo_noise)
    geo_fault = g0.clone()
    geo_fault[3, :100] = 0.0  # a tenth of one geometric row lost
    with pytest.raises(AssertionError):
        run(geo_fault)
    app_drift = g0.clone()
    app_drift[12] *= 1.0 + 1e-4
    with pytest.raises(AssertionError):
        run(app_drift)
    with pytest.raises(AssertionError):
        run(g0, l1=1.0 + 1e-4)
