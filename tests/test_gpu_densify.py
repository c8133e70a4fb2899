"""The densification ablation driver (Sec. III-A, Table 6 analogue) on one synthetic 640x480
frame with a short mapping run: the five seedings differ only where they should (strides set the
count, radius factors do not), pruning never grows the map, and the reported memory follows the
count."""
import math

import numpy as np
import pytest

from gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


def test_ablation_variants_on_one_frame():
    need_gpu()
    import paper_2503_01109_amd as F
    from paper_2503_01109_amd import densify
    ctx = F.Context()
    try:
        r = densify.run(F, ctx, [2000], iters=40, prune_every=20)
    finally:
        ctx.close()
    s = {row["variant"]: row for row in r["rows"]}
    for row in r["rows"]:
        print(row)
    assert s["sparse_large"]["seeded"] == s["sparse_small"]["seeded"]
    assert s["dense_large"]["seeded"] == s["dense_small"]["seeded"]
    assert s["sparse_large"]["seeded"] < s["adaptive"]["seeded"] < s["dense_large"]["seeded"]
    for row in r["rows"]:
        k = row["kept_after_each_prune"]
        assert len(k) == 2 and k[0] <= row["seeded"] and k[1] <= k[0] and k[1] == row["kept"]
        assert row["map_mb"] == pytest.approx(row["kept"] * 56 / 1e6)
        assert row["map_with_adam_mb"] == pytest.approx(row["kept"] * 168 / 1e6)
        assert math.isfinite(row["psnr_db"]) and 0.0 < row["ssim"] <= 1.0
        assert row["ms_per_iter"] > 0
    assert set(r["summary"]) == set(densify.VARIANTS)
    # the seedings that cover the frame (small gaussians on the sparse lattice leave most of it
    # empty after a short run: measured 7 dB)
    for v in ("dense_small", "adaptive"):
        assert s[v]["psnr_db"] > 25.0, (v, s[v]["psnr_db"])
