"""Host logic of the learned prior's evaluation: the headline counts and ratios."""
import pytest

from paper_2503_01109_amd import prior


def run(ms, iters=100, seed_ms=0.5, ms_per_iter=0.2, seeds=1000, final_db=30.0):
    return dict(ms=ms, iters=None if ms is None else iters, seed_ms=seed_ms, ms_per_iter=ms_per_iter, seeds=seeds,
                final_db=final_db)


def row(scene, plain, prior_ms, repeat):
    return dict(scene=scene, target_db=29.9, plain=run(plain), prior=run(prior_ms), plain_repeat=run(repeat),
                prior_fraction=0.9)


def test_summary_counts_failures_as_losses_and_needs_a_margin():
    rows = [row(0, 10.0, 8.0, 10.2),   # win: 8 < 10 - 0.2
            row(1, 10.0, 9.95, 10.1),  # within the spread: a loss
            row(2, 10.0, None, 10.0),  # never reached: a loss
            row(3, 10.0, 11.0, 10.0)]  # slower: a loss
    s = prior.summarize(rows)
    assert (s["scenes"], s["wins"], s["losses"], s["prior_never_reached"]) == (4, 1, 3, 1)
    assert s["ms_ratio_median"] == pytest.approx(0.995)
    assert s["prior_ms_mean"] == pytest.approx((8.0 + 9.95 + 11.0) / 3)
    assert s["plain_never_reached"] == 0


def test_a_repeat_short_of_the_target_uses_the_median_spread():
    rows = [row(0, 10.0, 9.0, 10.4), row(1, 10.0, 9.0, 10.2),  # spreads 0.4 and 0.2: median 0.3
            row(2, 10.0, 9.8, None),   # 9.8 > 10 - 0.3: a loss
            row(3, 10.0, 9.6, None)]   # 9.6 < 10 - 0.3: a win
    s = prior.summarize(rows)
    assert (s["wins"], s["losses"], s["repeat_short_of_target"]) == (3, 1, 2)
