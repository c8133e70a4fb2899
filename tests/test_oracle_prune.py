"""Pins of the oracle's pruning (Sec. III-D, "Gaussian Pruning") against facts that do not come
from the oracle itself: a hand-worked example, the plain definitions (sigmoid below the opacity
threshold, any exp(log-scale) above the size threshold) evaluated with numpy away from the
thresholds, the inclusive side of each threshold, and numpy's boolean indexing as the compaction."""
import numpy as np
import pytest

import oracle


def block(n, seed=0, logit=None, log_scale=None):
    g = np.random.default_rng(seed)
    p = g.normal(size=(14, n))
    if logit is not None:
        p[10] = logit
    if log_scale is not None:
        p[3:6] = log_scale
    return p.astype(np.float32).astype(np.float64)


def test_hand_example():
    """Thresholds opacity 0.1, scale 0.5. Gaussians: opacity 0.5 and scales 0.1 (kept); opacity
    0.05 (removed: faint); opacity 0.9 with one scale 0.6 (removed: too large on one axis);
    opacity 0.2 with two scales equal to the size threshold (kept: not above it); a NaN logit
    (removed)."""
    logit = np.log(np.array([0.5 / 0.5, 0.05 / 0.95, 0.9 / 0.1, 0.2 / 0.8, np.nan]))
    ls = np.log(np.array([[0.1, 0.1, 0.1, 0.5, 0.1], [0.1, 0.1, 0.6, 0.5, 0.1], [0.1, 0.1, 0.1, 0.2, 0.1]]))
    p = block(5, logit=logit, log_scale=ls)
    keep = oracle.prune_keep(p, 0.1, 0.5)
    assert keep.tolist() == [1, 0, 0, 1, 0]


@pytest.mark.parametrize("tau,smax", [(0.005, 0.5), (0.3, 0.05), (0.0, 0.2), (0.01, 0.0), (0.01, np.inf)])
def test_agrees_with_the_plain_definition_away_from_the_thresholds(tau, smax):
    n = 20000
    g = np.random.default_rng(1)
    p = block(n, 2, logit=g.normal(-2, 3, n), log_scale=g.normal(-2.5, 1.0, (3, n)))
    opacity = 1.0 / (1.0 + np.exp(-p[10]))
    scale = np.exp(p[3:6])
    want = opacity >= tau
    if smax > 0 and np.isfinite(smax):
        want &= (scale <= smax).all(axis=0)
        near = (np.abs(scale / smax - 1.0) < 1e-6).any(axis=0)
    else:
        near = np.zeros(n, bool)
    if tau > 0:
        near |= np.abs(opacity / tau - 1.0) < 1e-6
    keep = oracle.prune_keep(p, tau, smax)
    assert 0 < keep[~near].sum() < n
    assert np.array_equal(keep[~near].astype(bool), want[~near])


def test_thresholds_are_inclusive_on_the_kept_side():
    """A logit equal to the converted opacity threshold is kept and the next float below it is not;
    a log-scale equal to the converted size threshold is kept and the next float above is not."""
    L_o, L_s = oracle.prune_thresholds(0.005, 0.5)
    tau = float(np.float32(0.005))  # the thresholds are binary32 values
    assert L_o == float(np.float32(np.log(tau / (1 - tau)))) and L_s == float(np.float32(np.log(0.5)))
    below = float(np.nextafter(np.float32(L_o), np.float32(-np.inf)))
    above = float(np.nextafter(np.float32(L_s), np.float32(np.inf)))
    logit = np.array([L_o, below, 0.0, 0.0])
    ls = np.full((3, 4), -5.0)
    ls[1, 2], ls[2, 3] = L_s, above
    keep = oracle.prune_keep(block(4, logit=logit, log_scale=ls), 0.005, 0.5)
    assert keep.tolist() == [1, 0, 1, 0]


def test_tests_off_and_non_finite_values():
    """min_opacity 0 keeps every finite logit, max_scale 0 or inf keeps every finite log-scale; NaN
    in the logit or any log-scale is removed either way; +inf log-scale is removed by a size test."""
    logit = np.array([-80.0, 3.0, np.nan, 1.0, 1.0])
    ls = np.full((3, 5), 40.0)
    ls[1, 3], ls[0, 4] = np.nan, np.inf
    p = block(5, logit=logit, log_scale=ls)
    assert oracle.prune_keep(p, 0.0, 0.0).tolist() == [1, 1, 0, 0, 1]
    assert oracle.prune_keep(p, 0.0, np.inf).tolist() == [1, 1, 0, 0, 1]
    assert oracle.prune_keep(p, 0.0, 10.0).tolist() == [0, 0, 0, 0, 0]
    with pytest.raises(ValueError):
        oracle.prune_keep(p, 1.0, 0.0)
    with pytest.raises(ValueError):
        oracle.prune_keep(p, 0.1, np.nan)


def test_compaction_is_numpy_boolean_indexing():
    n = 5003
    g = np.random.default_rng(3)
    p = block(n, 4, logit=g.normal(-4, 2, n))
    m, v = g.normal(size=(14, n)), g.uniform(size=(14, n))
    kept, keep, km, kv = oracle.prune(p, 0.01, 0.3, m, v)
    sel = keep.astype(bool)
    assert 0 < sel.sum() < n
    assert np.array_equal(kept, p[:, sel]) and np.array_equal(km, m[:, sel]) and np.array_equal(kv, v[:, sel])


def test_all_kept_none_kept_and_empty():
    p = block(300, 5, logit=np.full(300, 5.0), log_scale=np.full((3, 300), -3.0))
    kept, keep = oracle.prune(p, 0.5, 1.0)
    assert keep.all() and np.array_equal(kept, p)
    kept, keep = oracle.prune(p, 0.999, 1.0)
    assert not keep.any() and kept.shape == (14, 0)
    kept, keep = oracle.prune(np.zeros((14, 0)), 0.5, 1.0)
    assert kept.shape == (14, 0) and keep.shape == (0,)
