"""Pins of the oracle's partial re-learning (Section 3.3, reading R9): frames
widen the model only at pixels their I_FIZI marks as background. Pinned to
the (separately pinned) learning function and to pixel independence."""
import numpy as np
import pytest

from oracle import oracle


def _scene(W=128, H=24, n_bg=4, n_run=3, seed=0):
    rng = np.random.default_rng(seed)
    base = rng.integers(30, 220, (1, H, W, 3))
    bg = np.clip(base + rng.normal(0, 2, (n_bg, H, W, 3)).round(), 0, 255).astype(np.uint8)
    # running frames: brighter, noisier, with a drift the box does not hold
    run = np.clip(base * 1.1 + 6 + rng.normal(0, 4, (n_run, H, W, 3)).round(), 0, 255).astype(np.uint8)
    masks = (rng.random((n_run, H, W)) < 0.3).astype(np.uint8)
    return bg, run, masks


def _learned(bg, p=None):
    m = oracle.Model(bg.shape[2], bg.shape[1], p)
    m.learn(bg)
    return m


def test_all_masked_leaves_the_model():
    bg, run, masks = _scene()
    m = _learned(bg)
    before = (m.bgmin.copy(), m.bgmax.copy(), m.yref.copy())
    m.relearn(run, np.ones_like(masks))
    assert np.array_equal(m.bgmin, before[0]) and np.array_equal(m.bgmax, before[1])
    assert np.array_equal(m.yref, before[2])


def test_nothing_masked_is_incremental_learning():
    bg, run, masks = _scene(seed=1)
    a, b = _learned(bg), _learned(bg)
    inv_a = a.relearn(run, np.zeros_like(masks))
    inv_b = b.learn(run, reset=False)
    assert np.array_equal(a.bgmin, b.bgmin) and np.array_equal(a.bgmax, b.bgmax)
    assert np.array_equal(inv_a, inv_b)
    assert not np.array_equal(a.bgmax, _learned(bg).bgmax)      # the drift did widen it


@pytest.mark.parametrize("seed", [2, 3])
def test_pixels_are_independent(seed):
    """With one frame and mask M, every unmasked pixel gets exactly what
    unmasked learning gives it, every masked pixel keeps the old model."""
    bg, run, masks = _scene(seed=seed, n_run=1)
    old = _learned(bg)
    full = _learned(bg)
    full.learn(run, reset=False)
    part = _learned(bg)
    part.relearn(run, masks)
    M = masks[0].astype(bool)[..., None]
    assert np.array_equal(part.bgmin, np.where(M, old.bgmin, full.bgmin))
    assert np.array_equal(part.bgmax, np.where(M, old.bgmax, full.bgmax))


def test_frame_order_does_not_matter():
    bg, run, masks = _scene(seed=4, n_run=4)
    a, b = _learned(bg), _learned(bg)
    a.relearn(run, masks)
    b.relearn(run[::-1].copy(), masks[::-1].copy())
    assert np.array_equal(a.bgmin, b.bgmin) and np.array_equal(a.bgmax, b.bgmax)


def test_own_background_frame_changes_nothing():
    """A learning frame seen again lies inside the box wherever it is not masked."""
    bg, run, masks = _scene(seed=5)
    m = _learned(bg)
    lo, hi = m.bgmin.copy(), m.bgmax.copy()
    m.relearn(bg[1:3], np.zeros((2,) + bg.shape[1:3], np.uint8))
    assert np.array_equal(m.bgmin, lo) and np.array_equal(m.bgmax, hi)


def test_needs_a_learned_model():
    m = oracle.Model(64, 8)
    with pytest.raises(ValueError):
        m.relearn(np.zeros((1, 8, 64, 3), np.uint8), np.zeros((1, 8, 64), np.uint8))
