"""Pins of the oracle's adaptive-threshold variant (Section 3.2, the option to
adapt the thresholds instead of correcting the pixels; reading R12): the box
bounds and the gray tolerance are multiplied by the frame's gain 2^16 / inv,
the pixels stay raw. Pinned to exact rational thresholds, to the corrected
masks at unit gain, to scale invariance, to a saturation case where the two
options differ, and end to end on a frame twice as bright as the reference."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle


def _rand(seed, H=16, W=64):
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    lo = rng.integers(0, 200, (H, W, 3))
    bgmin = lo.astype(np.uint8)
    bgmax = np.minimum(255, lo + rng.integers(0, 60, (H, W, 3))).astype(np.uint8)
    return f, bgmin, bgmax


@pytest.mark.parametrize("seed", range(3))
def test_unit_gain_is_the_corrected_masks(seed):
    """At inv = 2^16 the correction is the identity, so both options agree."""
    f, bgmin, bgmax = _rand(seed)
    a = oracle.masks_scaled(f, 65536, bgmin, bgmax)
    b = oracle.masks(f, bgmin, bgmax)
    for k in ("r1", "r2", "r3", "raw"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("k", [2, 4])
def test_a_scaled_frame_meets_scaled_thresholds(k):
    """A frame k times as bright, with inv = 2^16 / k, gives the masks of the
    original frame against the unscaled bounds (hue is scale-invariant)."""
    rng = np.random.default_rng(k)
    u = rng.integers(0, 256 // k, (16, 64, 3))
    _, bgmin, bgmax = _rand(10 + k)
    a = oracle.masks_scaled((k * u).astype(np.uint8), 65536 // k, bgmin, bgmax)
    b = oracle.masks(u.astype(np.uint8), bgmin, bgmax)
    for key in ("r1", "r2", "r3", "raw"):
        assert np.array_equal(a[key], b[key]), key
    assert a["raw"].any() and not a["raw"].all()


@pytest.mark.parametrize("inv", [32768, 45000, 65536, 70001, 131072, 1 << 20])
def test_bounds_are_the_thresholds_times_the_gain(inv):
    """Every channel value against bounds scaled by the exact rational gain."""
    p = oracle.params(bg_delta=7, gray_S=25)
    g = Fraction(65536, inv)
    rng = np.random.default_rng(inv)
    n = 256
    f = np.zeros((1, n, 3), np.uint8)
    f[0, :, 0] = np.arange(n)                        # every value on channel 0
    f[0, :, 1] = rng.integers(0, 256, n)
    f[0, :, 2] = rng.integers(0, 256, n)
    bgmin = rng.integers(0, 150, (1, n, 3)).astype(np.uint8)
    bgmax = np.minimum(255, bgmin.astype(int) + rng.integers(0, 80, (1, n, 3))).astype(np.uint8)
    m = oracle.masks_scaled(f, inv, bgmin, bgmax, p)
    for i in range(n):
        v = [int(c) for c in f[0, i]]
        out = any(not ((int(bgmin[0, i, c]) - 7) * g <= v[c] <= (int(bgmax[0, i, c]) + 7) * g) for c in range(3))
        assert m["r1"][0, i] == out, (i, v)
        assert m["r2"][0, i] == (max(v) - min(v) >= 25 * g), (i, v)
        assert m["r3"][0, i] == oracle.hue_in(*v)


def test_no_saturation_unlike_correction():
    """A dark frame brightened by inv = 2^17: correcting saturates 200 to 255,
    inside a box reaching 250 + delta; scaling keeps 200 above (250 + 10) / 2."""
    f = np.array([[[200, 60, 40]]], np.uint8)
    bgmin = np.array([[[0, 0, 0]]], np.uint8)
    bgmax = np.array([[[250, 250, 250]]], np.uint8)
    corrected = oracle.correct(f, 131072)
    assert corrected[0, 0, 0] == 255
    assert oracle.masks(corrected, bgmin, bgmax)["r1"][0, 0] == 0
    assert oracle.masks_scaled(f, 131072, bgmin, bgmax)["r1"][0, 0] == 1


def _twice_as_bright_scene(W=128, H=48):
    rng = np.random.default_rng(7)
    base = rng.integers(1, 128, (H, W, 3))
    # gray-ish background with a little noise, kept within 1..127
    bg = np.clip(base[None] + rng.integers(-1, 2, (4, H, W, 3)), 1, 127).astype(np.uint8)
    frame = bg[0].copy()
    frame[10:34, 40:80] = (120, 80, 60)              # a skin-hued square (hue 20 degrees)
    return bg, frame


def test_twice_as_bright_gives_the_same_hand():
    bg, frame = _twice_as_bright_scene()
    assert oracle.hue_in(120, 80, 60)
    p = oracle.params(brightness_mode=1)
    m = oracle.Model(bg.shape[2], bg.shape[1], p)
    m.learn(bg)
    a = m.process(frame, want_raw=True)
    b = m.process(2 * frame, want_raw=True)
    # usable pixels of the frame equal the reference's: the gain is exactly 1, then 1/2
    assert a["pointer"]["inv_gain_q16"] == 65536
    assert b["pointer"]["inv_gain_q16"] == 32768
    assert np.array_equal(a["raw"], b["raw"]) and np.array_equal(a["fizi"], b["fizi"])
    pa, pb = dict(a["pointer"]), dict(b["pointer"])
    pa.pop("inv_gain_q16"), pb.pop("inv_gain_q16")
    assert pa == pb and pa["present"] == 1 and pa["area"] == 24 * 40


@pytest.mark.parametrize("seed", range(2))
def test_the_gain_does_not_depend_on_the_option(seed):
    rng = np.random.default_rng(seed)
    H, W = 32, 128
    base = rng.integers(20, 200, (H, W, 3))
    bg = np.clip(base[None] + rng.normal(0, 2, (4, H, W, 3)).round(), 0, 255).astype(np.uint8)
    run = np.clip(base * 0.8 + rng.normal(0, 3, (H, W, 3)).round(), 0, 255).astype(np.uint8)
    outs = []
    for mode in (0, 1):
        m = oracle.Model(W, H, oracle.params(brightness_mode=mode))
        m.learn(bg)
        outs.append(m.process(run))
    assert outs[0]["pointer"]["inv_gain_q16"] == outs[1]["pointer"]["inv_gain_q16"] != 65536
