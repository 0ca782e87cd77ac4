"""Pins of the oracle's over-exposure filter (Section 3.2: an over-exposed
hand looks white and is removed as gray, so the Luminosity component is
modified in the most obvious cases; reading R14): with lum_hi > 0, a pixel
whose HSL lightness exceeds lum_hi / 255 has it brought down to lum_hi / 255,
hue and HSL saturation kept, and the gray test I_R2 sees the result.
Pinned to the textbook HLS conversion of Python's colorsys, to special
cases, and end to end on an over-exposed hand."""
import colorsys

import numpy as np
import pytest

from oracle import oracle


def _colorsys_chroma(r, g, b, lum_hi):
    """Chroma (x 255) after lowering the HLS lightness to lum_hi / 255."""
    h, l, s = colorsys.rgb_to_hls(r / 255.0, g / 255.0, b / 255.0)
    if lum_hi and l > lum_hi / 255.0:
        rr, gg, bb = colorsys.hls_to_rgb(h, lum_hi / 255.0, s)
        return (max(rr, gg, bb) - min(rr, gg, bb)) * 255.0
    return float(max(r, g, b) - min(r, g, b))


@pytest.mark.parametrize("lum_hi", [128, 160, 191, 230, 254])
def test_filtered_chroma_is_the_hls_conversion(lum_hi):
    rng = np.random.default_rng(lum_hi)
    px = rng.integers(0, 256, size=(20000, 3))
    # bias half of them towards over-exposure
    px[::2] = 255 - rng.integers(0, 40, size=(10000, 3))
    for r, g, b in px.tolist():
        n, d = oracle.filtered_chroma(r, g, b, lum_hi)
        assert d > 0
        want = _colorsys_chroma(r, g, b, lum_hi)
        assert abs(n / d - want) <= 1e-9 * max(1.0, want), (r, g, b, n, d, want)


def test_special_cases():
    assert oracle.filtered_chroma(255, 255, 255, 191) == (0, 1)        # white stays white
    n, d = oracle.filtered_chroma(230, 230, 230, 191)                   # gray stays gray
    assert n == 0
    assert oracle.filtered_chroma(120, 80, 60, 191) == (60, 1)          # L = 90/255 <= lum_hi: unchanged
    assert oracle.filtered_chroma(252, 244, 238, 0) == (14, 1)          # filter off
    # (252, 244, 238): L2 = 490 > 382; C' = 14 * (510 - 382) / (510 - 490) = 89.6
    assert oracle.filtered_chroma(252, 244, 238, 191) == (14 * 128, 20)
    # at the threshold itself: max + min = 2 lum_hi is not over-exposed
    assert oracle.filtered_chroma(200, 182, 172, 186) == (28, 1)
    assert oracle.filtered_chroma(200, 182, 173, 186) == (27 * (510 - 372), 510 - 373)


def test_lowering_the_lightness_raises_the_chroma():
    rng = np.random.default_rng(7)
    for r, g, b in (255 - rng.integers(0, 60, size=(5000, 3))).tolist():
        n, d = oracle.filtered_chroma(r, g, b, 191)
        assert n >= (max(r, g, b) - min(r, g, b)) * d


def test_gray_decision_and_hue():
    """A washed-out skin pixel: gray (chroma 14 < 20) without the filter,
    not gray with lum_hi 191; the hue test does not change."""
    f = np.array([[[252, 244, 238], [255, 255, 255], [100, 60, 40]]], np.uint8)
    bgmin = np.zeros_like(f)
    bgmax = np.zeros_like(f)
    off = oracle.masks(f, bgmin, bgmax, oracle.params())
    on = oracle.masks(f, bgmin, bgmax, oracle.params(lum_hi=191))
    assert off["r2"].tolist() == [[0, 0, 1]]
    assert on["r2"].tolist() == [[1, 0, 1]]
    assert np.array_equal(off["r3"], on["r3"]) and off["r3"][0, 0] == 1
    assert np.array_equal(off["r1"], on["r1"])


def _scene(hand_rgb, H=48, W=64):
    bg = np.zeros((4, H, W, 3), np.uint8)
    bg[...] = (40, 40, 90)
    fr = bg[:1].copy()
    fr[0, 10:30, 20:44] = hand_rgb            # 24 x 20 rectangle
    return bg, fr[0]


def test_over_exposed_hand_end_to_end():
    """Without the filter the white-looking hand is removed as gray and no
    hand is found; with it the rectangle is the hand (closed-form stats)."""
    bg, fr = _scene((252, 244, 238))
    for lum_hi, present in ((0, 0), (191, 1)):
        m = oracle.Model(64, 48, oracle.params(lum_hi=lum_hi, open_iters=0, close_iters=0))
        m.learn(bg)
        p = m.process(fr)["pointer"]
        assert p["present"] == present, lum_hi
        if present:
            assert p["area"] == 480 and (p["x0"], p["y0"], p["x1"], p["y1"]) == (20, 10, 43, 29)
            assert p["sum_x"] == 20 * sum(range(20, 44)) and p["sum_y"] == 24 * sum(range(10, 30))
