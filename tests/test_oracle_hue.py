"""Pins of the oracle's skin-hue and gray tests (Section 3.1 (ii), (iii))."""
import colorsys
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hue_boundaries.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("case", _golden())
def test_hue_golden(orc, case):
    r, g, b, a1, a2, expected = case
    assert orc.hue_in(r, g, b, a1, a2) == bool(expected)


def _colorsys_in(r, g, b, a1, a2):
    h, s, v = colorsys.rgb_to_hsv(r / 255.0, g / 255.0, b / 255.0)
    deg = h * 360.0
    return deg, s > 0


def test_hue_against_colorsys_sample(orc):
    """Library hue (Python's colorsys) on 200k random colours, several
    intervals, away from the interval ends by more than 1e-7 degrees."""
    rng = np.random.default_rng(7)
    cols = rng.integers(0, 256, size=(200_000, 3))
    intervals = [(33000, 7500), (0, 6000), (12000, 24000), (35000, 500), (9000, 27000)]
    for a1, a2 in intervals:
        lo, hi = a1 / 100.0, a2 / 100.0
        checked = 0
        for r, g, b in cols[:40_000]:
            deg, chroma = _colorsys_in(r, g, b, a1, a2)
            if not chroma:
                assert not orc.hue_in(r, g, b, a1, a2)
                continue
            if min(abs(deg - lo), abs(deg - hi), abs(deg - lo - 360), abs(deg - hi + 360),
                   abs(deg - 360 - hi), abs(deg + 360 - lo)) < 1e-7:
                continue
            inside = (lo <= deg <= hi) if a1 <= a2 else (deg >= lo or deg <= hi)
            assert orc.hue_in(r, g, b, a1, a2) == inside, (r, g, b, a1, a2, deg)
            checked += 1
        assert checked > 30_000


def test_hue_fraction_matches_colorsys(orc):
    rng = np.random.default_rng(11)
    for r, g, b in rng.integers(0, 256, size=(5000, 3)):
        fr = orc.hue_fraction(r, g, b)
        h, s, v = colorsys.rgb_to_hsv(r / 255.0, g / 255.0, b / 255.0)
        if s == 0:
            assert fr is None
        else:
            hn, hd = fr
            assert 0 <= hn < 360 * hd
            assert abs(hn / hd - h * 360.0) < 1e-9


def test_gray_never_skin(orc):
    for v in range(256):
        assert not orc.hue_in(v, v, v, 0, 35999)
        assert not orc.hue_in(v, v, v, 33000, 7500)


def test_gray_test_threshold(orc):
    """I_R2 keeps a pixel iff max - min >= S (Section 3.1 (ii))."""
    p = orc.params(gray_S=20, bg_delta=0)
    fc = np.array([[[100, 119, 110], [100, 120, 110], [0, 0, 0], [255, 235, 240]]], np.uint8)
    bg = np.zeros_like(fc)
    out = orc.masks(fc, bg, bg, p)
    assert out["r2"].tolist() == [[0, 1, 0, 1]]
