"""Pins of the oracle's brightness correction (Section 2, Section 3.2)."""
from fractions import Fraction

import numpy as np


def _exact_correct(v, inv):
    """Round-half-up of v * inv / 65536, saturated at 255, in exact rationals."""
    q = Fraction(v * inv, 65536)
    r = int(q + Fraction(1, 2)) if q >= 0 else None  # floor(q + 1/2) for q >= 0
    return min(255, r)


def test_correct_value_exhaustive(orc):
    rng = np.random.default_rng(3)
    invs = [32768, 32769, 65535, 65536, 65537, 98304, 131071, 131072] + \
        [int(x) for x in rng.integers(32768, 131073, size=60)]
    for inv in invs:
        for v in range(256):
            assert orc.correct_value(v, inv) == _exact_correct(v, inv), (v, inv)


def _scene(H=48, W=64, seed=0):
    rng = np.random.default_rng(seed)
    return rng.integers(20, 230, size=(H, W, 3), dtype=np.uint8)


def test_first_frame_gain_is_identity(orc):
    for seed in range(5):
        f0 = _scene(seed=seed)
        f0[0, :5] = 255      # clipped pixels get the sentinel
        yref = orc.make_yref(f0)
        assert orc.gain(f0, yref) == 65536
        assert (orc.correct(f0, 65536) == f0).all()


def test_gray_frame_closed_form(orc):
    """A gray frame scaled by g (no clipping): every sampled pixel is usable,
    so inv = round_half_up(65536 * sum(Y0) / sum(Y_g)) with Y = 4v."""
    rng = np.random.default_rng(5)
    H, W = 40, 64
    v0 = rng.integers(30, 200, size=(H, W)).astype(np.int64)
    f0 = np.repeat(v0[:, :, None], 3, axis=2).astype(np.uint8)
    yref = orc.make_yref(f0)
    for g in (0.8, 0.93, 1.0, 1.07, 1.2):
        vg = np.rint(v0 * g).astype(np.int64)
        fg = np.repeat(vg[:, :, None], 3, axis=2).astype(np.uint8)
        num = int((4 * v0[::8]).sum())
        den = int((4 * vg[::8]).sum())
        expect = (num * 65536 + den // 2) // den
        got = orc.gain(fg, yref)
        assert got == expect
        # and close to 1/g: rounding moves each Y by at most 2 of ~4*v*g
        n = v0[::8].size
        bound = 65536 * 2 * n / (g * den) * 4 + 1
        assert abs(got - 65536 / g) <= bound


def test_gain_ignores_skin_and_clipped(orc):
    f0 = _scene(seed=9)
    # make the sampled row pixels non-skin so the usable set is known
    yref = orc.make_yref(f0)
    f1 = f0.copy()
    base = orc.gain(f1, yref)
    # paint skin-hued pixels (hue 15 deg) and clipped pixels on sampled rows
    f1[0, 10:30] = (200, 50, 0)
    f1[8, 0:20] = (255, 100, 100)
    g_skin = orc.gain(f1, yref)
    f2 = f0.copy()
    f2[0, 10:30] = (220, 80, 25)   # another skin hue: same exclusion
    f2[8, 0:20] = (255, 3, 7)
    assert orc.gain(f2, yref) == g_skin
    # replacing usable pixels changes the gain in general
    assert isinstance(base, int)


def test_gain_degenerate_and_clamp(orc):
    H, W = 16, 64
    f = np.full((H, W, 3), 255, np.uint8)
    yref = orc.make_yref(f)                # all sentinel
    assert orc.gain(f, yref) == 65536
    f0 = np.full((H, W, 3), 100, np.uint8)
    yref = orc.make_yref(f0)
    dark = np.full((H, W, 3), 20, np.uint8)   # 5x darker: clamp at 2.0
    assert orc.gain(dark, yref) == 131072
    bright = np.full((H, W, 3), 254, np.uint8)  # 2.54x brighter: clamp at 0.5
    assert orc.gain(bright, yref) == 32768
    p = orc.params(gain_lo_q16=60000, gain_hi_q16=70000)
    assert orc.gain(dark, yref, p) == 70000
