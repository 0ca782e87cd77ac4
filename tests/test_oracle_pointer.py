"""Pins of the oracle's hand-zone selection and pointer (Section 2, Mouse and
Interface modules): closed-form ellipses, ties, click and absence."""
import numpy as np


def _ellipse(H, W, cx, cy, a, b):
    ys, xs = np.mgrid[0:H, 0:W]
    dx, dy = xs - cx, ys - cy
    return ((dx * dx * b * b + dy * dy * a * a) <= a * a * b * b).astype(np.uint8)


def test_ellipse_area_and_centroid_closed_form(orc):
    """An ellipse centred on a pixel is point-symmetric, so the centroid sums
    are exactly cx*A and cy*A; the area is the lattice count of
    dx^2 b^2 + dy^2 a^2 <= a^2 b^2 and approaches pi a b."""
    for (cx, cy, a, b) in [(60, 50, 25, 30), (100, 60, 7, 11), (64, 64, 40, 20)]:
        H, W = 128, 192
        m = _ellipse(H, W, cx, cy, a, b)
        lattice = sum(1 for dx in range(-a, a + 1) for dy in range(-b, b + 1)
                      if dx * dx * b * b + dy * dy * a * a <= a * a * b * b)
        p = orc.pointer_of(m)
        assert p["present"] == 1 and p["n_components"] == 1
        assert p["area"] == lattice
        assert abs(lattice - np.pi * a * b) < 2 * (a + b) + 4
        assert p["sum_x"] == cx * p["area"] and p["sum_y"] == cy * p["area"]
        assert (p["x0"], p["x1"], p["y0"], p["y1"]) == (cx - a, cx + a, cy - b, cy + b)
        # morphology keeps the point symmetry
        fz = orc.morph(m, 1, 1)
        q = orc.pointer_of(fz)
        assert q["sum_x"] == cx * q["area"] and q["sum_y"] == cy * q["area"]


def test_rotated_ellipse_symmetry(orc):
    H, W = 96, 128
    cx, cy = 60, 50
    ys, xs = np.mgrid[0:H, 0:W]
    dx, dy = (xs - cx).astype(float), (ys - cy).astype(float)
    th = 0.4
    u = dx * np.cos(th) + dy * np.sin(th)
    v = -dx * np.sin(th) + dy * np.cos(th)
    m = ((u / 30.0) ** 2 + (v / 14.0) ** 2 <= 1.0).astype(np.uint8)
    fz = orc.morph(m, 1, 1)
    p = orc.pointer_of(fz)
    assert p["sum_x"] == cx * p["area"] and p["sum_y"] == cy * p["area"]


def test_largest_wins_and_ties_go_to_first(orc):
    m = np.zeros((40, 64), np.uint8)
    m[2:7, 40:45] = 1     # 25 px, first in raster order
    m[20:25, 5:10] = 1    # 25 px, later
    p = orc.pointer_of(m)
    assert p["n_components"] == 2 and p["area"] == 25
    assert (p["x0"], p["y0"]) == (40, 2)
    m[30:36, 50:56] = 1   # 36 px, last but largest
    p = orc.pointer_of(m)
    assert p["area"] == 36 and (p["x0"], p["y0"]) == (50, 30)


def test_diagonal_touch_is_connected(orc):
    m = np.zeros((8, 64), np.uint8)
    m[2, 3] = m[3, 4] = m[4, 3] = 1
    assert orc.pointer_of(m)["n_components"] == 1


def test_click_fill_rule(orc):
    """A filled palm clicks; the same palm with long thin fingers does not."""
    H, W = 160, 192
    palm = _ellipse(H, W, 96, 100, 25, 30)
    p = orc.pointer_of(palm)
    assert p["click"] == 1                  # fill about pi/4 > 0.7
    hand = palm.copy()
    for k in range(4):
        x = 86 + 6 * k
        hand[15:80, x:x + 3] = 1
    q = orc.pointer_of(hand)
    assert q["n_components"] == 1 and q["click"] == 0


def test_absent_and_min_area(orc):
    m = np.zeros((16, 64), np.uint8)
    p = orc.pointer_of(m, inv=70000, frame_index=3)
    assert p == dict(present=0, click=0, area=0, n_components=0, inv_gain_q16=70000,
                     x0=0, y0=0, x1=0, y1=0, sum_x=0, sum_y=0, frame_index=3)
    m[4:8, 4:8] = 1
    p = orc.pointer_of(m, orc.params(min_area=17))
    assert p["present"] == 0 and p["n_components"] == 1 and p["area"] == 0
    p = orc.pointer_of(m, orc.params(min_area=16))
    assert p["present"] == 1 and p["area"] == 16


def test_hand_mask_is_selected_component(orc):
    m = np.zeros((30, 64), np.uint8)
    m[2:5, 2:5] = 1
    m[10:20, 20:40] = 1
    p, hand = orc.pointer_of(m, want_hand=True)
    assert hand.sum() == p["area"] == 200 and hand[2:5, 2:5].sum() == 0
