"""Pins of the oracle's temporal tracking (reading R10): among components of
area >= min_area, the one nearest to the previous frame's centroid pixel
(squared distance to its nearest pixel; 0 when it covers the point) keeps
the hand when that distance is at most track_radius, ties to the larger
area, then the smaller first index; otherwise the largest component (R7).
Checked on rectangles whose area, coordinate sums and boxes have closed
forms, with distances worked by hand."""
import numpy as np
import pytest

from oracle import oracle


def rect(m, x0, y0, x1, y1):
    m[y0:y1 + 1, x0:x1 + 1] = 1


def rect_stats(x0, y0, x1, y1):
    w, h = x1 - x0 + 1, y1 - y0 + 1
    return dict(area=w * h, sum_x=h * (x0 + x1) * w // 2, sum_y=w * (y0 + y1) * h // 2,
                x0=x0, y0=y0, x1=x1, y1=y1)


def check(ptr, st):
    for k, v in st.items():
        assert ptr[k] == v, (k, ptr[k], v)


BIG = (10, 10, 49, 39)      # 40 x 30 = 1200 px
SMALL = (70, 20, 79, 29)    # 10 x 10 = 100 px


def scene():
    m = np.zeros((64, 128), np.uint8)
    rect(m, *BIG)
    rect(m, *SMALL)
    return m


def test_no_track_is_the_largest():
    m = scene()
    assert oracle.pointer_of(m, track=None) == oracle.pointer_of(m)
    check(oracle.pointer_of(m), rect_stats(*BIG))


@pytest.mark.parametrize("track,expect", [((75, 25), SMALL), ((70, 20), SMALL), ((79, 29), SMALL),
                                          ((30, 25), BIG), ((60, 25), BIG), ((69, 25), BIG),
                                          ((-1, 5), BIG), ((500, 5), BIG)])
def test_containment_only_with_radius_0(track, expect):
    """track_radius 0: only the component covering the point keeps the hand."""
    p = oracle.pointer_of(scene(), oracle.params(track_radius=0), track=track)
    assert p["present"] == 1 and p["n_components"] == 2
    check(p, rect_stats(*expect))


@pytest.mark.parametrize("track,expect", [((75, 25), SMALL), ((30, 25), BIG),
                                          ((60, 25), SMALL),    # SMALL at d^2 100, BIG at 121
                                          ((59, 25), BIG),      # BIG at d^2 100, SMALL at 121
                                          ((69, 25), SMALL), ((50, 40), BIG),
                                          ((-1, 5), BIG)])
def test_nearest_component_with_the_default_radius(track, expect):
    """Default radius 64: the nearest component to the point, by the squared
    distance to its nearest pixel (BIG spans columns 10..49, SMALL 70..79)."""
    p = oracle.pointer_of(scene(), track=track)
    assert p["present"] == 1 and p["n_components"] == 2
    check(p, rect_stats(*expect))


def test_small_tracked_component_below_min_area_falls_back():
    p = oracle.pointer_of(scene(), oracle.params(min_area=101), track=(75, 25))
    check(p, rect_stats(*BIG))
    p = oracle.pointer_of(scene(), oracle.params(min_area=100), track=(75, 25))
    check(p, rect_stats(*SMALL))


def test_ring_whose_centroid_is_its_hole():
    """A ring's centroid is its hole. Its nearest pixels, (74, 29) and
    (79, 24), are 5 px away (d^2 = 25); BIG's nearest, (49, 29), is 30 px
    away. Within the default radius the ring keeps the hand; with radius 4
    (16 < 25) or 0 (containment only) the largest takes it."""
    m = np.zeros((64, 128), np.uint8)
    rect(m, *BIG)
    rect(m, 70, 20, 89, 39)
    m[25:35, 75:85] = 0                       # 20x20 ring, centroid (79, 29) is in the hole
    ring = oracle.pointer_of(m, track=(71, 21))
    assert ring["area"] == 400 - 100
    c = oracle.centroid_pixel(ring)
    assert c == (79, 29) and m[c[1], c[0]] == 0
    kept = oracle.pointer_of(m, track=c)
    assert kept["area"] == 300 and (kept["x0"], kept["y0"], kept["x1"], kept["y1"]) == (70, 20, 89, 39)
    assert oracle.pointer_of(m, oracle.params(track_radius=5), track=c)["area"] == 300
    check(oracle.pointer_of(m, oracle.params(track_radius=4), track=c), rect_stats(*BIG))
    check(oracle.pointer_of(m, oracle.params(track_radius=0), track=c), rect_stats(*BIG))


@pytest.mark.parametrize("radius,expect", [(64, SMALL), (11, SMALL), (10, BIG), (0, BIG)])
def test_jump_keeps_the_nearest_within_the_radius(radius, expect):
    """The hand jumped: the previous centroid (90, 25) is 11 px right of
    SMALL's column 79 (d^2 = 121) and 41 px from BIG's column 49
    (d^2 = 1681): SMALL within a radius of 11 (inclusive), BIG beyond."""
    p = oracle.pointer_of(scene(), oracle.params(track_radius=radius), track=(90, 25))
    check(p, rect_stats(*expect))


def test_point_outside_the_image():
    """(130, 25) is beyond the right edge (W = 128): SMALL's nearest pixel is
    51 px away (2601 <= 64^2); (500, 5) is 421 px away: the largest."""
    check(oracle.pointer_of(scene(), track=(130, 25)), rect_stats(*SMALL))
    check(oracle.pointer_of(scene(), track=(500, 5)), rect_stats(*BIG))


def test_distance_ties():
    """Two squares at the same distance from (50, 30): the larger wins; two
    equal squares at the same distance: the one first in raster order."""
    m = np.zeros((64, 128), np.uint8)
    rect(m, 30, 20, 39, 29)          # 10 x 10, nearest pixel (39, 29): dx 11, dy 1 -> 122
    rect(m, 61, 31, 72, 42)          # 12 x 12, nearest pixel (61, 31): dx 11, dy 1 -> 122
    rect(m, 100, 50, 127, 63)        # 28 x 14 = 392, the largest, far away
    check(oracle.pointer_of(m, track=(50, 30)), rect_stats(61, 31, 72, 42))
    m = np.zeros((64, 128), np.uint8)
    rect(m, 30, 20, 39, 29)          # equal squares, both at d^2 = 122
    rect(m, 61, 31, 70, 40)
    rect(m, 100, 50, 127, 63)
    check(oracle.pointer_of(m, track=(50, 30)), rect_stats(30, 20, 39, 29))


def test_nearest_skips_components_below_min_area():
    """From (90, 25) SMALL (100 px) is nearest, but with min_area 101 only
    BIG qualifies, 41 px away, within a radius of 64."""
    p = oracle.pointer_of(scene(), oracle.params(min_area=101), track=(90, 25))
    check(p, rect_stats(*BIG))


def _frames(masks):
    """Frames whose I_FIZI is exactly `masks`: skin where set on a bluish
    background learned beforehand, no morphology."""
    bg = np.zeros((2,) + masks.shape[1:] + (3,), np.uint8)
    bg[...] = (40, 40, 90)
    fr = np.repeat(bg[:1], len(masks), axis=0).copy()
    fr[masks.astype(bool)] = (210, 140, 90)
    return bg, fr


def test_tracker_follows_the_moving_component():
    """A small square moving right 3 px per frame beside a large static one,
    gone in frame 4, through the whole oracle path (frames built so that
    I_FIZI equals the drawn masks)."""
    H, W = 64, 128
    masks = []
    for k in range(6):
        m = np.zeros((H, W), np.uint8)
        rect(m, *BIG)
        if k != 4:
            x0 = 60 + 3 * k
            rect(m, x0, 20, x0 + 9, 29)
        masks.append(m)
    masks = np.stack(masks)
    bg, fr = _frames(masks)
    p = oracle.params(open_iters=0, close_iters=0)
    model = oracle.Model(W, H, p)
    model.learn(bg)
    t = oracle.Tracker(model)
    # frame 0: no previous hand -> the largest; then the tracker stays on it
    outs = [t.process(fr[k], frame_index=k) for k in range(6)]
    for k, o in enumerate(outs):
        assert np.array_equal(o["fizi"], masks[k]), k
        check(o["pointer"], rect_stats(*BIG))
    # started on the small square, it follows it until it vanishes
    t2 = oracle.Tracker(model)
    t2.prev = (62, 22)
    for k in range(6):
        o = t2.process(fr[k], frame_index=k)
        if k < 4:
            x0 = 60 + 3 * k
            check(o["pointer"], rect_stats(x0, 20, x0 + 9, 29))
        else:
            check(o["pointer"], rect_stats(*BIG))   # gone, then the big one keeps the hand
