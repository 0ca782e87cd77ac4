"""Pins of the oracle's temporal tracking (reading R10): the component that
covers the previous frame's centroid pixel keeps the hand when its area
reaches min_area; otherwise the largest component (R7). Checked on
rectangles whose area, coordinate sums and boxes have closed forms."""
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
def test_tracked_pixel_selects_its_component(track, expect):
    p = oracle.pointer_of(scene(), track=track)
    assert p["present"] == 1 and p["n_components"] == 2
    check(p, rect_stats(*expect))


def test_small_tracked_component_below_min_area_falls_back():
    p = oracle.pointer_of(scene(), oracle.params(min_area=101), track=(75, 25))
    check(p, rect_stats(*BIG))
    p = oracle.pointer_of(scene(), oracle.params(min_area=100), track=(75, 25))
    check(p, rect_stats(*SMALL))


def test_centroid_pixel_outside_its_component_is_lost():
    """A ring's centroid is its hole: tracking from it falls back to the largest."""
    m = np.zeros((64, 128), np.uint8)
    rect(m, *BIG)
    rect(m, 70, 20, 89, 39)
    m[25:35, 75:85] = 0                       # 20x20 ring, centroid (79, 29) is in the hole
    ring = oracle.pointer_of(m, track=(71, 21))
    assert ring["area"] == 400 - 100
    c = oracle.centroid_pixel(ring)
    assert c == (79, 29) and m[c[1], c[0]] == 0
    check(oracle.pointer_of(m, track=c), rect_stats(*BIG))


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
