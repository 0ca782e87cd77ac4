"""Pins of the oracle's click debouncing (reading R13; Section 2: the Mouse
module tracks the hand and reports its state, click or not; a fill-ratio
click flickers when the hand's outline is noisy): with tracking on and
click_debounce D, a change of the reported click needs D consecutive frames
that show the new state; a frame without a hand reports no click and starts
over. Pinned on hand-worked sequences and on D <= 1 being no filter."""
import numpy as np
import pytest

from oracle import oracle


def run(raw, present, D):
    st = oracle.ClickDebounce(D)
    return [st.step(p, r) for r, p in zip(raw, present)]


def test_no_filter_at_d0_and_d1():
    rng = np.random.default_rng(0)
    raw = rng.integers(0, 2, 50).tolist()
    present = (rng.random(50) < 0.9).astype(int).tolist()
    want = [r if p else 0 for r, p in zip(raw, present)]
    assert run(raw, present, 0) == want
    assert run(raw, present, 1) == want


def test_hand_worked_sequence_d3():
    #          0  1  2  3  4  5  6  7  8  9 10 11 12 13
    raw = [1, 1, 0, 1, 1, 1, 1, 0, 0, 1, 0, 0, 0, 1]
    present = [1] * len(raw)
    # frames 0-1 see a click twice: not yet adopted; frame 2 releases (count
    # restarts); 3, 4, 5 are three clicks in a row: adopted at 5; 7, 8 are two
    # releases, 9 clicks again (count restarts); 10, 11, 12 release: adopted
    # at 12; 13 is a single click
    want = [0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 0, 0]
    assert run(raw, present, 3) == want


def test_absent_hand_reports_no_click_and_starts_over():
    raw = [1, 1, 1, 0, 1, 1, 1]
    present = [1, 1, 1, 0, 1, 1, 1]
    # D = 2: adopted at frame 1; frame 3 has no hand (0, state cleared);
    # frames 4, 5 click again: adopted at 5
    assert run(raw, present, 2) == [0, 1, 1, 0, 0, 1, 1]


def test_isolated_flips_never_pass():
    raw = [0, 1, 0, 1, 0, 1, 0, 0, 1, 0] * 3
    assert run(raw, [1] * len(raw), 2) == [0] * len(raw)
    steady = [1] * 5
    assert run(steady, [1] * 5, 5) == [0, 0, 0, 0, 1]


def _shapes():
    """A filled square (fill 1: click) and a hollow one (fill 0.64: no click)
    at a slowly moving position."""
    W, H = 128, 64
    seq = "FFHFFHHHFHHH"
    masks = []
    for k, s in enumerate(seq):
        m = np.zeros((H, W), np.uint8)
        x0, y0 = 20 + 2 * k, 10
        m[y0:y0 + 30, x0:x0 + 30] = 1
        if s == "H":
            m[y0 + 6:y0 + 24, x0 + 6:x0 + 24] = 0
        masks.append(m)
    return np.stack(masks)


def test_tracker_debounces_the_pointer():
    masks = _shapes()
    H, W = masks.shape[1:]
    bg = np.zeros((2, H, W, 3), np.uint8)
    bg[...] = (40, 40, 90)
    fr = np.repeat(bg[:1], len(masks), axis=0).copy()
    fr[masks.astype(bool)] = (210, 140, 90)
    clicks = {}
    for D in (0, 2, 3):
        m = oracle.Model(W, H, oracle.params(open_iters=0, close_iters=0, click_debounce=D))
        m.learn(bg)
        t = oracle.Tracker(m)
        clicks[D] = [t.process(fr[k], frame_index=k)["pointer"]["click"] for k in range(len(fr))]
    assert clicks[0] == [1 if s == "F" else 0 for s in "FFHFFHHHFHHH"]
    # D = 2: adopted at frame 1; single H at 2 filtered; H H at 5-6: released
    # at 6; F at 8 alone: filtered
    assert clicks[2] == [0, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0]
    # D = 3: F F then H restarts the count; F F at 3-4 then H: never adopted
    assert clicks[3] == [0] * 12
