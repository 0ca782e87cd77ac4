"""Pins of background learning and of the empty-scene invariants
(Section 2 initialisation, Section 3.1 (i))."""
import numpy as np


def test_identical_frames_give_a_point_box(orc):
    rng = np.random.default_rng(1)
    f = rng.integers(10, 240, size=(24, 64, 3), dtype=np.uint8)
    m = orc.Model(64, 24)
    inv = m.learn(np.stack([f] * 4))
    assert (inv == 65536).all()
    assert (m.bgmin == f).all() and (m.bgmax == f).all()


def test_empty_scene(orc):
    """A noise-free constant background and any later identical frame give an
    empty mask and no pointer."""
    f = np.full((32, 64, 3), (90, 140, 60), np.uint8)
    m = orc.Model(64, 32)
    m.learn(np.stack([f] * 3))
    out = m.process(f, frame_index=7, want_raw=True)
    assert out["raw"].sum() == 0 and out["fizi"].sum() == 0
    assert out["pointer"]["present"] == 0 and out["pointer"]["n_components"] == 0
    assert out["pointer"]["frame_index"] == 7


def test_training_frames_are_background(orc):
    """Every learning frame, processed afterwards, is all background for any
    margin delta >= 0: its corrected value lies inside the learned box."""
    from paper_1907_04393_amd import scene
    sc = scene.Scene(scene.SceneSpec(128, 64, sigma=4.0, n_bg=8, n_hand=4, seed=(1, 2, 3, 4)))
    bg = sc.bg_frames(0, 8).numpy()
    # put skin-hued blobs in the learning frames too: still background
    bg[3, 10:20, 10:30] = (200, 120, 90)
    for delta in (0, 10):
        m = orc.Model(128, 64, orc.params(bg_delta=delta))
        inv = m.learn(bg)
        for k in range(8):
            out = m.process(bg[k], want_raw=True)
            assert out["raw"].sum() == 0, (delta, k)
            assert out["pointer"]["inv_gain_q16"] == inv[k]


def test_learning_continues_without_reset(orc):
    rng = np.random.default_rng(2)
    a = rng.integers(50, 200, size=(3, 16, 64, 3), dtype=np.uint8)
    m1 = orc.Model(64, 16)
    m1.learn(a)
    m2 = orc.Model(64, 16)
    m2.learn(a[:1])
    m2.learn(a[1:], reset=False)
    assert (m1.bgmin == m2.bgmin).all() and (m1.bgmax == m2.bgmax).all()
    assert (m1.yref == m2.yref).all()


def test_box_margin_inclusive(orc):
    """I_R1: values inside [min - delta, max + delta] are background; one
    level outside in one channel is foreground."""
    bgmin = np.array([[[50, 60, 70]]], np.uint8)
    bgmax = np.array([[[80, 90, 100]]], np.uint8)
    for delta in (0, 10):
        p = orc.params(bg_delta=delta)
        inside = [(50 - delta, 60, 70), (80 + delta, 90 + delta, 100 + delta), (65, 75, 85)]
        outside = [(49 - delta, 60, 70), (80, 91 + delta, 100), (65, 75, 101 + delta)]
        for v in inside:
            assert orc.masks(np.array([[v]], np.uint8), bgmin, bgmax, p)["r1"][0, 0] == 0
        for v in outside:
            assert orc.masks(np.array([[v]], np.uint8), bgmin, bgmax, p)["r1"][0, 0] == 1
