"""GPU parity of temporal tracking (reading R10) with the oracle's Tracker:
plain contexts (frames of a call tracked in order, in chunks), the batched
form in every launch mode, and the reset on enabling."""
import numpy as np
import pytest
import torch

from helpers import need_gpu

pytestmark = pytest.mark.gpu

W, H = 128, 64
BIG = (10, 10, 49, 39)


def _rect(m, x0, y0, x1, y1):
    m[y0:y1 + 1, x0:x1 + 1] = 1


def _sequence():
    """Frames 0-1: a small square alone; 2-5: a big static rectangle joins
    while the square moves on; 6: the square is gone; 7-8: it is back."""
    masks = []
    for k in range(9):
        m = np.zeros((H, W), np.uint8)
        if k >= 2:
            _rect(m, *BIG)
        if k != 6:
            x0 = 60 + 3 * k
            _rect(m, x0, 20, x0 + 9, 29)
        masks.append(m)
    masks = np.stack(masks)
    bg = np.zeros((2, H, W, 3), np.uint8)
    bg[...] = (40, 40, 90)
    fr = np.repeat(bg[:1], len(masks), axis=0).copy()
    fr[masks.astype(bool)] = (210, 140, 90)
    return torch.from_numpy(bg), torch.from_numpy(fr), masks


PARAMS = dict(open_iters=0, close_iters=0)


def _oracle_track(bg, fr, params, prev=None):
    from oracle import oracle
    m = oracle.Model(bg.shape[2], bg.shape[1], oracle.params(**params))
    m.learn(bg.numpy())
    t = oracle.Tracker(m)
    t.prev = prev
    return [t.process(fr[k].numpy(), frame_index=k, want_hand=True) for k in range(fr.shape[0])]


@pytest.mark.parametrize("chunk", [1, 3, 8])
def test_plain_tracking_matches_oracle(chunk):
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, fr, masks = _sequence()
    ref = _oracle_track(bg, fr, PARAMS)
    # the tracker really departs from the largest component here
    assert ref[3]["pointer"]["area"] == 100 and ref[7]["pointer"]["area"] == 1200
    ctx = fizi.Context(W, H, fizi.default_params(**PARAMS), chunk=chunk, device=dev)
    ctx.learn_background(bg.to(dev))
    ctx.set_tracking(True)
    out = ctx.process_frames(fr.to(dev), want_fizi=True, want_hand=True)
    torch.cuda.synchronize()
    got = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(out["pointers"])]
    hand = fizi.unpack_bits(out["hand"], W)
    for k in range(fr.shape[0]):
        assert got[k] == ref[k]["pointer"], (chunk, k, got[k], ref[k]["pointer"])
        assert np.array_equal(hand[k], ref[k]["hand"]), (chunk, k)


def test_tracking_across_calls_and_reset():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, fr, _ = _sequence()
    ref = _oracle_track(bg, fr, PARAMS)
    ctx = fizi.Context(W, H, fizi.default_params(**PARAMS), chunk=2, device=dev)
    ctx.learn_background(bg.to(dev))
    ctx.set_tracking(True)
    got = []
    for k in range(5):                          # one frame per call
        out = ctx.process_frames(fr[k:k + 1].to(dev))
        torch.cuda.synchronize()
        got.append(fizi.pointer_dict(fizi.pointers_to_numpy(out["pointers"])[0]))
    for k in range(5):
        g = dict(got[k]); g["frame_index"] = k
        assert g == ref[k]["pointer"], k
    # enabling again forgets the previous hand: frame 5 then takes the largest
    ctx.set_tracking(True)
    out = ctx.process_frames(fr[5:6].to(dev))
    torch.cuda.synchronize()
    p = fizi.pointer_dict(fizi.pointers_to_numpy(out["pointers"])[0])
    assert p["area"] == 1200
    ctx.set_tracking(False)


def test_scene_tracking_matches_oracle():
    """A generated scene with two static skin distractors, 40 frames in
    chunks of 16."""
    from paper_1907_04393_amd import fizi, scene
    dev = need_gpu()
    sp = scene.SceneSpec(320, 240, sigma=3, seed=(9, 2, 0, 0), distractors=2)
    sc = scene.Scene(sp)
    bg, hand = sc.bg_frames(0, 20), sc.hand_frames(0, 40)
    ref = _oracle_track(bg, hand, {})
    ctx = fizi.Context(320, 240, chunk=16, device=dev)
    ctx.learn_background(bg.to(dev))
    ctx.set_tracking(True)
    out = ctx.process_frames(hand.to(dev), want_hand=True)
    torch.cuda.synchronize()
    got = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(out["pointers"])]
    hd = fizi.unpack_bits(out["hand"], 320)
    for k in range(40):
        assert got[k] == ref[k]["pointer"], k
        assert np.array_equal(hd[k], ref[k]["hand"]), k


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5])
def test_batch_tracking_matches_oracle(mode):
    from oracle import oracle
    from paper_1907_04393_amd import fizi
    from test_gpu_plain import _blob_scene
    dev = need_gpu()
    bg, fr, _ = _sequence()
    bgb, frb = _blob_scene(192, 70, 4, 9, seed=21)
    b = fizi.Batch([(W, H), (192, 70)], [fizi.default_params(**PARAMS), fizi.default_params()], device=dev)
    b.set_mode(mode)
    b.learn(0, bg.to(dev))
    b.learn(1, bgb.to(dev))
    b.set_tracking(0, True)
    ref_a = _oracle_track(bg, fr, PARAMS)
    mb = oracle.Model(192, 70)
    mb.learn(bgb.numpy())
    fa, fb = fr.to(dev), frb.to(dev)
    bufs = []
    for k in range(fr.shape[0]):
        bufs.append(torch.empty((2, 56), dtype=torch.uint8, device=dev))
        b.step([fa[k], fb[k]], bufs[-1])
    b.flush()
    torch.cuda.synchronize()
    for k, ptrs in enumerate(bufs):
        got = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(ptrs)]
        assert got[0] == ref_a[k]["pointer"], (mode, k)
        assert got[1] == mb.process(frb[k].numpy(), frame_index=k)["pointer"], (mode, k)
    assert b.status() == 0
    b.close()


def _jump_sequence():
    """A 10x10 square alone, then jumping 20 px right (its old centroid pixel
    misses it) while a larger rectangle appears farther away, then growing
    into a ring whose centroid is its hole, then gone, then back far away.
    The oracle's picks are worked out in the tests below."""
    masks = []
    for k in range(7):
        m = np.zeros((H, W), np.uint8)
        if k >= 1:
            _rect(m, 0, 40, 29, 59)                   # 30 x 20 = 600 px
        if k == 0:
            _rect(m, 40, 10, 49, 19)
        elif k == 1:
            _rect(m, 60, 10, 69, 19)
        elif k in (2, 3):
            _rect(m, 60, 10, 79, 29)
            m[15:25, 65:75] = 0                       # ring, centroid (69, 19) in the hole
        elif k == 5:
            _rect(m, 100, 10, 109, 19)
        masks.append(m)
    masks = np.stack(masks)
    bg = np.zeros((2, H, W, 3), np.uint8)
    bg[...] = (40, 40, 90)
    fr = np.repeat(bg[:1], len(masks), axis=0).copy()
    fr[masks.astype(bool)] = (210, 140, 90)
    return torch.from_numpy(bg), torch.from_numpy(fr)


@pytest.mark.parametrize("radius", [64, 0])
@pytest.mark.parametrize("chunk", [1, 3, 7])
def test_plain_nearest_component_tracking(chunk, radius):
    """Tracking with the nearest-component pick (default radius) and with
    containment only (radius 0), in chunks of frames, against the oracle."""
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    params = dict(PARAMS, track_radius=radius)
    bg, fr = _jump_sequence()
    ref = _oracle_track(bg, fr, params)
    areas = [r["pointer"]["area"] for r in ref]
    # radius 64: the jumped square (100 px) and the ring (300 px) keep the
    # hand over the larger rectangle; radius 0: the rectangle takes it
    assert areas == ([100, 100, 300, 300, 600, 600, 600] if radius else [100, 600, 600, 600, 600, 600, 600])
    ctx = fizi.Context(W, H, fizi.default_params(**params), chunk=chunk, device=dev)
    ctx.learn_background(bg.to(dev))
    ctx.set_tracking(True)
    out = ctx.process_frames(fr.to(dev), want_fizi=True, want_hand=True)
    torch.cuda.synchronize()
    got = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(out["pointers"])]
    hand = fizi.unpack_bits(out["hand"], W)
    for k in range(fr.shape[0]):
        assert got[k] == ref[k]["pointer"], (chunk, radius, k, got[k], ref[k]["pointer"])
        assert np.array_equal(hand[k], ref[k]["hand"]), (chunk, radius, k)


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5])
def test_batch_nearest_component_tracking(mode):
    """The same sequence as one tracked stream of a batch (one frame per
    step: the pick is made inside the component stage) beside an untracked
    stream, in every launch mode."""
    from oracle import oracle
    from paper_1907_04393_amd import fizi
    from test_gpu_plain import _blob_scene
    dev = need_gpu()
    bg, fr = _jump_sequence()
    bgb, frb = _blob_scene(192, 70, 4, fr.shape[0], seed=29)
    b = fizi.Batch([(W, H), (192, 70)], [fizi.default_params(**PARAMS), fizi.default_params()], device=dev)
    b.set_mode(mode)
    b.learn(0, bg.to(dev))
    b.learn(1, bgb.to(dev))
    b.set_tracking(0, True)
    ref_a = _oracle_track(bg, fr, PARAMS)
    mb = oracle.Model(192, 70)
    mb.learn(bgb.numpy())
    fa, fb = fr.to(dev), frb.to(dev)
    bufs = []
    for k in range(fr.shape[0]):
        bufs.append(torch.empty((2, 56), dtype=torch.uint8, device=dev))
        b.step([fa[k], fb[k]], bufs[-1])
    b.flush()
    torch.cuda.synchronize()
    for k, ptrs in enumerate(bufs):
        got = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(ptrs)]
        assert got[0] == ref_a[k]["pointer"], (mode, k, got[0], ref_a[k]["pointer"])
        assert got[1] == mb.process(frb[k].numpy(), frame_index=k)["pointer"], (mode, k)
    assert b.status() == 0
    b.close()


SHAPES = "FFHFFHHHFHHH"   # filled square (clicks) / hollow square (does not)


def _shape_frames():
    masks = []
    for k, s in enumerate(SHAPES):
        m = np.zeros((H, W), np.uint8)
        x0 = 20 + 2 * k
        m[10:40, x0:x0 + 30] = 1
        if s == "H":
            m[16:34, x0 + 6:x0 + 24] = 0
        masks.append(m)
    bg = np.zeros((2, H, W, 3), np.uint8)
    bg[...] = (40, 40, 90)
    fr = np.repeat(bg[:1], len(masks), axis=0).copy()
    fr[np.stack(masks).astype(bool)] = (210, 140, 90)
    return torch.from_numpy(bg), torch.from_numpy(fr)


@pytest.mark.parametrize("D,chunk", [(2, 1), (2, 5), (3, 12), (0, 4)])
def test_plain_click_debounce_matches_oracle(D, chunk):
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    params = dict(PARAMS, click_debounce=D)
    bg, fr = _shape_frames()
    ref = _oracle_track(bg, fr, params)
    assert [r["pointer"]["click"] for r in ref] != [int(s == "F") for s in SHAPES] or D == 0
    ctx = fizi.Context(W, H, fizi.default_params(**params), chunk=chunk, device=dev)
    ctx.learn_background(bg.to(dev))
    ctx.set_tracking(True)
    out = ctx.process_frames(fr.to(dev))
    torch.cuda.synchronize()
    got = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(out["pointers"])]
    for k in range(len(SHAPES)):
        assert got[k] == ref[k]["pointer"], (D, chunk, k)
    # re-enabling clears the debouncer: two filled frames are needed again
    ctx.set_tracking(True)
    out = ctx.process_frames(fr[:2].to(dev))
    torch.cuda.synchronize()
    clicks = [int(r["click"]) for r in fizi.pointers_to_numpy(out["pointers"])]
    assert clicks == ([1, 1] if D <= 1 else [0, 1] if D == 2 else [0, 0])
    # without tracking the setting has no effect
    ctx.set_tracking(False)
    out = ctx.process_frames(fr.to(dev))
    torch.cuda.synchronize()
    assert [int(r["click"]) for r in fizi.pointers_to_numpy(out["pointers"])] == [int(s == "F") for s in SHAPES]


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5])
def test_batch_click_debounce_matches_oracle(mode):
    from oracle import oracle
    from paper_1907_04393_amd import fizi
    from test_gpu_plain import _blob_scene
    dev = need_gpu()
    params = dict(PARAMS, click_debounce=2)
    bg, fr = _shape_frames()
    bgb, frb = _blob_scene(192, 70, 4, len(SHAPES), seed=23)
    b = fizi.Batch([(W, H), (192, 70)], [fizi.default_params(**params), fizi.default_params(click_debounce=3)],
                   device=dev)
    b.set_mode(mode)
    b.learn(0, bg.to(dev))
    b.learn(1, bgb.to(dev))
    b.set_tracking(0, True)
    ref_a = _oracle_track(bg, fr, params)
    mb = oracle.Model(192, 70, oracle.params(click_debounce=3))
    mb.learn(bgb.numpy())
    fa, fb = fr.to(dev), frb.to(dev)
    bufs = []
    for k in range(len(SHAPES)):
        bufs.append(torch.empty((2, 56), dtype=torch.uint8, device=dev))
        b.step([fa[k], fb[k]], bufs[-1])
    b.flush()
    torch.cuda.synchronize()
    for k, ptrs in enumerate(bufs):
        got = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(ptrs)]
        assert got[0] == ref_a[k]["pointer"], (mode, k)
        # stream 1 is not tracked: its clicks are the frame's own
        assert got[1] == mb.process(frb[k].numpy(), frame_index=k)["pointer"], (mode, k)
    assert b.status() == 0
    b.close()
