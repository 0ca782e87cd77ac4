"""GPU parity of the over-exposure filter (lum_hi, reading R14: the HSL
lightness of over-exposed corrected pixels is brought down to lum_hi before
the gray test) with the CPU oracle: over-exposed pixels crowded around the
filtered gray threshold, an over-exposed hand found only with the filter,
generated scenes, and streams with and without the filter mixed in one
batch in every launch mode."""
import numpy as np
import pytest
import torch

from helpers import compare, gpu_run, need_gpu, oracle_run

pytestmark = pytest.mark.gpu


def _washed_scene(W, H, seed):
    """A dark bluish background; running frames whose middle half of columns
    is bright and washed out (max + min between 380 and 510, chroma 0..40,
    red largest and green above blue: skin hues, so the gain comes from the
    background alone and stays near 1), so the gray test decides most of
    them and many sit at its filtered threshold."""
    rng = np.random.default_rng(seed)
    bg = np.zeros((4, H, W, 3), np.int64)
    bg[...] = (40, 40, 90)
    bg = np.clip(bg + rng.integers(-2, 3, bg.shape), 0, 255)
    hand = np.repeat(bg[:1], 3, axis=0).copy()
    top = rng.integers(190, 256, (3, H, W // 2, 1))
    db = rng.integers(0, 41, (3, H, W // 2))
    dg = (rng.random((3, H, W // 2)) * (db + 1)).astype(np.int64)   # dg <= db
    washed = np.repeat(top, 3, axis=-1)
    washed[..., 1] -= dg
    washed[..., 2] -= db
    hand[:, :, W // 4:W // 4 + W // 2] = np.clip(washed, 0, 255)
    return torch.from_numpy(bg.astype(np.uint8)), torch.from_numpy(hand.astype(np.uint8))


@pytest.mark.parametrize("lum_hi", [128, 191, 230])
@pytest.mark.parametrize("S", [20, 0])
def test_washed_pixels_at_the_filtered_threshold(lum_hi, S):
    bg, hand = _washed_scene(320, 64, seed=lum_hi + S)
    prm = dict(lum_hi=lum_hi, gray_S=S, open_iters=0, close_iters=0)
    print("washed pixels, lum_hi", lum_hi, "S", S, flush=True)
    g = gpu_run(bg, hand, prm, chunk=2)
    m, outs = oracle_run(bg, hand, prm)
    compare(g, m, outs, f"lum_hi {lum_hi} S {S}")
    # the filter really changes the decision here
    if S:
        _, off = oracle_run(bg, hand, dict(prm, lum_hi=0), want_hand=False)
        assert any(not np.array_equal(outs[k]["fizi"], off[k]["fizi"]) for k in outs)


def test_over_exposed_hand_only_with_the_filter():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    H, W = 96, 128
    bg = np.zeros((4, H, W, 3), np.uint8)
    bg[...] = (40, 40, 90)
    fr = np.repeat(bg[:1], 3, axis=0).copy()
    fr[:, 20:60, 30:70] = (252, 244, 238)
    bg, fr = torch.from_numpy(bg), torch.from_numpy(fr)
    for lum_hi, present in ((0, 0), (191, 1)):
        g = gpu_run(bg, fr, dict(lum_hi=lum_hi))
        m, outs = oracle_run(bg, fr, dict(lum_hi=lum_hi))
        compare(g, m, outs, f"hand lum_hi {lum_hi}")
        assert all(p["present"] == present for p in g["pointers"]), lum_hi


def test_generated_scene_with_the_filter():
    from paper_1907_04393_amd import scene
    sc = scene.Scene(scene.small_plain(seed_stream=5))
    bg, hand = sc.bg_frames(0, 30), sc.hand_frames(0, 24)
    g = gpu_run(bg, hand, dict(lum_hi=160), chunk=8)
    m, outs = oracle_run(bg, hand, dict(lum_hi=160))
    compare(g, m, outs, "scene lum_hi 160")


@pytest.mark.parametrize("mode", (0, 1, 2, 3, 4, 5))
def test_batch_mixes_filtered_and_plain_streams(mode):
    from oracle import oracle
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    shapes = [(320, 64), (192, 48), (640, 40)]
    params = [dict(lum_hi=191), dict(), dict(lum_hi=140, gray_S=25)]
    b = fizi.Batch(shapes, [fizi.default_params(**p) for p in params], device=dev)
    b.set_mode(mode)
    data, orc = [], []
    for i, ((W, H), pr) in enumerate(zip(shapes, params)):
        bg, hand = _washed_scene(W, H, seed=40 + i)
        b.learn(i, bg.to(dev))
        m = oracle.Model(W, H, oracle.params(**pr))
        m.learn(bg.numpy())
        data.append(hand.to(dev))
        orc.append((m, hand))
    bufs = []
    for k in range(3):
        ptrs = torch.empty((len(shapes), 56), dtype=torch.uint8, device=dev)
        fz = [torch.empty((H, W // 64), dtype=torch.int64, device=dev) for W, H in shapes]
        b.step([h[k] for h in data], ptrs, fizi=fz)
        bufs.append((ptrs, fz))
    b.flush()
    torch.cuda.synchronize()
    for k, (ptrs, fz) in enumerate(bufs):
        got = fizi.pointers_to_numpy(ptrs)
        for i, (W, H) in enumerate(shapes):
            m, hand = orc[i]
            ref = m.process(hand[k].numpy(), frame_index=k)
            assert fizi.pointer_dict(got[i]) == ref["pointer"], (mode, k, i)
            assert np.array_equal(fizi.unpack_bits(fz[i], W), ref["fizi"]), (mode, k, i)
    assert b.status() == 0
    b.close()


def test_bad_filter_settings_are_rejected():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    for bad in (dict(lum_hi=100), dict(lum_hi=255), dict(lum_hi=191, brightness_mode=1)):
        with pytest.raises(fizi.FiziError):
            fizi.Context(64, 8, fizi.default_params(**bad), device=dev)
