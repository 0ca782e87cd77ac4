"""One-frame calls of a context. When a table slot on the device already
holds a call's table apart from job 0's per-call fields (frame, outputs,
frame index), the call uploads nothing: the gain launch carries those fields
and the component stage zeroes the gain sums for the next such call. Long
runs of one-frame calls (more than the 8 slots, so every slot is reused)
with every kind of change between them are checked against the oracle,
pointer, I_FIZI and hand bits: outputs allocated by the binding or one
pointer buffer reused and read back by get_pointer, a call of several
frames, partial re-learning, learning again, tracking switched on, and the
short morphology bands switched off."""
import numpy as np
import pytest
import torch

from helpers import need_gpu

pytestmark = pytest.mark.gpu

W, H = 320, 240


def _scene():
    from paper_1907_04393_amd import scene
    sp = scene.SceneSpec(W, H, sigma=3, seed=(11, 3, 0, 0), distractors=2)
    sc = scene.Scene(sp)
    return sc.bg_frames(0, 20), sc.bg_frames(20, 30), sc.hand_frames(0, 64)


def test_one_frame_calls_match_oracle():
    from oracle import oracle
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, bg2, hand = _scene()
    hd = hand.to(dev)
    ctx = fizi.Context(W, H, chunk=4, device=dev)
    ctx.learn_background(bg.to(dev))
    m = oracle.Model(W, H)
    m.learn(bg.numpy())
    st = {"trk": None, "next": 0, "refs": {}}
    own = torch.empty((1, 56), dtype=torch.uint8, device=dev)

    def ref_of(i):
        t = st["trk"]
        if t is not None:
            r = t.process(hand[i].numpy(), frame_index=i, want_hand=True)
        else:
            r = m.process(hand[i].numpy(), frame_index=i, want_hand=True)
        st["refs"][i] = r
        return r

    def one_frame_calls(n, label):
        for _ in range(n):
            i = st["next"]
            st["next"] += 1
            print(label, "frame", i, flush=True)
            if i % 2 == 0:
                o = ctx.process_frames(hd[i:i + 1].contiguous(), want_fizi=True, want_hand=True)
                torch.cuda.synchronize()
                p = fizi.pointer_dict(fizi.pointers_to_numpy(o["pointers"])[0])
                fz = fizi.unpack_bits(o["fizi"], W)[0]
                hb = fizi.unpack_bits(o["hand"], W)[0]
            else:
                ctx.process_into(hd[i:i + 1].contiguous(), 1, pointers=own)
                p = ctx.get_pointer(i)
                fz = hb = None
            r = ref_of(i)
            assert p == r["pointer"], (label, i, p, r["pointer"])
            if fz is not None:
                assert np.array_equal(fz, r["fizi"]), (label, i)
                assert np.array_equal(hb, r["hand"]), (label, i)

    one_frame_calls(12, "first run")
    # a call of three frames takes a slot with a table of three jobs
    i0 = st["next"]
    st["next"] += 3
    o = ctx.process_frames(hd[i0:i0 + 3].contiguous(), want_fizi=True)
    torch.cuda.synchronize()
    for k in range(3):
        r = ref_of(i0 + k)
        assert fizi.pointer_dict(fizi.pointers_to_numpy(o["pointers"])[k]) == r["pointer"], i0 + k
        assert np.array_equal(fizi.unpack_bits(o["fizi"], W)[k], r["fizi"]), i0 + k
    one_frame_calls(10, "after a three-frame call")
    # partial re-learning with the oracle's masks of four earlier frames
    masks = np.stack([st["refs"][k]["fizi"] for k in range(4)])
    ctx.relearn_background(hd[:4].contiguous(), fizi.pack_bits(masks, device=dev))
    m.relearn(hand[:4].numpy(), masks)
    one_frame_calls(10, "after re-learning")
    # learning again from other background frames
    ctx.learn_background(bg2.to(dev))
    m.learn(bg2.numpy())
    one_frame_calls(10, "after learning again")
    ctx.set_tracking(True)
    st["trk"] = oracle.Tracker(m)
    one_frame_calls(10, "tracked")
    ctx.set_short_bands(False)
    one_frame_calls(9, "tracked, 8-row bands")
    assert st["next"] == 64
    ctx.close()


@pytest.mark.parametrize("track", [False, True])
def test_one_frame_calls_on_two_streams(track):
    """Back-to-back one-frame calls alternating between two streams, outputs
    read once at the end: each call is ordered after the previous one (whose
    component stage zeroed the accumulators its slot's next call relies on)
    whatever stream it comes on."""
    from oracle import oracle
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, _, hand = _scene()
    hd = hand.to(dev)
    ctx = fizi.Context(W, H, chunk=4, device=dev)
    ctx.learn_background(bg.to(dev))
    ctx.set_tracking(track)
    m = oracle.Model(W, H)
    m.learn(bg.numpy())
    t = oracle.Tracker(m) if track else None
    streams = [torch.cuda.current_stream(dev), torch.cuda.Stream(device=dev)]
    streams[1].wait_stream(streams[0])
    outs = []
    for i in range(20):
        s = streams[i % 2]
        with torch.cuda.stream(s):
            outs.append(ctx.process_frames(hd[i:i + 1].contiguous(), want_fizi=True, stream=s))
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        r = t.process(hand[i].numpy(), frame_index=i) if t else m.process(hand[i].numpy(), frame_index=i)
        assert fizi.pointer_dict(fizi.pointers_to_numpy(o["pointers"])[0]) == r["pointer"], (track, i)
        assert np.array_equal(fizi.unpack_bits(o["fizi"], W)[0], r["fizi"]), (track, i)
    ctx.close()
