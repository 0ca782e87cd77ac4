"""Pipelined context calls (fizi_set_pipelined): a call leaves the
morphology and components of its last internal batch running on the
context's side stream, and the next call, or a flush, completes them. On the
same frames every I_FIZI bit, hand bit and pointer equals the oracle's:
through calls of several batches and of one, a switch of stream between
calls, tracking across calls, get_pointer before any flush, one output
buffer reused by every call, and partial re-learning from a call that is
still pending."""
import numpy as np
import pytest
import torch

from helpers import need_gpu

pytestmark = pytest.mark.gpu

W, H = 320, 240
SIZES = [20, 5, 16, 1, 19]     # calls of several internal batches of 8, and of one


def _scene():
    from paper_1907_04393_amd import scene
    sp = scene.SceneSpec(W, H, sigma=3, seed=(9, 7, 0, 0), distractors=2)
    sc = scene.Scene(sp)
    return sc.bg_frames(0, 20), sc.hand_frames(0, sum(SIZES))


def _oracle(bg, hand, track):
    from oracle import oracle
    m = oracle.Model(W, H)
    m.learn(bg.numpy())
    if track:
        t = oracle.Tracker(m)
        return [t.process(hand[k].numpy(), frame_index=k, want_hand=True) for k in range(hand.shape[0])]
    return [m.process(hand[k].numpy(), frame_index=k, want_hand=True) for k in range(hand.shape[0])]


def _ctx(bg, dev, track):
    from paper_1907_04393_amd import fizi
    ctx = fizi.Context(W, H, chunk=8, device=dev)
    ctx.learn_background(bg.to(dev))
    ctx.set_tracking(track)
    ctx.set_pipelined(True)
    return ctx


@pytest.mark.parametrize("track", [False, True])
def test_pipelined_calls_match_oracle(track):
    """Outputs allocated per call, read after a flush; the third call on a
    second stream."""
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, hand = _scene()
    ref = _oracle(bg, hand, track)
    ctx = _ctx(bg, dev, track)
    hd = hand.to(dev)
    other = torch.cuda.Stream(device=dev)
    outs, f0 = [], 0
    for i, n in enumerate(SIZES):
        print(f"pipelined call {i}: frames {f0}..{f0 + n - 1}, track {track}", flush=True)
        s = other if i == 2 else torch.cuda.current_stream(dev)
        if i == 2:
            s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s):
            outs.append(ctx.process_frames(hd[f0:f0 + n].contiguous(), want_fizi=True, want_hand=True,
                                           stream=s))
        if i == 2:
            torch.cuda.current_stream(dev).wait_stream(s)
        f0 += n
    ctx.flush()
    torch.cuda.synchronize()
    f0 = 0
    for o, n in zip(outs, SIZES):
        ptrs = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(o["pointers"])]
        fz = fizi.unpack_bits(o["fizi"], W)
        hb = fizi.unpack_bits(o["hand"], W)
        for k in range(n):
            r = ref[f0 + k]
            assert ptrs[k] == r["pointer"], (f0 + k, ptrs[k], r["pointer"])
            assert np.array_equal(fz[k], r["fizi"]), f0 + k
            assert np.array_equal(hb[k], r["hand"]), f0 + k
        f0 += n


def test_pipelined_get_pointer_and_reused_buffer():
    """One pointer buffer for every call (its earlier contents are
    overwritten only by later calls' own work, in order on the side stream);
    get_pointer waits on its own, before any flush."""
    dev = need_gpu()
    bg, hand = _scene()
    ref = _oracle(bg, hand, False)
    ctx = _ctx(bg, dev, False)
    hd = hand.to(dev)
    ptrs = torch.empty((max(SIZES), 56), dtype=torch.uint8, device=dev)
    f0 = 0
    for i, n in enumerate(SIZES):
        print(f"reused buffer call {i}: frames {f0}..{f0 + n - 1}", flush=True)
        ctx.process_into(hd[f0:f0 + n].contiguous(), n, pointers=ptrs)
        for k in (f0, f0 + n - 1):
            assert ctx.get_pointer(k) == ref[k]["pointer"], k
        f0 += n
    for k in range(f0):
        assert ctx.get_pointer(k) == ref[k]["pointer"], k
    ctx.flush()
    torch.cuda.synchronize()


def test_switching_pipelining_off_completes_pending_work():
    """set_pipelined(False) waits for the pending call; later calls complete
    their outputs themselves."""
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, hand = _scene()
    ref = _oracle(bg, hand, False)
    ctx = _ctx(bg, dev, False)
    hd = hand.to(dev)
    a = ctx.process_frames(hd[:20].contiguous(), want_fizi=True)
    ctx.set_pipelined(False)
    b = ctx.process_frames(hd[20:25].contiguous(), want_fizi=True)
    torch.cuda.synchronize()
    for o, lo, n in ((a, 0, 20), (b, 20, 5)):
        ptrs = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(o["pointers"])]
        fz = fizi.unpack_bits(o["fizi"], W)
        for k in range(n):
            assert ptrs[k] == ref[lo + k]["pointer"], lo + k
            assert np.array_equal(fz[k], ref[lo + k]["fizi"]), lo + k


def test_relearn_from_a_pending_call():
    """Partial re-learning fed with the masks of a pipelined call that has
    not been flushed: the context orders it after that call's last batch, so
    the model, and the next call's outputs, equal those of a context whose
    calls complete their own outputs."""
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, hand = _scene()
    hd = hand.to(dev)
    res = []
    for pipelined in (False, True):
        ctx = fizi.Context(W, H, chunk=8, device=dev)
        ctx.learn_background(bg.to(dev))
        ctx.set_pipelined(pipelined)
        a = ctx.process_frames(hd[:20].contiguous(), want_fizi=True)
        ctx.relearn_background(hd[:20].contiguous(), a["fizi"])
        b = ctx.process_frames(hd[20:40].contiguous(), want_fizi=True)
        ctx.flush()
        torch.cuda.synchronize()
        bgmin, bgmax, _ = ctx.model()
        res.append((bgmin.cpu().numpy(), bgmax.cpu().numpy(), b["pointers"].cpu().numpy(),
                    b["fizi"].cpu().numpy()))
    for x, y in zip(res[0], res[1]):
        assert np.array_equal(x, y)
