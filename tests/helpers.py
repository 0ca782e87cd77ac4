"""Shared test drivers: run the same frames through the HIP path (C ABI) and
the CPU oracle and compare every output bit for bit."""
from __future__ import annotations

import numpy as np
import torch


def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def gpu_run(bg, hand, params: dict, chunk=16, learn_split=None, want_hand=True, short_bands=True):
    """bg, hand: (n, H, W, 3) uint8 CPU tensors. Returns a dict of numpy
    outputs of the HIP path."""
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    H, W = bg.shape[1], bg.shape[2]
    ctx = fizi.Context(W, H, fizi.default_params(**params), chunk=chunk, device=dev)
    ctx.set_short_bands(short_bands)
    bgd = bg.to(dev).contiguous()
    if learn_split:
        s = 0
        for k, n in enumerate(learn_split):
            ctx.learn_background(bgd[s:s + n].contiguous(), reset=(k == 0))
            s += n
    else:
        ctx.learn_background(bgd)
    out = ctx.process_frames(hand.to(dev).contiguous(), want_fizi=True, want_hand=want_hand)
    torch.cuda.synchronize()
    bgmin, bgmax, yref = ctx.model()
    res = dict(ctx=ctx,
               bgmin=bgmin.cpu().numpy(), bgmax=bgmax.cpu().numpy(),
               yref=yref.cpu().numpy().view(np.uint16),
               pointers=[fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(out["pointers"])],
               fizi=fizi.unpack_bits(out["fizi"], W))
    if want_hand:
        res["hand"] = fizi.unpack_bits(out["hand"], W)
    return res


def oracle_run(bg, hand, params: dict, want_hand=True, frames=None):
    from oracle import oracle
    H, W = bg.shape[1], bg.shape[2]
    m = oracle.Model(W, H, oracle.params(**params))
    m.learn(bg.numpy())
    idx = range(hand.shape[0]) if frames is None else frames
    outs = {k: m.process(hand[k].numpy(), frame_index=k, want_hand=want_hand) for k in idx}
    return m, outs


def compare(g, m, outs, label=""):
    assert np.array_equal(g["bgmin"], m.bgmin), f"{label} bgmin"
    assert np.array_equal(g["bgmax"], m.bgmax), f"{label} bgmax"
    assert np.array_equal(g["yref"], m.yref), f"{label} yref"
    for k, o in outs.items():
        assert g["pointers"][k] == o["pointer"], (label, k, g["pointers"][k], o["pointer"])
        if not np.array_equal(g["fizi"][k], o["fizi"]):
            bad = np.argwhere(g["fizi"][k] != o["fizi"])
            raise AssertionError(f"{label} frame {k}: fizi differs at {len(bad)} px, first {bad[:5].tolist()}")
        if "hand" in g and "hand" in o:
            assert np.array_equal(g["hand"][k], o["hand"]), f"{label} frame {k} hand"
