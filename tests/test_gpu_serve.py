"""Serving on the GPU: continuous batching over two lanes; every served
frame's pointer equals the same frame processed alone, and a tight budget
defers admissions without dropping frames."""
import numpy as np
import pytest
import torch

from helpers import need_gpu

pytestmark = pytest.mark.gpu


def _sessions(dev, n, dur, session_len=None, seed=0, rate=30.0):
    from paper_1907_04393_amd import scene, serve
    rng = np.random.default_rng(seed)
    sizes = [(320, 240), (640, 480), (128, 96)]
    out, scenes = [], []
    for i in range(n):
        w, h = sizes[i % 3]
        sc = scene.Scene(scene.SceneSpec(w, h, sigma=3, seed=(11, seed, i, 0)), device=dev)
        pool = sc.hand_frames(0, 4)
        start = 0.0 if session_len is None else float(rng.uniform(0, dur - session_len))
        end = dur if session_len is None else start + session_len
        arr = serve.poisson_arrivals(rate, start, end, rng)
        out.append(serve.Session(i, w, h, (lambda sc=sc: sc.bg_frames(0, 6)), (lambda k, p=pool: p[k % 4]),
                                 arr, start=start))
        scenes.append(sc)
    return out, scenes


def _check_alone(sessions, results, dev):
    """Every served pointer equals the oracle's for that session's learning
    frames and the same hand frame, and the HIP plain path's for the frame
    processed alone."""
    from oracle import oracle
    from paper_1907_04393_amd import fizi
    by = {s.sid: s for s in sessions}
    ctxs, models, seen = {}, {}, {}
    for r in results:
        s = by[r.sid]
        if r.sid not in ctxs:
            bg = s.bg()
            c = fizi.Context(s.width, s.height, chunk=1, device=dev)
            c.learn_background(bg)
            ctxs[r.sid] = c
            m = oracle.Model(s.width, s.height)
            m.learn(bg.cpu().numpy())
            models[r.sid] = m
        frame = s.frames(r.seq)
        got = dict(r.pointer)
        got["frame_index"] = 0
        # the oracle, on the bytes the server processed
        if (r.sid, r.seq % 4) not in seen:
            seen[(r.sid, r.seq % 4)] = models[r.sid].process(frame.cpu().numpy(), frame_index=0)["pointer"]
        assert got == seen[(r.sid, r.seq % 4)], ("oracle", r.sid, r.seq)
        out = ctxs[r.sid].process_frames(frame.unsqueeze(0).contiguous(), want_fizi=False)
        torch.cuda.synchronize()
        ref = fizi.pointer_dict(fizi.pointers_to_numpy(out["pointers"])[0])
        ref["frame_index"] = 0
        assert got == ref, ("alone", r.sid, r.seq)


def test_mix_equals_alone():
    from paper_1907_04393_amd import serve
    dev = need_gpu()
    # 9 streams at 2000 frames/s each: arrivals overlap device work, so steps
    # carry frames of several streams
    sessions, _ = _sessions(dev, 9, 0.3, rate=2000.0)
    be = serve.GpuBackend([(s.width, s.height) for s in sessions], lanes=2, device=dev)
    srv = serve.Server(be)
    res = srv.run(sessions, 0.3)
    want = {(s.sid, k) for s in sessions for k in range(len(s.arrivals))}
    assert {(r.sid, r.seq) for r in res} == want and len(res) == len(want)
    print("steps", srv.steps, "frames", len(res), "largest step", srv.max_step, flush=True)
    assert srv.max_step > 1 and srv.steps < len(res)
    _check_alone(sessions, res, dev)
    be.close()


def test_frames_made_on_demand():
    """Frames rendered on the current stream at the moment the server asks
    for them (no pool made ahead): the lanes wait for them and keep their
    memory alive, and the results still equal the oracle's."""
    from paper_1907_04393_amd import serve
    dev = need_gpu()
    sessions, scenes = _sessions(dev, 4, 0.2, rate=500.0, seed=5)
    for s, sc in zip(sessions, scenes):
        s.frames = (lambda k, sc=sc: sc.hand_frame(k % 4))
    be = serve.GpuBackend([(s.width, s.height) for s in sessions], lanes=2, device=dev)
    srv = serve.Server(be)
    res = srv.run(sessions, 0.2)
    want = {(s.sid, k) for s in sessions for k in range(len(s.arrivals))}
    assert {(r.sid, r.seq) for r in res} == want
    _check_alone(sessions, res, dev)
    be.close()


def test_tight_budget_on_gpu():
    from paper_1907_04393_amd import serve
    dev = need_gpu()
    sessions, _ = _sessions(dev, 8, 1.5, session_len=0.4, seed=2)
    be = serve.GpuBackend([(320, 240), (640, 480), (128, 96)] * 1, lanes=2, device=dev)
    srv = serve.Server(be)
    res = srv.run(sessions, 1.5)
    want = {(s.sid, k) for s in sessions for k in range(len(s.arrivals))}
    assert {(r.sid, r.seq) for r in res} == want
    assert srv.deferred
    _check_alone(sessions, res, dev)
    be.close()
