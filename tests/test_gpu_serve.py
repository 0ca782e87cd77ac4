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
    from paper_1907_04393_amd import fizi
    by = {s.sid: s for s in sessions}
    ctxs = {}
    for r in results:
        s = by[r.sid]
        if r.sid not in ctxs:
            c = fizi.Context(s.width, s.height, chunk=1, device=dev)
            c.learn_background(s.bg())
            ctxs[r.sid] = c
        out = ctxs[r.sid].process_frames(s.frames(r.seq).unsqueeze(0).contiguous(), want_fizi=False)
        torch.cuda.synchronize()
        ref = fizi.pointer_dict(fizi.pointers_to_numpy(out["pointers"])[0])
        got = dict(r.pointer)
        got["frame_index"] = ref["frame_index"] = 0
        assert got == ref, (r.sid, r.seq)


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
