"""Workload builders shared by the benchmark and the full-size tests.

batched(): the multi-stream workload - 64 camera streams whose resolutions
are drawn by seed from {640x480, 1280x720, 1920x1080, 3840x2160}, each with
its own background (learned from 30 user-free frames), Lissajous hand path,
phase and brightness drift; a small pool of resident hand frames per stream
is cycled through the steps.
"""
from __future__ import annotations

import torch

from . import fizi, scene

# launch mode of the multi-stream benchmark before autotuning: steps
# software-pipelined across frames (a step's outputs are complete after the
# next step or a flush)
BATCH_MODE = fizi.BATCH_PIPELINED


def batched(n_streams=64, pool=4, n_bg=30, device="cuda", seed=2, log=None):
    specs = scene.batched_streams(n_streams, seed=seed)
    scenes = [scene.Scene(sp, device=device) for sp in specs]
    batch = fizi.Batch([(sp.width, sp.height) for sp in specs], device=device)
    frames = []
    for i, sc in enumerate(scenes):
        bg = sc.bg_frames(0, n_bg)
        batch.learn(i, bg)
        frames.append(sc.hand_frames(0, pool))
        if log and (i + 1) % 16 == 0:
            log(f"  learned {i + 1}/{n_streams} streams")
    torch.cuda.synchronize()
    px = sum(sp.width * sp.height for sp in specs)
    return dict(specs=specs, scenes=scenes, batch=batch, frames=frames, pool=pool, px_per_step=px)


def step_frames(w, k):
    """Frames of step k (one per stream, cycling through the pool)."""
    return [f[k % w["pool"]] for f in w["frames"]]


def serving(n_streams=256, duration=10.0, rate=30.0, pool=4, n_bg=8, budget=None, session_len=None,
            lanes=2, device="cuda", seed=4, log=None):
    """The serving workload: n_streams cameras (resolutions drawn by seed
    from 640x480 .. 3840x2160) sending frames at `rate` per second with
    Poisson arrivals, over `duration` seconds. With a budget (bytes) the slot
    pool is sized to it; with session_len, sessions come and go (start
    uniform over the run, each lasting session_len seconds) so that slots
    are reused. Returns (sessions, backend, admitted, px_of)."""
    import numpy as np
    from . import serve
    specs = scene.batched_streams(n_streams, seed=seed)
    scenes = [scene.Scene(sp, device=device) for sp in specs]
    rng = np.random.default_rng(seed)
    pools = []
    for i, sc in enumerate(scenes):
        pools.append(sc.hand_frames(0, pool))
        if log and (i + 1) % 64 == 0:
            log(f"  rendered {i + 1}/{n_streams} streams")
    sessions = []
    for i, (sp, sc) in enumerate(zip(specs, scenes)):
        start = 0.0 if session_len is None else float(rng.uniform(0.0, max(0.0, duration - session_len)))
        end = duration if session_len is None else start + session_len
        arr = serve.poisson_arrivals(rate, start, end, rng)
        sessions.append(serve.Session(i, sp.width, sp.height,
                                      (lambda sc=sc: sc.bg_frames(0, n_bg)),
                                      (lambda k, p=pools[i]: p[k % pool]), arr, start=start))
    classes = sorted({(sp.width, sp.height) for sp in specs})
    counts = {c: sum(1 for sp in specs if (sp.width, sp.height) == c) for c in classes}
    size = {c: fizi.Batch.stream_bytes(c) for c in classes}
    plan = serve.plan_slots(classes, counts, size, budget if budget is not None else float("inf"))
    slot_geoms = [c for c in classes for _ in range(plan[c])]
    be = serve.GpuBackend(slot_geoms, lanes=lanes, device=device)
    admitted = {}
    if session_len is None:
        # every camera is admitted and learned before the clock starts
        for s in sessions:
            slot = be.acquire(s.width, s.height)
            if slot is None:
                continue
            be.learn(slot, s.bg())
            admitted[s.sid] = slot
        torch.cuda.synchronize()
    px_of = {sp_i: sp.width * sp.height for sp_i, sp in enumerate(specs)}
    return sessions, be, admitted, px_of, plan, size
