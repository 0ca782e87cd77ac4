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

# launch configuration of the multi-stream benchmark
BATCH_MODE = fizi.BATCH_PERSISTENT_GRAPH


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
