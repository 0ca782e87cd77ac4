#!/usr/bin/env python3
"""Benchmark of the FIZI/Mouse pipeline on one MI355X.

Workload (plain method, one camera stream): 1920x1080 RGB uint8 frames of
the synthetic scene (noise sigma 5, two static skin-coloured distractors,
i.i.d. brightness gain in [0.8, 1.2]); the background is learned from 50
user-free frames, then hand frames are processed. A step is one
process_frames call over a batch of resident hand frames (every stage:
gain, classify, morphology, components, pointer, plus the copy of the
pointers to the host ring).

Printed: one JSON line with Mpixel/s (value), frames/s, p50/p99 latency of
single-frame calls, the roofline of the dominant kernel (classify) from HIP
events around its launches in the timed region, and the CPU oracle timed on a
bounded sample of the same frames.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s and frames/s per GPU (% of HBM roofline); p99 frame latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per pixel: frame 3 + background min/max 6 + reference
# luminance 2/8 + I_FIZI bits 1/8 (whole path); classify alone reads the
# frame and the model and writes the raw mask bits: 3 + 6 + 1/8
PATH_BYTES_PER_PX = 9.375
CLASSIFY_BYTES_PER_PX = 9.125


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256, help="frames per step")
    ap.add_argument("--chunk", type=int, default=None, help="frames per internal launch batch")
    ap.add_argument("--latency-frames", type=int, default=300)
    ap.add_argument("--cpu-frames", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (the pipeline has no multi-GPU path); "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1907_04393_amd import fizi, scene

    dev = torch.device("cuda:0")
    spec = scene.hd_plain()
    W, H = spec.width, spec.height
    px = W * H
    chunk = args.chunk or scene.HD_CHUNK
    log(f"workload 1920x1080 plain: batch {args.batch}, chunk {chunk}")
    sc = scene.Scene(spec, device=dev)
    bg = sc.bg_frames(0, spec.n_bg)
    pool = sc.hand_frames(0, args.batch)
    torch.cuda.synchronize()
    ctx = fizi.Context(W, H, chunk=chunk, device=dev)
    ctx.learn_background(bg)
    stream = torch.cuda.current_stream()
    fz = torch.empty((args.batch, H, W // 64), dtype=torch.int64, device=dev)
    ptrs = torch.empty((args.batch, 56), dtype=torch.uint8, device=dev)

    def step():
        ctx.process_into(pool, args.batch, fizi=fz, pointers=ptrs, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    ctx.stage_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = ctx.stage_times()
    ctx.stage_timing(False)
    log("timed region done", stages)

    sec_per_step = (t1 - t0) / args.steps
    fps = args.batch / sec_per_step
    mpxs = fps * px / 1e6
    cls_ms, cls_n = stages["classify"]
    frames_per_launch = args.batch / max(1, -(-args.batch // chunk))
    cls_avg_s = cls_ms / 1e3 / max(1, cls_n)
    cls_bytes = CLASSIFY_BYTES_PER_PX * px * (args.batch * args.steps / max(1, cls_n))
    achieved = cls_bytes / cls_avg_s / 1e9 if cls_avg_s > 0 else 0.0

    # single-frame latency: submit one frame, wait for its pointer on the host
    lat = []
    torch.cuda.synchronize()
    ctx_l = fizi.Context(W, H, chunk=1, device=dev)
    ctx_l.learn_background(bg)
    one_ptr = torch.empty((1, 56), dtype=torch.uint8, device=dev)
    for i in range(args.latency_frames + 10):
        f = pool[i % args.batch:i % args.batch + 1]
        t = time.perf_counter()
        ctx_l.process_into(f, 1, pointers=one_ptr, stream=stream)
        ctx_l.get_pointer(i)
        if i >= 10:
            lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat)
    log(f"latency p50 {np.percentile(lat, 50):.3f} ms p99 {np.percentile(lat, 99):.3f} ms")

    # parity spot check of the timed outputs against the oracle
    cpu = None
    if not args.no_cpu:
        from oracle import oracle
        m = oracle.Model(W, H)
        m.learn(bg.cpu().numpy())
        hand = pool[:args.cpu_frames].cpu().numpy()
        got = fizi.pointers_to_numpy(ptrs)
        t = time.perf_counter()
        for k in range(hand.shape[0]):
            r = m.process(hand[k], frame_index=0)
            if k < 4:
                g = fizi.pointer_dict(got[k])
                r["pointer"]["frame_index"] = g["frame_index"]
                assert g == r["pointer"], (k, g, r["pointer"])
        dt = time.perf_counter() - t
        cpu = {"value": round(hand.shape[0] * px / dt / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{hand.shape[0]} frames 1920x1080 of the timed batch, single thread, "
                         f"{dt:.1f} s"}
        log("cpu oracle", cpu)

    out = {
        "metric": METRIC,
        "value": round(mpxs, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_per_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "plain method, one 1920x1080 RGB uint8 stream, 50 learned "
                               "background frames, hand frames with 2 distractors and "
                               "brightness gain U[0.8,1.2]",
                   "frames_per_step": args.batch, "chunk_frames": chunk},
        "frames_per_s": round(fps, 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "mode": "one frame per call, pointer read back on the host"},
        "path_roofline_frac": round(mpxs * 1e6 * PATH_BYTES_PER_PX / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": {"bound": "hbm", "kernel": "k_classify",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_launch_us": round(cls_avg_s * 1e6, 2),
                     "frames_per_launch": frames_per_launch},
        "stage_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items() if v[1]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
