#!/usr/bin/env python3
"""Benchmark of the FIZI/Mouse pipeline on one MI355X.

Headline workload (batched form): 64 camera streams whose resolutions are
drawn by seed from {640x480, 1280x720, 1920x1080, 3840x2160}, each with its
own learned background, hand path and brightness drift. A step is one frame
for every stream through the whole per-frame path (gain, classify,
morphology, components, pointer): four kernels replayed from one hipGraph
(with --autotune, the launch shape the batch's autotuner picks on these
frames). Inputs are resident in HBM before the timed region.

Also measured, next to it: the plain single-stream form on 1920x1080 frames
(throughput of process_frames over resident frames, and the latency of
single-frame calls with the pointer read back on the host).

Printed: one JSON line. `roofline` is the dominant kernel's (classify's, or
the fused kernel's in a persistent launch shape) algorithmic bytes per launch
over its average duration, taken from the kernel's own dispatch events;
`cpu_baseline` is the CPU oracle on a bounded sample of the same frames.
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
# algorithmic bytes per pixel of the whole per-frame path: frame 3 +
# background min/max 6 + reference luminance 2/8 + I_FIZI bits 1/8
PATH_BYTES_PER_PX = 9.375
# of the classify kernel: frame 3 + background min/max 6 + raw mask bits 1/8
CLASSIFY_BYTES_PER_PX = 9.125


LAUNCH_NAMES = {0: "four kernels, direct launches", 1: "four kernels replayed from a hipGraph",
                2: "persistent fused kernel", 3: "persistent fused kernel, hipGraph"}

# measured HBM bytes per launch of the dominant kernel on this workload:
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (the factors a 1 GiB -> 1 GiB
# elementwise kernel gives), keyed by kernel; valid only for the kernel code
# the counters were taken on
TRAFFIC = {"k_classify<4> (I_R1, I_R2, I_R3 per pixel)": 1714.1e6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(a, q):
    import numpy as np
    return round(float(np.percentile(np.asarray(a), q)), 4)


def bench_batched(args, torch, fizi, workloads):
    dev = torch.device("cuda:0")
    log("building the 64-stream workload")
    w = workloads.batched(64, pool=args.pool, device=dev, log=log)
    b, n, px = w["batch"], len(w["specs"]), w["px_per_step"]
    ptrs = torch.empty((n, 56), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    b.set_mode(workloads.BATCH_MODE)
    if args.autotune:
        best, ms = b.autotune(workloads.step_frames(w, 0), ptrs, steps=5, stream=stream)
        log(f"autotuned launch shape {best}: {ms:.3f} ms/step")
    tuning = b.get_tuning()
    for k in range(args.warmup):
        b.step(workloads.step_frames(w, k), ptrs, stream=stream)
    torch.cuda.synchronize()
    assert b.status() == 0
    log("warmup done; timed region")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        b.step(workloads.step_frames(w, k), ptrs, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert b.status() == 0
    sec = (t1 - t0) / args.steps

    # per-step latency: submit a step, wait for its pointers on the host
    host = torch.empty((n, 56), dtype=torch.uint8, pin_memory=True)
    lat = []
    for k in range(args.latency_steps):
        t = time.perf_counter()
        b.step(workloads.step_frames(w, k), ptrs, stream=stream)
        host.copy_(ptrs, non_blocking=True)
        stream.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)

    # the same step with every stream tracked (temporal tracking, one frame
    # per stream per step: the component stage stays parallel)
    for i in range(n):
        b.set_tracking(i, True)
    for k in range(2):
        b.step(workloads.step_frames(w, k), ptrs, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        b.step(workloads.step_frames(w, k), ptrs, stream=stream)
    torch.cuda.synchronize()
    track_sec = (time.perf_counter() - t0) / args.steps
    for i in range(n):
        b.set_tracking(i, False)

    # kernel durations from their own dispatch events: the same kernels and
    # grids, launched directly so that the events can be attached (the
    # persistent kernel reports its whole launch under "classify")
    persistent = tuning["mode"] in (fizi.BATCH_PERSISTENT, fizi.BATCH_PERSISTENT_GRAPH)
    b.set_mode(fizi.BATCH_PERSISTENT if persistent else fizi.BATCH_DIRECT)
    b.stage_timing(True)
    for k in range(args.steps):
        b.step(workloads.step_frames(w, k), ptrs, stream=stream)
    torch.cuda.synchronize()
    st = b.stage_times()
    b.stage_timing(False)
    b.set_mode(tuning["mode"])
    assert b.status() == 0
    stages_us = {k: round(v[0] * 1e3 / v[1], 2) for k, v in st.items() if v[1]}
    k_ms, k_n = st["classify"]
    k_avg = k_ms / 1e3 / max(1, k_n)
    if persistent:
        kernel, bpp = "k_step (fused gain, classify, morphology, components)", PATH_BYTES_PER_PX
    else:
        kernel, bpp = f"k_classify<{tuning['cls_iters']}> (I_R1, I_R2, I_R3 per pixel)", CLASSIFY_BYTES_PER_PX
    achieved = bpp * px / k_avg / 1e9
    return dict(w=w, px=px, n=n, sec=sec, lat=lat, k_avg=k_avg, achieved=achieved, kernel=kernel, bpp=bpp,
                tuning=tuning, stages_us=stages_us, track_sec=track_sec)


def bench_plain(args, torch, fizi, scene):
    dev = torch.device("cuda:0")
    spec = scene.hd_plain()
    W, H = spec.width, spec.height
    sc = scene.Scene(spec, device=dev)
    bg = sc.bg_frames(0, spec.n_bg)
    pool = sc.hand_frames(0, args.plain_batch)
    ctx = fizi.Context(W, H, chunk=scene.HD_CHUNK, device=dev)
    ctx.learn_background(bg)
    stream = torch.cuda.current_stream()
    ptrs = torch.empty((args.plain_batch, 56), dtype=torch.uint8, device=dev)
    for _ in range(2):
        ctx.process_into(pool, args.plain_batch, pointers=ptrs, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        ctx.process_into(pool, args.plain_batch, pointers=ptrs, stream=stream)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    fps = args.plain_batch / sec
    # temporal tracking: the component stage of a call's frames runs in order
    ctx.set_tracking(True)
    ctx.process_into(pool, args.plain_batch, pointers=ptrs, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.process_into(pool, args.plain_batch, pointers=ptrs, stream=stream)
    torch.cuda.synchronize()
    track_fps = args.plain_batch * reps / (time.perf_counter() - t0)
    ctx.set_tracking(False)
    ctx1 = fizi.Context(W, H, chunk=1, device=dev)
    ctx1.learn_background(bg)
    one = torch.empty((1, 56), dtype=torch.uint8, device=dev)
    lat = []
    for i in range(args.latency_frames + 10):
        f = pool[i % args.plain_batch:i % args.plain_batch + 1]
        t = time.perf_counter()
        ctx1.process_into(f, 1, pointers=one, stream=stream)
        ctx1.get_pointer(i)
        if i >= 10:
            lat.append((time.perf_counter() - t) * 1e3)
    return {"workload": "one 1920x1080 stream, frames processed in batches of "
                        f"{args.plain_batch} (internal launches of {scene.HD_CHUNK} frames)",
            "Mpixel_per_s": round(fps * W * H / 1e6, 1), "frames_per_s": round(fps, 1),
            "tracking_frames_per_s": round(track_fps, 1),
            "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99),
                           "mode": "one frame per call, pointer read back on the host"}}


def bench_serving(args, torch, workloads, budget=None, session_len=None, duration=None):
    from paper_1907_04393_amd import serve
    duration = duration or args.serve_seconds
    sessions, be, admitted, px_of, plan, size = workloads.serving(
        256, duration=duration, budget=budget, session_len=session_len, log=log)
    srv = serve.Server(be)
    t0 = time.perf_counter()
    res = srv.run(sessions, duration, admitted=admitted)
    wall = time.perf_counter() - t0
    out = serve.summarize(res, px_of, wall)
    out.update({"streams": len(sessions), "seconds": duration,
                "offered_frames": sum(len(s.arrivals) for s in sessions),
                "steps": srv.steps, "slots": {f"{c[0]}x{c[1]}": n for c, n in plan.items()},
                "state_GB": round(sum(plan[c] * size[c] for c in plan) / 1e9, 2),
                "deferred_sessions": len(srv.deferred)})
    be.close()
    torch.cuda.synchronize()
    return out


def bench_learn(args, torch, fizi, scene):
    """Background learning, 50 frames of 1920x1080: every frame is read once
    (3 B/px), the model is read and written once (12 B/px per call)."""
    dev = torch.device("cuda:0")
    spec = scene.hd_plain()
    W, H, n = spec.width, spec.height, spec.n_bg
    bg = scene.Scene(spec, device=dev).bg_frames(0, n)
    ctx = fizi.Context(W, H, chunk=1, device=dev)
    ctx.learn_background(bg)
    torch.cuda.synchronize()
    ctx.stage_timing(True)
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.learn_background(bg)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    ms, launches = ctx.stage_times()["learn"]
    k_s = ms / 1e3 / max(1, launches)
    byts = W * H * (3 * n + 12)
    out = {"workload": f"{n} frames 1920x1080 per call", "ms_per_call": round(sec * 1e3, 3),
           "frames_per_s": round(n / sec, 1), "minmax_kernel_us": round(k_s * 1e6, 1),
           "minmax_GBps": round(byts / k_s / 1e9, 1), "minmax_frac": round(byts / k_s / 1e9 / HBM_PEAK_GBS, 4)}
    # partial re-learning: running frames fed back with their I_FIZI masks
    # (model 12 B/px once per call, each frame 3 B/px + its mask 1/8 B/px)
    hand = scene.Scene(spec, device=dev).hand_frames(0, 8)
    bits = ctx.process_frames(hand, want_fizi=True)["fizi"]
    torch.cuda.synchronize()
    ctx.stage_times()
    for k in (1, 8):
        ctx.relearn_background(hand[:k], bits[:k])
        torch.cuda.synchronize()
        ctx.stage_times()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.relearn_background(hand[:k], bits[:k])
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        ms, launches = ctx.stage_times()["learn"]
        k_s = ms / 1e3 / max(1, launches)
        byts = W * H * ((3 + 1 / 8) * k + 12)
        out[f"relearn_{k}_frames"] = {"ms_per_call": round(sec * 1e3, 3), "kernel_us": round(k_s * 1e6, 1),
                                      "GBps": round(byts / k_s / 1e9, 1),
                                      "frac": round(byts / k_s / 1e9 / HBM_PEAK_GBS, 4)}
    ctx.stage_timing(False)
    return out


def bench_soft(args, torch, scene):
    """Soft mask on the calibration workload (32 frames 1280x720): forward
    (3 B in, 4 B out per px), backward from dL/dm (3 + 4 B in), fused BCE
    loss and gradient (3 + 1 B in)."""
    from paper_1907_04393_amd import soft
    dev = torch.device("cuda:0")
    f, gt = scene.Scene(scene.calibration(), device=dev).hand_frames(0, 32, with_gt=True)
    gt = gt.to(torch.uint8)
    npx = f.numel() // 3
    prm = torch.tensor((102.0, 153.0, 208.3, 10.0, 133.3, 2.5), dtype=torch.float64)
    m = soft.soft_forward(f, prm, 0.5)
    dm = torch.randn_like(m)
    soft.soft_backward(f, dm, prm, 0.5)
    torch.cuda.synchronize()
    reps = 20
    out = {"workload": "32 frames 1280x720 (29.5 Mpx), T = 0.5"}
    for name, fn, bpp in (("forward", lambda: soft.soft_forward(f, prm, 0.5, out=m), 7),
                          ("backward", lambda: soft.soft_backward(f, dm, prm, 0.5), 7),
                          ("fused_bce", lambda: soft.soft_bce(f, gt, prm, 0.5), 4)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        out[name] = {"us": round(sec * 1e6, 1), "GBps": round(npx * bpp / sec / 1e9, 1),
                     "frac": round(npx * bpp / sec / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def cpu_baseline(args, fizi, w):
    """The oracle on a sample of the batched workload's frames (learning of
    the sampled streams' models is set-up, not timed)."""
    from oracle import oracle
    import numpy as np
    rng = np.random.default_rng(1)
    n = len(w["specs"])
    picks = rng.choice(n, size=args.cpu_streams, replace=False)
    total_px, total_s, frames = 0, 0.0, 0
    for i in picks:
        sp, sc = w["specs"][i], w["scenes"][i]
        m = oracle.Model(sp.width, sp.height)
        m.learn(sc.bg_frames(0, 30).cpu().numpy())
        hand = w["frames"][i].cpu().numpy()
        for k in range(min(args.cpu_frames, hand.shape[0])):
            t = time.perf_counter()
            m.process(hand[k], frame_index=k)
            total_s += time.perf_counter() - t
            total_px += sp.width * sp.height
            frames += 1
    return {"value": round(total_px / total_s / 1e6, 3), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"{frames} frames from {len(picks)} streams of the batched workload "
                      f"({total_px / 1e6:.1f} Mpx), single thread, {total_s:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--pool", type=int, default=4, help="resident hand frames per stream")
    ap.add_argument("--latency-steps", type=int, default=50)
    ap.add_argument("--plain-batch", type=int, default=256)
    ap.add_argument("--latency-frames", type=int, default=300)
    ap.add_argument("--cpu-streams", type=int, default=4)
    ap.add_argument("--cpu-frames", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time candidate launch shapes on the workload first and keep the fastest")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a 1 GiB -> 1 GiB elementwise kernel 3 times (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (the pipeline has no multi-GPU path); "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_04393_amd import fizi, scene, workloads

    if args.copy_probe:
        # a plain streaming kernel of known traffic (1 GiB read, 1 GiB
        # written per launch) to scale the HBM byte counters by
        a = torch.zeros(1 << 28, dtype=torch.int32, device="cuda:0")
        c = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=c)
        torch.cuda.synchronize()
        del a, c
    r = bench_batched(args, torch, fizi, workloads)
    mpxs = r["px"] / r["sec"] / 1e6
    fps = r["n"] / r["sec"]
    log(f"batched: {mpxs:.0f} Mpx/s, {fps:.0f} frames/s, {r['sec'] * 1e3:.3f} ms/step")
    plain = None if args.no_plain else bench_plain(args, torch, fizi, scene)
    if plain:
        plain["learn_background"] = bench_learn(args, torch, fizi, scene)
        log("plain:", plain)
    soft_res = None if args.no_plain else bench_soft(args, torch, scene)
    if soft_res:
        log("soft:", soft_res)
    serving = None
    if not args.no_serve:
        serving = {"budget_all_resident": bench_serving(args, torch, workloads)}
        log("serving:", serving["budget_all_resident"])
        serving["budget_4GB_sessions_come_and_go"] = bench_serving(
            args, torch, workloads, budget=4e9, session_len=2.0, duration=min(6.0, args.serve_seconds))
        log("serving tight:", serving["budget_4GB_sessions_come_and_go"])
    cpu = None if args.no_cpu else cpu_baseline(args, fizi, r["w"])
    if cpu:
        log("cpu:", cpu)
    out = {
        "metric": METRIC,
        "value": round(mpxs, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["sec"] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "batched: 64 streams, resolutions drawn by seed from 640x480, 1280x720, "
                               "1920x1080, 3840x2160, RGB uint8, one frame per stream per step",
                   "px_per_step": r["px"], "streams": r["n"], "launch": LAUNCH_NAMES[r["tuning"]["mode"]],
                   "tuning": r["tuning"]},
        "frames_per_s": round(fps, 1),
        "latency_ms": {"p50": pct(r["lat"], 50), "p99": pct(r["lat"], 99),
                       "mode": "one step of 64 frames submitted, pointers read back on the host"},
        "path_roofline_frac": round(mpxs * 1e6 * PATH_BYTES_PER_PX / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": {"bound": "hbm", "kernel": r["kernel"],
                     "achieved": round(r["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["achieved"] / HBM_PEAK_GBS, 4), "traffic": TRAFFIC.get(r["kernel"]),
                     "avg_launch_us": round(r["k_avg"] * 1e6, 2),
                     "bytes_per_launch": int(r["bpp"] * r["px"])},
        "stage_us": r["stages_us"],
        "tracking_ms_per_step": round(r["track_sec"] * 1e3, 4),
        "plain_single_stream": plain,
        "serving": serving,
        "soft_mask": soft_res,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
