#!/usr/bin/env python3
"""Benchmark of the FIZI/Mouse pipeline on one MI355X.

Headline workload (batched form): 64 camera streams whose resolutions are
drawn by seed from {640x480, 1280x720, 1920x1080, 3840x2160}, each with its
own learned background, hand path and brightness drift. A step is one frame
for every stream through the whole per-frame path (gain, classify,
morphology, components, pointer). The launch shape (launch mode, classify
tile, grid, band height) is the one the batch's autotuner picks on these
frames during set-up. In the software-pipelined modes a step's morphology
and components run beside the next step's classify; the timed region ends
with a flush, so it holds exactly the timed steps' work. Inputs are resident
in HBM before the timed region.

Also measured, next to it: the plain single-stream form on 1920x1080 frames
(throughput of process_frames over resident frames, and the latency of
single-frame calls with the pointer read back on the host), background
learning, the soft mask, serving, and the CPU oracle on this host.

Printed: one JSON line. `roofline` is the dominant kernel's (classify's, or
the fused kernel's in a persistent launch shape) algorithmic bytes per launch
over its average duration, taken from the kernel's own dispatch events in
the headline launch form; `traffic` is the HBM bytes rocprofv3 counted for
that kernel's code (null when the built kernel differs from the one the
counters were taken on); `cpu_baseline` is the CPU oracle on this host.
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
# of the classify kernel: frame 3 + background min/max 6 (its raw-mask
# output is an intermediate, counted as overhead)
CLASSIFY_BYTES_PER_PX = 9.0

LAUNCH_NAMES = {0: "four kernels, direct launches", 1: "four kernels replayed from a hipGraph",
                2: "persistent fused kernel", 3: "persistent fused kernel, hipGraph",
                4: "four kernels, pipelined across steps (back half on a side stream)",
                5: "four kernels, pipelined across steps, hipGraphs"}
# launch form whose kernels carry dispatch events: the same kernels in the
# same order and streams as the mode timed (graph replays cannot carry them)
TIMED_FORM = {0: 0, 1: 0, 2: 2, 3: 2, 4: 4, 5: 4}

# HBM bytes per launch of the dominant kernel on this workload, from
# rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (the factors a 1 GiB -> 1 GiB
# elementwise kernel gives), with the code hash of the kernel they were
# taken on (the build writes lib/kernel_hashes.json)
TRAFFIC = {"_ZN4fizi12_GLOBAL__N_110k_classifyILi8EEEvPNS_5TableE": ("85c419a3c64feb26", 1714.7e6),
           "_ZN4fizi12_GLOBAL__N_110k_classifyILi4EEEvPNS_5TableE": ("51db8709717845f7", 1714.4e6)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(a, q):
    import numpy as np
    return round(float(np.percentile(np.asarray(a), q)), 4)


def kernel_hash(symbol):
    try:
        with open(os.path.join(ROOT, "paper_1907_04393_amd", "lib", "kernel_hashes.json")) as f:
            return json.load(f).get(symbol)
    except OSError:
        return None


def measured_traffic(symbol):
    want = TRAFFIC.get(symbol)
    if want is None or kernel_hash(symbol) != want[0]:
        return None
    return want[1]


def copy_peak(torch):
    """A plain device copy, 1 GiB read and 1 GiB written per launch, timed
    with events: the bandwidth this machine's HBM gives a simple stream."""
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
    c = torch.empty_like(a)
    a.fill_(1)
    for _ in range(2):
        c.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, c
    return round(2 * (1 << 30) / sec / 1e9, 1)


def bench_batched(args, torch, fizi, workloads):
    dev = torch.device("cuda:0")
    log("building the 64-stream workload")
    w = workloads.batched(64, pool=args.pool, device=dev, log=log)
    b, n, px = w["batch"], len(w["specs"]), w["px_per_step"]
    ptrs = torch.empty((n, 56), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    b.set_mode(workloads.BATCH_MODE)
    autotuned = None
    if args.shape:
        c, r, g, m = (int(v) for v in args.shape.split(","))
        b.set_tuning(cls_iters=c, morph_rows=r, grid_per_cu=g, mode=m)
    elif not args.no_autotune:
        best, ms = b.autotune(workloads.step_frames(w, 0), ptrs, steps=30, stream=stream)
        autotuned = {"picked": best, "ms_per_step": round(ms, 4)}
        log(f"autotuned launch shape {best}: {ms:.3f} ms/step")
    tuning = b.get_tuning()

    def run(steps):
        for k in range(steps):
            b.step(workloads.step_frames(w, k), ptrs, stream=stream)
        b.flush(stream=stream)

    run(args.warmup)
    torch.cuda.synchronize()
    assert b.status() == 0
    log("warmup done; timed region")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert b.status() == 0
    sec = (t1 - t0) / args.steps

    # per-step latency: submit a step, make its outputs complete (flush),
    # wait for its pointers on the host
    host = torch.empty((n, 56), dtype=torch.uint8, pin_memory=True)
    lat = []
    for k in range(args.latency_steps):
        t = time.perf_counter()
        b.step(workloads.step_frames(w, k), ptrs, stream=stream)
        b.flush(stream=stream)
        host.copy_(ptrs, non_blocking=True)
        stream.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)

    # the same steps with every stream tracked (temporal tracking, one frame
    # per stream per step: the component stage stays parallel)
    for i in range(n):
        b.set_tracking(i, True)
    run(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    track_sec = (time.perf_counter() - t0) / args.steps
    for i in range(n):
        b.set_tracking(i, False)

    # kernel durations from their own dispatch events, in the launch form of
    # the timed mode (the persistent kernel reports its whole launch under
    # "classify")
    form = TIMED_FORM[tuning["mode"]]
    b.set_mode(form)
    b.stage_timing(True)
    run(args.steps)
    torch.cuda.synchronize()
    st = b.stage_times()
    b.stage_timing(False)
    b.set_mode(tuning["mode"])
    assert b.status() == 0
    stages_us = {k: round(v[0] * 1e3 / v[1], 2) for k, v in st.items() if v[1]}
    k_ms, k_n = st["classify"]
    k_avg = k_ms / 1e3 / max(1, k_n)
    if form == fizi.BATCH_PERSISTENT:
        kernel, bpp, sym = "k_flow (fused gain, classify, morphology, components)", PATH_BYTES_PER_PX, None
    else:
        kernel = f"k_classify<{tuning['cls_iters']}> (I_R1, I_R2, I_R3 per pixel)"
        bpp, sym = CLASSIFY_BYTES_PER_PX, f"_ZN4fizi12_GLOBAL__N_110k_classifyILi{tuning['cls_iters']}EEEvPNS_5TableE"
    achieved = bpp * px / k_avg / 1e9
    return dict(w=w, px=px, n=n, sec=sec, lat=lat, k_avg=k_avg, achieved=achieved, kernel=kernel, bpp=bpp,
                tuning=tuning, stages_us=stages_us, track_sec=track_sec, autotuned=autotuned,
                timed_form=LAUNCH_NAMES[form], traffic=measured_traffic(sym) if sym else None,
                code_hash=kernel_hash(sym) if sym else None)


def bench_plain(args, torch, fizi, scene):
    dev = torch.device("cuda:0")
    spec = scene.hd_plain()
    W, H = spec.width, spec.height
    sc = scene.Scene(spec, device=dev)
    bg = sc.bg_frames(0, spec.n_bg)
    pool = sc.hand_frames(0, args.plain_batch)
    ctx = fizi.Context(W, H, chunk=scene.HD_CHUNK, device=dev)
    ctx.learn_background(bg)
    # back-to-back calls: each call's last batch completes beside the next
    # call's first one; the flush inside the timed region completes the last
    ctx.set_pipelined(True)
    stream = torch.cuda.current_stream()
    ptrs = torch.empty((args.plain_batch, 56), dtype=torch.uint8, device=dev)
    for _ in range(6):
        ctx.process_into(pool, args.plain_batch, pointers=ptrs, stream=stream)
    ctx.flush(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        ctx.process_into(pool, args.plain_batch, pointers=ptrs, stream=stream)
    ctx.flush(stream)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    fps = args.plain_batch / sec
    # temporal tracking: the component stage of a call's frames runs in order
    ctx.set_tracking(True)
    ctx.process_into(pool, args.plain_batch, pointers=ptrs, stream=stream)
    ctx.flush(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.process_into(pool, args.plain_batch, pointers=ptrs, stream=stream)
    ctx.flush(stream)
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
    return {"workload": "one 1920x1080 stream, frames processed in calls of "
                        f"{args.plain_batch} (internal launches of {scene.HD_CHUNK} frames; calls pipelined, "
                        "flushed at the end of the timed region)",
            "Mpixel_per_s": round(fps * W * H / 1e6, 1), "frames_per_s": round(fps, 1),
            "path_roofline_frac": round(fps * W * H * PATH_BYTES_PER_PX / (HBM_PEAK_GBS * 1e9), 4),
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
    # wall time per call with the stage clock off (its events cost more
    # than a call), then the kernel's own time from its dispatch events
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.learn_background(bg)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    ctx.stage_timing(True)
    for _ in range(reps):
        ctx.learn_background(bg)
    torch.cuda.synchronize()
    ms, launches = ctx.stage_times()["learn"]
    k_s = ms / 1e3 / max(1, launches)
    byts = W * H * (3 * n + 12)
    out = {"workload": f"{n} frames 1920x1080 per call", "ms_per_call": round(sec * 1e3, 3),
           "frames_per_s": round(n / sec, 1), "minmax_kernel_us": round(k_s * 1e6, 1),
           "minmax_GBps": round(byts / k_s / 1e9, 1), "minmax_frac": round(byts / k_s / 1e9 / HBM_PEAK_GBS, 4)}
    # partial re-learning: running frames fed back with their I_FIZI masks
    # (model 12 B/px once per call, each frame 3 B/px + its mask 1/8 B/px)
    hand = scene.Scene(spec, device=dev).hand_frames(0, 8)
    ctx.stage_timing(False)
    bits = ctx.process_frames(hand, want_fizi=True)["fizi"]
    torch.cuda.synchronize()
    for k in (1, 8):
        ctx.relearn_background(hand[:k], bits[:k])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.relearn_background(hand[:k], bits[:k])
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        ctx.stage_timing(True)
        for _ in range(reps):
            ctx.relearn_background(hand[:k], bits[:k])
        torch.cuda.synchronize()
        ms, launches = ctx.stage_times()["learn"]
        ctx.stage_timing(False)
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
    loss and gradient (3 + 1 B in). Kernel times come from their own
    dispatch events; `call_us` is the Python call as the autograd path makes
    it (allocations and two launches included)."""
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
    for name, fn, bpp, stage in (("forward", lambda: soft.soft_forward(f, prm, 0.5, out=m), 7, "forward"),
                                 ("backward", lambda: soft.soft_backward(f, dm, prm, 0.5), 7, "backward"),
                                 ("fused_bce", lambda: soft.soft_bce(f, gt, prm, 0.5), 4, "backward")):
        fn()
        torch.cuda.synchronize()
        # the call's wall time with the dispatch events off, then the
        # kernels' own times from their events
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        soft.times()
        soft.timing(True)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        tm = soft.times()
        soft.timing(False)
        k_s = tm[stage][0] / 1e3 / max(1, tm[stage][1])
        rec = {"kernel_us": round(k_s * 1e6, 2), "GBps": round(npx * bpp / k_s / 1e9, 1),
               "frac": round(npx * bpp / k_s / 1e9 / HBM_PEAK_GBS, 4), "call_us": round(sec * 1e6, 1)}
        if tm["final"][1]:
            rec["final_reduce_us"] = round(tm["final"][0] * 1e3 / tm["final"][1], 2)
        out[name] = rec
    return out


def host_threads():
    """Threads the CPU baseline may use: this process's CPU affinity, capped
    by OMP_NUM_THREADS when that is set (the share of the host this job has)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, scene, w):
    """The CPU oracle timed on this host beside the GPU: (1) on all host
    threads, the batched workload (every stream, args.cpu_steps frame steps,
    one stream per thread at a time); (2) one thread, the 320x240 workload in
    full (30 learning + 100 hand frames); (3) one thread, the first
    args.cpu_hd_frames hand frames of the 1920x1080 stream. Learning of the
    batched streams' models is set-up, not timed."""
    from oracle import oracle
    import concurrent.futures as cf
    import numpy as np
    nthr = host_threads()
    specs, n = w["specs"], len(w["specs"])
    frames = [f.cpu().numpy() for f in w["frames"]]

    def learned(i):
        sp = specs[i]
        m = oracle.Model(sp.width, sp.height)
        m.learn(w["scenes"][i].bg_frames(0, 30).cpu().numpy())
        return m

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(nthr) as pool:
        models = list(pool.map(learned, range(n)))
    log(f"cpu: {n} oracle models learned in {time.perf_counter() - t0:.1f} s on {nthr} threads")

    def run(i):
        for k in range(args.cpu_steps):
            models[i].process(frames[i][k % w["pool"]], frame_index=k)

    # largest streams first, so that the pool's tail is short
    order = sorted(range(n), key=lambda i: -specs[i].width * specs[i].height)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(nthr) as pool:
        list(pool.map(run, order))
    all_s = time.perf_counter() - t0
    all_px = args.cpu_steps * w["px_per_step"]
    del models

    # one thread: the 320x240 workload in full, learning included
    sp0 = scene.small_plain()
    sc0 = scene.Scene(sp0)
    bg0, hand0 = sc0.bg_frames(0, sp0.n_bg).numpy(), sc0.hand_frames(0, sp0.n_hand).numpy()
    t0 = time.perf_counter()
    m0 = oracle.Model(sp0.width, sp0.height)
    m0.learn(bg0)
    for k in range(sp0.n_hand):
        m0.process(hand0[k], frame_index=k)
    small_s = time.perf_counter() - t0
    small_px = sp0.width * sp0.height * (sp0.n_bg + sp0.n_hand)

    # the 1920x1080 stream: one thread on its first frames, then all host
    # threads on more of them (one frame per thread at a time; a frame's
    # result does not depend on the others without tracking)
    sp1 = scene.hd_plain()
    sc1 = scene.Scene(sp1, device="cuda:0")
    m1 = oracle.Model(sp1.width, sp1.height)
    m1.learn(sc1.bg_frames(0, sp1.n_bg).cpu().numpy())
    hand1 = sc1.hand_frames(0, max(args.cpu_hd_frames, args.cpu_hd_all_frames)).cpu().numpy()
    t0 = time.perf_counter()
    for k in range(args.cpu_hd_frames):
        m1.process(hand1[k], frame_index=k)
    hd_s = time.perf_counter() - t0
    hd_px = sp1.width * sp1.height * args.cpu_hd_frames
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(nthr) as pool:
        list(pool.map(lambda k: m1.process(hand1[k], frame_index=k), range(args.cpu_hd_all_frames)))
    hd_all_s = time.perf_counter() - t0

    # the soft mask's FP64 gradient (fused BCE) on 8 of the 32 calibration
    # frames, scaled to the 32
    from oracle import soft as osoft
    f3, gt3 = scene.Scene(scene.calibration()).hand_frames(0, 8, with_gt=True)
    f3, gt3 = f3.numpy(), gt3.numpy().astype(np.uint8)
    t0 = time.perf_counter()
    osoft.grad_bce(f3, gt3, osoft.CHECK_POINT, 0.5)
    osoft.bce_loss(f3, gt3, osoft.CHECK_POINT, 0.5)
    soft_s = time.perf_counter() - t0
    return {"value": round(all_px / all_s / 1e6, 2), "unit": "Mpixel/s", "cores": nthr, "kind": "oracle",
            "sample": f"batched workload: all {n} streams x {args.cpu_steps} frame steps "
                      f"({all_px / 1e6:.0f} Mpx) on {nthr} host threads, one stream per thread at a time, "
                      f"{all_s:.1f} s",
            "cpu_model": cpu_model(),
            "frames_per_s": round(n * args.cpu_steps / all_s, 2),
            "single_thread": {
                "320x240_full": {"frames": sp0.n_bg + sp0.n_hand, "seconds": round(small_s, 3),
                                 "Mpixel_per_s": round(small_px / small_s / 1e6, 2),
                                 "frames_per_s": round((sp0.n_bg + sp0.n_hand) / small_s, 1),
                                 "note": "30 learning + 100 hand frames, learning included"},
                "1920x1080": {"frames": args.cpu_hd_frames, "seconds": round(hd_s, 3),
                              "Mpixel_per_s": round(hd_px / hd_s / 1e6, 2),
                              "frames_per_s": round(args.cpu_hd_frames / hd_s, 2),
                              "note": f"the first {args.cpu_hd_frames} of the stream's 2000 hand frames"},
                "soft_fp64_gradient_32x1280x720_s": round(soft_s * 4, 3)},
            "all_threads_1920x1080": {"frames": args.cpu_hd_all_frames, "threads": nthr,
                                      "seconds": round(hd_all_s, 3),
                                      "frames_per_s": round(args.cpu_hd_all_frames / hd_all_s, 2),
                                      "Mpixel_per_s": round(sp1.width * sp1.height * args.cpu_hd_all_frames
                                                            / hd_all_s / 1e6, 2)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--pool", type=int, default=4, help="resident hand frames per stream")
    ap.add_argument("--latency-steps", type=int, default=50)
    ap.add_argument("--plain-batch", type=int, default=256)
    ap.add_argument("--latency-frames", type=int, default=300)
    ap.add_argument("--cpu-steps", type=int, default=10, help="frame steps of the batched workload on the CPU")
    ap.add_argument("--cpu-hd-frames", type=int, default=60, help="1920x1080 frames on one CPU thread")
    ap.add_argument("--cpu-hd-all-frames", type=int, default=256,
                    help="1920x1080 frames on all host threads, one frame per thread")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape instead of the autotuner's pick")
    ap.add_argument("--shape", default="",
                    help="fixed launch shape cls_iters,morph_rows,grid_per_cu,mode instead of the autotuner's "
                         "pick (to profile one shape)")
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
    copy_gbs = copy_peak(torch)
    log(f"device copy: {copy_gbs} GB/s")
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
    cpu = None if args.no_cpu else cpu_baseline(args, scene, r["w"])
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
                   "tuning": r["tuning"], "autotuned": r["autotuned"]},
        "frames_per_s": round(fps, 1),
        "latency_ms": {"p50": pct(r["lat"], 50), "p99": pct(r["lat"], 99),
                       "mode": "one step of 64 frames submitted and flushed, pointers read back on the host"},
        "path_roofline_frac": round(mpxs * 1e6 * PATH_BYTES_PER_PX / (HBM_PEAK_GBS * 1e9), 4),
        "path_frac_of_copy": round(mpxs * 1e6 * PATH_BYTES_PER_PX / (copy_gbs * 1e9), 4),
        "roofline": {"bound": "hbm", "kernel": r["kernel"],
                     "achieved": round(r["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["achieved"] / HBM_PEAK_GBS, 4), "traffic": r["traffic"],
                     "avg_launch_us": round(r["k_avg"] * 1e6, 2),
                     "bytes_per_px": r["bpp"], "bytes_per_launch": int(r["bpp"] * r["px"]),
                     "timed_in": r["timed_form"], "code_hash": r["code_hash"],
                     "measured_copy_GBps": copy_gbs,
                     "frac_of_copy": round(r["achieved"] / copy_gbs, 4)},
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
