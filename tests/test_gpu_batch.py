"""GPU parity of the batched form: every stream's I_FIZI and pointer equal
the CPU oracle's, in every launch mode (direct kernels, hipGraph replay,
persistent fused kernel, persistent kernel from a hipGraph, and the
software-pipelined steps, direct and from hipGraphs). Steps write into fresh
output buffers and are read after a flush, so that the pipelined modes (whose
outputs the next step writes) are checked the same way."""
import numpy as np
import pytest
import torch

from helpers import need_gpu

pytestmark = pytest.mark.gpu

MODES = (0, 1, 2, 3, 4, 5)


def _streams():
    """Five streams of different sizes and thresholds."""
    from paper_1907_04393_amd import scene
    specs = [scene.SceneSpec(320, 240, sigma=3, seed=(5, 1, 0, 0)),
             scene.SceneSpec(640, 480, sigma=4, seed=(5, 1, 0, 1), distractors=1),
             scene.SceneSpec(128, 96, sigma=2, seed=(5, 1, 0, 2)),
             scene.SceneSpec(192, 64, sigma=3, seed=(5, 1, 0, 3), gain="drift"),
             scene.SceneSpec(64, 33, sigma=3, seed=(5, 1, 0, 4))]
    params = [dict(), dict(), dict(open_iters=2, close_iters=0), dict(bg_delta=0, gray_S=5),
              dict(alpha1_cdeg=30000, alpha2_cdeg=9000)]
    data = []
    for sp in specs:
        sc = scene.Scene(sp)
        data.append((sc.bg_frames(0, 8), sc.hand_frames(0, 6)))
    return specs, params, data


# which streams have a frame in each of the 6 steps
ACTIVE = [[1, 1, 1, 1, 1], [1, 0, 1, 0, 1], [0, 1, 1, 1, 0], [1, 1, 0, 1, 1], [0, 0, 0, 0, 1],
          [1, 1, 1, 1, 1]]


def _oracle(specs, params, data):
    from oracle import oracle
    out = []
    for sp, pr, (bg, hand) in zip(specs, params, data):
        m = oracle.Model(sp.width, sp.height, oracle.params(**pr))
        m.learn(bg.numpy())
        out.append((m, hand))
    return out


@pytest.mark.parametrize("mode", MODES)
def test_batch_matches_oracle(mode):
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    specs, params, data = _streams()
    print("batch mode", mode, flush=True)
    b = fizi.Batch([(sp.width, sp.height) for sp in specs],
                   [fizi.default_params(**p) for p in params], device=dev)
    b.set_mode(mode)
    for i, (bg, _) in enumerate(data):
        b.learn(i, bg.to(dev))
    hands = [h.to(dev) for _, h in data]
    orc = _oracle(specs, params, data)
    counts = [0] * len(specs)
    outs = []
    for k, act in enumerate(ACTIVE):
        ptrs = torch.full((len(specs), 56), 0xAB, dtype=torch.uint8, device=dev)
        fz = [torch.empty((sp.height, sp.width // 64), dtype=torch.int64, device=dev) for sp in specs]
        frames = [hands[i][k] if act[i] else None for i in range(len(specs))]
        b.step(frames, ptrs, fizi=fz)
        outs.append((ptrs, fz))
    b.flush()
    torch.cuda.synchronize()
    for k, act in enumerate(ACTIVE):
        ptrs, fz = outs[k]
        got = fizi.pointers_to_numpy(ptrs)
        raw = ptrs.cpu().numpy()
        for i, sp in enumerate(specs):
            if not act[i]:
                assert (raw[i] == 0xAB).all(), (k, i)
                continue
            m, hand = orc[i]
            ref = m.process(hand[k].numpy(), frame_index=counts[i])
            counts[i] += 1
            assert fizi.pointer_dict(got[i]) == ref["pointer"], (mode, k, i)
            assert np.array_equal(fizi.unpack_bits(fz[i], sp.width), ref["fizi"]), (mode, k, i)
    assert b.status() == 0
    b.close()


def test_batch_learned_model_matches_oracle():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    specs, params, data = _streams()
    b = fizi.Batch([(sp.width, sp.height) for sp in specs],
                   [fizi.default_params(**p) for p in params], device=dev)
    for i, (bg, _) in enumerate(data):
        b.learn(i, bg[:3].to(dev))
        b.learn(i, bg[3:].to(dev), reset=False)
    torch.cuda.synchronize()
    for i, (m, _) in enumerate(_oracle(specs, params, data)):
        bgmin, bgmax, yref = b.model(i)
        assert np.array_equal(bgmin.cpu().numpy(), m.bgmin)
        assert np.array_equal(bgmax.cpu().numpy(), m.bgmax)
        assert np.array_equal(yref.cpu().numpy().view(np.uint16), m.yref)


def test_batch_unlearned_stream_is_an_error():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    b = fizi.Batch([(64, 8), (128, 8)], device=dev)
    b.learn(0, torch.full((1, 8, 64, 3), 50, dtype=torch.uint8, device=dev))
    ptrs = torch.zeros((2, 56), dtype=torch.uint8, device=dev)
    with pytest.raises(fizi.FiziError) as e:
        b.step([None, torch.zeros((8, 128, 3), dtype=torch.uint8, device=dev)], ptrs)
    assert e.value.code == fizi.FIZI_ESTATE
    b.step([None, None], ptrs)              # an empty step is a no-op
    b.step([torch.full((8, 64, 3), 50, dtype=torch.uint8, device=dev), None], ptrs)
    torch.cuda.synchronize()
    p = fizi.pointer_dict(fizi.pointers_to_numpy(ptrs)[0])
    assert p["present"] == 0 and p["frame_index"] == 0 and p["inv_gain_q16"] == 65536


def test_batched_workload_full_size():
    """The 64-stream workload at full size, in the benchmark's launch mode:
    every stream's outputs equal the direct-launch mode's, and a sample of
    streams equals the oracle."""
    from oracle import oracle
    from paper_1907_04393_amd import fizi, workloads
    dev = need_gpu()
    print("building 64-stream workload", flush=True)
    w = workloads.batched(64, pool=2, device=dev, log=lambda m: print(m, flush=True))
    b = w["batch"]
    n = len(w["specs"])
    res = {}
    for mode in (workloads.BATCH_MODE, fizi.BATCH_DIRECT):
        b.set_mode(mode)
        outs = []
        for k in range(2):
            ptrs = torch.empty((n, 56), dtype=torch.uint8, device=dev)
            fz = [torch.empty((sp.height, sp.width // 64), dtype=torch.int64, device=dev) for sp in w["specs"]]
            b.step(workloads.step_frames(w, k), ptrs, fizi=fz)
            b.flush()
            torch.cuda.synchronize()
            outs.append((fizi.pointers_to_numpy(ptrs).copy(), [f.cpu().numpy() for f in fz]))
        res[mode] = outs
        assert b.status() == 0
    for k in range(2):
        a, d = res[workloads.BATCH_MODE][k], res[fizi.BATCH_DIRECT][k]
        for i in range(n):
            ga, gd = fizi.pointer_dict(a[0][i]), fizi.pointer_dict(d[0][i])
            gd["frame_index"] = ga["frame_index"]
            assert ga == gd, (k, i)
            assert np.array_equal(a[1][i], d[1][i]), (k, i)
    rng = np.random.default_rng(0)
    sample = sorted(rng.choice(n, size=6, replace=False).tolist())
    print("oracle sample", sample, flush=True)
    for i in sample:
        sp, sc = w["specs"][i], w["scenes"][i]
        m = oracle.Model(sp.width, sp.height)
        m.learn(sc.bg_frames(0, 30).cpu().numpy())
        for k in range(2):
            ref = m.process(w["frames"][i][k].cpu().numpy(), frame_index=k)
            got = fizi.pointer_dict(res[workloads.BATCH_MODE][k][0][i])
            assert got == ref["pointer"], (i, k)
            bits = res[workloads.BATCH_MODE][k][1][i]
            assert np.array_equal(fizi.unpack_bits(torch.from_numpy(bits), sp.width), ref["fizi"]), (i, k)


def _run_steps(b, hands, specs, nsteps, dev):
    from paper_1907_04393_amd import fizi
    bufs, outs = [], []
    for k in range(nsteps):
        ptrs = torch.empty((len(specs), 56), dtype=torch.uint8, device=dev)
        fz = [torch.empty((sp.height, sp.width // 64), dtype=torch.int64, device=dev) for sp in specs]
        b.step([h[k] for h in hands], ptrs, fizi=fz)
        bufs.append((ptrs, fz))
    b.flush()
    torch.cuda.synchronize()
    for ptrs, fz in bufs:
        ps = [fizi.pointer_dict(p) for p in fizi.pointers_to_numpy(ptrs)]
        for p in ps:
            p.pop("frame_index")
        outs.append((ps, [f.cpu().numpy() for f in fz]))
    assert b.status() == 0
    return outs


def _same(a, b):
    for (pa, fa), (pb, fb) in zip(a, b):
        assert pa == pb
        assert all(np.array_equal(x, y) for x, y in zip(fa, fb))


def test_every_launch_shape_gives_the_same_result():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    specs, params, data = _streams()
    b = fizi.Batch([(sp.width, sp.height) for sp in specs],
                   [fizi.default_params(**p) for p in params], device=dev)
    for i, (bg, _) in enumerate(data):
        b.learn(i, bg.to(dev))
    hands = [h.to(dev) for _, h in data]
    b.set_tuning(mode=0, cls_iters=4, morph_rows=32, grid_per_cu=8)
    ref = _run_steps(b, hands, specs, 2, dev)
    # these streams are small enough for the short morphology bands, so
    # every tuned band height is taken with them off, and the short bands
    # once per four-kernel mode
    shapes = [dict(mode=m, cls_iters=c, morph_rows=r, grid_per_cu=g, short_bands=0)
              for m in MODES for c in (2, 8) for r in (8, 64) for g in ((1, 16) if m in (0, 4) else (8,))]
    shapes += [dict(mode=0, cls_iters=1, morph_rows=16, grid_per_cu=4, short_bands=0)]
    shapes += [dict(mode=m, cls_iters=4, morph_rows=16, grid_per_cu=8, short_bands=1) for m in (0, 1, 4, 5)]
    for sh in shapes:
        print("shape", sh, flush=True)
        b.set_tuning(**sh)
        assert b.get_tuning() == sh
        _same(_run_steps(b, hands, specs, 2, dev), ref)


def test_autotune_keeps_results():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    specs, params, data = _streams()
    b = fizi.Batch([(sp.width, sp.height) for sp in specs],
                   [fizi.default_params(**p) for p in params], device=dev)
    for i, (bg, _) in enumerate(data):
        b.learn(i, bg.to(dev))
    hands = [h.to(dev) for _, h in data]
    ref = _run_steps(b, hands, specs, 2, dev)
    ptrs = torch.empty((len(specs), 56), dtype=torch.uint8, device=dev)
    best, ms = b.autotune([h[0] for h in hands], ptrs, steps=3)
    print("autotuned", best, ms, flush=True)
    assert ms > 0 and best == b.get_tuning()
    _same(_run_steps(b, hands, specs, 2, dev), ref)
    with pytest.raises(fizi.FiziError):
        b.set_tuning(cls_iters=3)


def test_dense_masks_every_band_height():
    """Dense run masks (segment seams, rows of over 512 runs) at every band
    height and in the direct, persistent and pipelined launch modes, and in
    the short bands of one wave each."""
    from test_gpu_plain import dense_frames
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    cases = [(2048, 40, "mixed"), (640, 64, "noise"), (2048, 24, "checker")]
    prm = dict(open_iters=0, close_iters=0)
    data = [dense_frames(W, H, k) for W, H, k in cases]
    orc = []
    from oracle import oracle
    for (W, H, _), (bg, hand) in zip(cases, data):
        m = oracle.Model(W, H, oracle.params(**prm))
        m.learn(bg.numpy())
        orc.append([m.process(hand[k].numpy(), frame_index=k) for k in range(hand.shape[0])])
    b = fizi.Batch([(W, H) for W, H, _ in cases], [fizi.default_params(**prm)] * len(cases), device=dev)
    for i, (bg, _) in enumerate(data):
        b.learn(i, bg.to(dev))
    hands = [h.to(dev) for _, h in data]
    # every tuned band height (short bands off), then the short bands
    shapes = [(mode, rows, 0) for mode in (0, 2, 4) for rows in (8, 16, 32, 64)] + [(0, 16, 1), (4, 16, 1)]
    for mode, rows, short in shapes:
        print("dense batch mode", mode, "rows", rows, "short bands", short, flush=True)
        b.set_tuning(mode=mode, cls_iters=4, morph_rows=rows, grid_per_cu=8, short_bands=short)
        bufs = []
        for k in range(2):
            ptrs = torch.empty((len(cases), 56), dtype=torch.uint8, device=dev)
            fz = [torch.empty((H, W // 64), dtype=torch.int64, device=dev) for W, H, _ in cases]
            b.step([h[k] for h in hands], ptrs, fizi=fz)
            bufs.append((ptrs, fz))
        b.flush()
        torch.cuda.synchronize()
        for k, (ptrs, fz) in enumerate(bufs):
            got = fizi.pointers_to_numpy(ptrs)
            for i, (W, H, kind) in enumerate(cases):
                p = fizi.pointer_dict(got[i])
                ref = dict(orc[i][k]["pointer"])
                p.pop("frame_index"), ref.pop("frame_index")
                assert p == ref, (mode, rows, k, kind)
                assert np.array_equal(fizi.unpack_bits(fz[i], W), orc[i][k]["fizi"]), (mode, rows, k, kind)
        assert b.status() == 0
    b.close()


@pytest.mark.parametrize("mode,short", [(m, 0) for m in MODES] + [(0, 1), (4, 1)])
def test_batch_wide_and_narrow_streams(mode, short):
    """An 8192-pixel-wide stream beside narrow ones: the morphology launch
    takes two words per lane, and the narrow frames' packed bands run inside
    it with one (short bands off); with short bands on, every frame takes
    4-row bands of one wave each."""
    from oracle import oracle
    from test_gpu_plain import _blob_scene
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    shapes = [(8192, 24), (640, 48), (1920, 33), (1280, 17)]
    print("wide and narrow, mode", mode, "short bands", short, flush=True)
    b = fizi.Batch(shapes, device=dev)
    b.set_mode(mode)
    b.set_tuning(short_bands=short)
    data, orc = [], []
    for i, (W, H) in enumerate(shapes):
        bg, hand = _blob_scene(W, H, 3, 3, seed=31 * i + W)
        b.learn(i, bg.to(dev))
        m = oracle.Model(W, H)
        m.learn(bg.numpy())
        data.append(hand)
        orc.append(m)
    dev_frames = [h.to(dev) for h in data]
    bufs = []
    for k in range(3):
        ptrs = torch.empty((len(shapes), 56), dtype=torch.uint8, device=dev)
        fz = [torch.empty((H, W // 64), dtype=torch.int64, device=dev) for W, H in shapes]
        b.step([h[k] for h in dev_frames], ptrs, fizi=fz)
        bufs.append((ptrs, fz))
    b.flush()
    torch.cuda.synchronize()
    for k, (ptrs, fz) in enumerate(bufs):
        got = fizi.pointers_to_numpy(ptrs)
        for i, (W, H) in enumerate(shapes):
            ref = orc[i].process(data[i][k].numpy(), frame_index=k)
            assert fizi.pointer_dict(got[i]) == ref["pointer"], (mode, k, i)
            assert np.array_equal(fizi.unpack_bits(fz[i], W), ref["fizi"]), (mode, k, i)
    assert b.status() == 0
    b.close()


def test_default_cuda_device_accepts_indexed_frames():
    """A batch made on "cuda" takes frames allocated on "cuda:0"."""
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    b = fizi.Batch([(64, 8)], device="cuda")
    b.learn(0, torch.full((1, 8, 64, 3), 50, dtype=torch.uint8, device=dev))
    ptrs = torch.zeros((1, 56), dtype=torch.uint8, device=dev)
    b.step([torch.full((8, 64, 3), 50, dtype=torch.uint8, device=dev)], ptrs)
    torch.cuda.synchronize()
    assert fizi.pointer_dict(fizi.pointers_to_numpy(ptrs)[0])["present"] == 0
    b.close()


@pytest.mark.parametrize("mode", (4, 5))
def test_pipelined_outputs_at_every_completion_point(mode):
    """In the pipelined modes a step's outputs are complete once the next
    step has completed, and after every call that flushes or drains: an
    empty step leaves the pending one pending (flush completes it), learning
    flushes, status() and set_mode() drain."""
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    specs, params, data = _streams()
    n = len(specs)
    b = fizi.Batch([(sp.width, sp.height) for sp in specs],
                   [fizi.default_params(**p) for p in params], device=dev)
    b.set_mode(mode)
    for i, (bg, _) in enumerate(data):
        b.learn(i, bg.to(dev))
    hands = [h.to(dev) for _, h in data]
    orc = _oracle(specs, params, data)
    refs = [[m.process(hand[k].numpy(), frame_index=k)["pointer"] for k in range(5)] for m, hand in orc]

    def check(ptrs, k):
        got = fizi.pointers_to_numpy(ptrs)
        for i in range(n):
            assert fizi.pointer_dict(got[i]) == refs[i][k], (mode, k, i)

    def new():
        return torch.full((n, 56), 0xAB, dtype=torch.uint8, device=dev)

    p = [new() for _ in range(5)]
    b.step([h[0] for h in hands], p[0])
    b.step([h[1] for h in hands], p[1])
    torch.cuda.synchronize()
    check(p[0], 0)                              # completed by the next step
    idle = new()
    b.step([None] * n, idle)                    # nothing to do: step 1 stays pending
    b.flush()
    torch.cuda.synchronize()
    check(p[1], 1)
    assert (idle.cpu().numpy() == 0xAB).all()
    b.step([h[2] for h in hands], p[2])
    b.learn(0, data[0][0].to(dev))              # the same frames again: the model does not change
    torch.cuda.synchronize()
    check(p[2], 2)
    b.step([h[3] for h in hands], p[3])
    assert b.status() == 0                      # drains
    check(p[3], 3)
    b.step([h[4] for h in hands], p[4])
    b.set_mode(fizi.BATCH_GRAPH)                # drains
    check(p[4], 4)
    b.close()
