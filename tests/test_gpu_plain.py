"""GPU parity of the plain path (learn_background, process_frames,
get_pointer) against the CPU oracle: bit-exact model, I_FIZI, hand mask and
every pointer field."""
import numpy as np
import pytest
import torch

from helpers import compare, gpu_run, need_gpu, oracle_run

pytestmark = pytest.mark.gpu


def _small():
    from paper_1907_04393_amd import scene
    sc = scene.Scene(scene.small_plain())
    return sc.bg_frames(0, 30), sc.hand_frames(0, 100)


@pytest.mark.parametrize("short_bands", [True, False])
def test_small_scene_full_parity(short_bands):
    """320x240, 30 background + 100 hand frames, chunks of 16 (ragged last
    chunk); launches this small take 4-row morphology bands of one wave
    each unless short bands are off (8-row bands, two to a wave)."""
    bg, hand = _small()
    print("small scene: 320x240, 30 bg + 100 hand, short bands", short_bands, flush=True)
    g = gpu_run(bg, hand, {}, chunk=16, short_bands=short_bands)
    m, outs = oracle_run(bg, hand, {})
    compare(g, m, outs, "small")
    assert sum(o["pointer"]["present"] for o in outs.values()) >= 95


def test_incremental_learning_and_get_pointer():
    from paper_1907_04393_amd import fizi
    bg, hand = _small()
    g = gpu_run(bg, hand[:20], {}, chunk=8, learn_split=[7, 7, 16])
    m, outs = oracle_run(bg, hand[:20], {})
    compare(g, m, outs, "incremental")
    ctx = g["ctx"]
    for k in (0, 7, 19):
        assert ctx.get_pointer(k) == g["pointers"][k]
    with pytest.raises(fizi.FiziError) as e:
        ctx.get_pointer(20)
    assert e.value.code == fizi.FIZI_ERANGE
    # indices continue across calls
    dev = need_gpu()
    out = ctx.process_frames(hand[20:23].to(dev))
    torch.cuda.synchronize()
    ps = fizi.pointers_to_numpy(out["pointers"])
    assert [int(p["frame_index"]) for p in ps] == [20, 21, 22]
    assert ctx.get_pointer(21)["frame_index"] == 21


def test_process_before_learn_is_an_error():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    ctx = fizi.Context(64, 8, device=dev, chunk=2)
    with pytest.raises(fizi.FiziError) as e:
        ctx.process_frames(torch.zeros((1, 8, 64, 3), dtype=torch.uint8, device=dev))
    assert e.value.code == fizi.FIZI_ESTATE


def _blob_scene(W, H, n_bg, n_hand, seed):
    """Noisy random background and skin-hued blobs of random size."""
    g = torch.Generator().manual_seed(seed)
    base = torch.randint(30, 220, (1, H, W, 3), generator=g).float()
    bg = (base + torch.randn((n_bg, H, W, 3), generator=g) * 2).round().clamp(0, 255).to(torch.uint8)
    hand = (base + torch.randn((n_hand, H, W, 3), generator=g) * 2).round().clamp(0, 255)
    ys = torch.arange(H).view(H, 1)
    xs = torch.arange(W).view(1, W)
    for k in range(n_hand):
        for _ in range(int(torch.randint(0, 5, (1,), generator=g))):
            cx = int(torch.randint(0, W, (1,), generator=g))
            cy = int(torch.randint(0, H, (1,), generator=g))
            a = int(torch.randint(1, max(2, W // 3), (1,), generator=g))
            b = int(torch.randint(1, max(2, H // 2 + 1), (1,), generator=g))
            m = ((xs - cx) ** 2 * b * b + (ys - cy) ** 2 * a * a) <= a * a * b * b
            col = torch.tensor([200.0, 120.0 + 40 * torch.rand(1, generator=g).item(), 80.0])
            hand[k][m] = col
        gain = 0.85 + 0.3 * torch.rand(1, generator=g).item()
        hand[k] = (hand[k] * gain).round().clamp(0, 255)
    return bg, hand.to(torch.uint8)


@pytest.mark.parametrize("W,H", [(64, 1), (64, 2), (128, 37), (192, 100), (640, 33), (256, 257)])
def test_edge_geometries(W, H):
    print(f"edge geometry {W}x{H}", flush=True)
    bg, hand = _blob_scene(W, H, 5, 6, seed=W * 1000 + H)
    g = gpu_run(bg, hand, {}, chunk=4)
    m, outs = oracle_run(bg, hand, {})
    compare(g, m, outs, f"{W}x{H}")


PARAM_SETS = [
    dict(open_iters=0, close_iters=0),
    dict(open_iters=2, close_iters=1),
    dict(open_iters=3, close_iters=3),
    dict(open_iters=0, close_iters=2),
    dict(bg_delta=0, gray_S=0),
    dict(alpha1_cdeg=0, alpha2_cdeg=6000),          # narrow, no wrap
    dict(alpha1_cdeg=1000, alpha2_cdeg=1000),       # one hue
    dict(alpha1_cdeg=30000, alpha2_cdeg=12000),     # exactly a half turn
    dict(alpha1_cdeg=20000, alpha2_cdeg=15000),     # wide, wrapping
    dict(gain_row_stride=1, min_area=50, click_fill_permille=500),
    dict(gain_row_stride=64, gain_lo_q16=65536, gain_hi_q16=65536),
]


@pytest.mark.parametrize("k", range(len(PARAM_SETS)))
def test_parameter_readings(k):
    params = PARAM_SETS[k]
    print("params", params, flush=True)
    bg, hand = _blob_scene(192, 70, 6, 5, seed=77 + k)
    g = gpu_run(bg, hand, params, chunk=3)
    m, outs = oracle_run(bg, hand, params)
    compare(g, m, outs, str(params))


def test_degenerate_frames():
    """Frames identical to the background; an all-skin frame; a one-pixel
    checkerboard of skin (the most runs a row can have)."""
    W, H = 128, 48
    bgc = torch.full((2, H, W, 3), 40, dtype=torch.uint8)
    bgc[..., 2] = 90                                  # bluish, not skin
    skin = torch.tensor([210, 140, 90], dtype=torch.uint8)
    full = skin.view(1, 1, 1, 3).expand(1, H, W, 3).clone()
    chk = bgc[:1].clone()
    yy, xx = torch.meshgrid(torch.arange(H), torch.arange(W), indexing="ij")
    chk[0][((yy + xx) % 2) == 0] = skin
    stripes = bgc[:1].clone()
    stripes[0][:, ::2] = skin
    hand = torch.cat([bgc[:1], full, chk, stripes])
    for params in ({}, dict(open_iters=0, close_iters=0), dict(gain_lo_q16=65536, gain_hi_q16=65536)):
        print("degenerate", params, flush=True)
        g = gpu_run(bgc, hand, params, chunk=4)
        m, outs = oracle_run(bgc, hand, params)
        compare(g, m, outs, f"degenerate {params}")
    assert outs[0]["pointer"]["present"] == 0


def dense_pattern(W, H, kind, seed):
    """Foreground patterns with many runs per row: a one-pixel checkerboard
    (one 8-connected component), one-pixel stripes, 50% noise, and a mix of
    noise, checkerboard rows and full rows."""
    g = torch.Generator().manual_seed(seed)
    yy, xx = torch.meshgrid(torch.arange(H), torch.arange(W), indexing="ij")
    if kind == "checker":
        return (yy + xx) % 2 == 0
    if kind == "stripes":
        return (xx % 2 == 0).expand(H, W)
    if kind == "noise":
        return torch.rand((H, W), generator=g) < 0.5
    m = torch.rand((H, W), generator=g) < 0.3
    m |= ((yy % 7) < 2) & ((yy + xx) % 2 == 0)
    m |= (yy % 11) == 5
    return m


def dense_frames(W, H, kind, n=2):
    bg = torch.full((2, H, W, 3), 40, dtype=torch.uint8)
    bg[..., 2] = 90
    skin = torch.tensor([210, 140, 90], dtype=torch.uint8)
    hand = bg[:1].repeat(n, 1, 1, 1)
    for k in range(n):
        hand[k][dense_pattern(W, H, kind, k)] = skin
    return bg, hand


@pytest.mark.parametrize("W,H,kind", [(2048, 40, "checker"), (2048, 24, "stripes"), (640, 64, "noise"),
                                      (1088, 50, "mixed"), (128, 70, "checker")])
def test_dense_run_masks(W, H, kind):
    """More runs than a band's LDS segment table holds: segments close every
    few rows, rows of over 512 runs go to the run list directly, and
    components must join across every such seam."""
    bg, hand = dense_frames(W, H, kind)
    for params in ({}, dict(open_iters=0, close_iters=0)):
        print("dense", W, H, kind, params, flush=True)
        g = gpu_run(bg, hand, params, chunk=2)
        m, outs = oracle_run(bg, hand, params)
        compare(g, m, outs, f"dense {kind} {params}")


def test_hue_gray_all_2e24_colours():
    """Every RGB triple once (a 4096x4096 frame), gain pinned to 1, a
    background point-box that every colour leaves, no morphology: I_FIZI is
    then exactly I_R2 AND I_R3, compared with the oracle for all 2^24
    colours and several hue intervals."""
    from oracle import oracle
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    i = np.arange(1 << 24, dtype=np.uint32)
    frame = np.stack([(i >> 16) & 255, (i >> 8) & 255, i & 255], axis=1).astype(np.uint8)
    frame = frame.reshape(1, 4096, 4096, 3)
    bgf = ((frame.astype(np.int32) + 128) % 256).astype(np.uint8)
    fd = torch.from_numpy(frame).to(dev)
    bd = torch.from_numpy(bgf).to(dev)
    for (a1, a2, S) in [(33000, 7500, 20), (0, 6000, 0), (1000, 1000, 1), (30000, 12000, 5),
                        (20000, 15000, 20)]:
        print("2^24 sweep", a1, a2, S, flush=True)
        params = dict(alpha1_cdeg=a1, alpha2_cdeg=a2, gray_S=S, bg_delta=0, open_iters=0,
                      close_iters=0, gain_lo_q16=65536, gain_hi_q16=65536)
        ctx = fizi.Context(4096, 4096, fizi.default_params(**params), chunk=1, device=dev)
        ctx.learn_background(bd)
        out = ctx.process_frames(fd, want_fizi=True)
        torch.cuda.synchronize()
        got = fizi.unpack_bits(out["fizi"], 4096)[0].reshape(-1)
        ref = oracle.masks(frame[0], bgf[0], bgf[0], oracle.params(**params))
        assert ref["r1"].all()
        want = ref["raw"].reshape(-1)
        if not np.array_equal(got, want):
            bad = np.nonzero(got != want)[0][:5]
            raise AssertionError(f"({a1},{a2},{S}) differs at colours {[hex(int(b)) for b in bad]}")
        ctx.close()
        del out


@pytest.mark.parametrize("chunk", [16, 1])
def test_hd_scene_parity(chunk):
    """1920x1080, sigma 5, two distractors, 50 background frames, 32 hand
    frames in chunks of 16 (8-row morphology bands, two to a wave) or one
    by one (4-row bands of one wave each, the latency shape)."""
    from paper_1907_04393_amd import scene
    sc = scene.Scene(scene.hd_plain())
    bg = sc.bg_frames(0, 50)
    hand = sc.hand_frames(0, 32)
    print("hd scene 1920x1080, chunk", chunk, flush=True)
    g = gpu_run(bg, hand, {}, chunk=chunk)
    m, outs = oracle_run(bg, hand, {})
    compare(g, m, outs, "hd")
    assert all(o["pointer"]["present"] for o in outs.values())


def test_determinism():
    bg, hand = _small()
    a = gpu_run(bg, hand[:16], {}, chunk=16)
    b = gpu_run(bg, hand[:16], {}, chunk=5)
    assert a["pointers"] == b["pointers"]
    assert np.array_equal(a["fizi"], b["fizi"]) and np.array_equal(a["hand"], b["hand"])


def _offset_copy(t, offset, dev):
    """t copied to device memory that starts `offset` bytes past an aligned
    allocation."""
    flat = t.reshape(-1)
    buf = torch.zeros(flat.numel() + 64, dtype=torch.uint8, device=dev)
    buf[offset:offset + flat.numel()] = flat.to(dev)
    return buf[offset:offset + flat.numel()].view(t.shape)


def test_word_aligned_frames_match_oracle():
    """Frames 4-byte but not 16-byte aligned take the per-word gain path;
    results are the same."""
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, hand = _blob_scene(192, 70, 6, 5, seed=1234)
    ctx = fizi.Context(192, 70, chunk=3, device=dev)
    ctx.learn_background(_offset_copy(bg, 4, dev))
    out = ctx.process_frames(_offset_copy(hand, 4, dev), want_fizi=True)
    torch.cuda.synchronize()
    m, outs = oracle_run(bg, hand, {})
    got = [fizi.pointer_dict(r) for r in fizi.pointers_to_numpy(out["pointers"])]
    bits = fizi.unpack_bits(out["fizi"], 192)
    for k, o in outs.items():
        assert got[k] == o["pointer"], k
        assert np.array_equal(bits[k], o["fizi"]), k


def test_unaligned_frames_are_rejected():
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    bg, hand = _blob_scene(64, 8, 2, 1, seed=5)
    ctx = fizi.Context(64, 8, chunk=1, device=dev)
    with pytest.raises(fizi.FiziError) as e:
        ctx.learn_background(_offset_copy(bg, 1, dev))
    assert e.value.code == fizi.FIZI_EINVAL
    ctx.learn_background(bg.to(dev))
    with pytest.raises(fizi.FiziError) as e:
        ctx.process_frames(_offset_copy(hand, 2, dev))
    assert e.value.code == fizi.FIZI_EINVAL


def _mask_frames(masks):
    """Frames that classify to exactly the given masks: a flat blue
    background and skin-coloured foreground."""
    n, H, W = masks.shape
    bg = np.zeros((2, H, W, 3), np.uint8)
    bg[...] = (40, 40, 90)
    fr = np.repeat(bg[:1], n, axis=0).copy()
    fr[masks.astype(bool)] = (210, 140, 90)
    return torch.from_numpy(bg), torch.from_numpy(fr)


@pytest.mark.parametrize("kind", ["comb", "bars", "serpentine"])
def test_tall_components_many_border_joins(kind):
    """Components that cross every band border many times: thousands of
    cross-band joins (more than the resolve stage's list of linked roots
    holds), long root chains, one or hundreds of components."""
    W, H = 2048, 1024
    m = np.zeros((H, W), np.uint8)
    if kind == "comb":
        m[:, 0:W:4] = 1
        m[:, 1:W:4] = 1
        m[H - 3:, :] = 1                      # the bars joined at the bottom
    elif kind == "bars":
        m[:, 0:W:4] = 1
    else:
        for k, x in enumerate(range(0, W, 8)):
            m[:, x:x + 2] = 1
            y = H - 2 if k % 2 == 0 else 0    # joined alternately at the bottom and top
            m[y:y + 2, x:x + 10] = 1
    masks = np.stack([m, m[::-1].copy()])
    bg, fr = _mask_frames(masks)
    params = dict(open_iters=0, close_iters=0)
    print("tall components", kind, flush=True)
    g = gpu_run(bg, fr, params, chunk=2)
    mo, outs = oracle_run(bg, fr, params)
    compare(g, mo, outs, kind)
    expect = {"comb": 1, "bars": W // 4, "serpentine": 1}[kind]
    assert all(o["pointer"]["n_components"] == expect for o in outs.values())


@pytest.mark.parametrize("W", [64, 960, 1024, 1088, 2048, 2112])
@pytest.mark.parametrize("H", [1, 9, 40])
def test_lane_group_boundaries(W, H):
    """Morphology packs 4 bands per wave up to 16 words per row and 2 up to
    32: widths on both sides of each limit, heights whose last item leaves
    lane groups idle (1 and 9 rows: one or two bands of eight)."""
    print(f"lane groups {W}x{H}", flush=True)
    bg, hand = _blob_scene(W, H, 3, 3, seed=W + 7 * H)
    g = gpu_run(bg, hand, {}, chunk=3)
    m, outs = oracle_run(bg, hand, {})
    compare(g, m, outs, f"{W}x{H}")


@pytest.mark.parametrize("W", [4160, 8192])
@pytest.mark.parametrize("params", [{}, dict(open_iters=2, close_iters=0)])
def test_widest_frames(W, params):
    """Rows of more than 64 words (two words per lane in the morphology),
    up to the 8192-pixel limit."""
    print(f"widest {W}", params, flush=True)
    bg, hand = _blob_scene(W, 40, 3, 3, seed=W)
    g = gpu_run(bg, hand, params, chunk=2)
    m, outs = oracle_run(bg, hand, params)
    compare(g, m, outs, f"{W} {params}")


@pytest.mark.parametrize("W,H", [(64, 8192), (192, 8191)])
def test_tallest_frames(W, H):
    """The 8192-row limit on narrow frames (a thousand bands, four per wave),
    with a ragged last band."""
    print(f"tallest {W}x{H}", flush=True)
    bg, hand = _blob_scene(W, H, 3, 2, seed=H + W)
    g = gpu_run(bg, hand, {}, chunk=2)
    m, outs = oracle_run(bg, hand, {})
    compare(g, m, outs, f"{W}x{H}")
