"""The allocation-free entry point fizi_soft_bce_static (partial sums in the
library's static device array) against the entry point it varies,
fizi_soft_bce (caller workspace), called through the C ABI: two calls in a
row, the second on a smaller input with a ragged tail, each equal bit for
bit to fizi_soft_bce on the same input (same kernels, same grid, same
reduction order), and within the calibration form's stated tolerance of the
FP64 oracle (relative 1e-4 per gradient component, the loss to 1e-6)."""
import ctypes

import numpy as np
import pytest
import torch

from helpers import need_gpu

pytestmark = pytest.mark.gpu

P6 = (102.0, 153.0, 208.3, 10.0, 133.3, 2.5)


def _inputs(n_frames, rows, tail):
    """Seeded calibration frames (1280 wide, `rows` rows each) and their
    ground-truth masks, flattened to pixels, with `tail` extra pixels."""
    from paper_1907_04393_amd import scene
    sc = scene.Scene(scene.calibration())
    f, gt = sc.hand_frames(0, n_frames, with_gt=True)
    f = f[:, :rows].reshape(-1, 3)
    gt = gt[:, :rows].reshape(-1).to(torch.uint8)
    rng = np.random.default_rng(rows + tail)
    ft = torch.from_numpy(rng.integers(0, 256, size=(tail, 3), dtype=np.uint8))
    gtt = torch.from_numpy(rng.integers(0, 2, size=tail, dtype=np.uint8))
    return torch.cat([f, ft]).contiguous(), torch.cat([gt, gtt]).contiguous()


def _call_both(L, fizi, frames, gt, T, dev):
    npx = frames.shape[0]
    p6 = (ctypes.c_float * 6)(*P6)
    ws_bytes = int(L.fizi_soft_workspace_bytes(npx))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ref = torch.full((7,), float("nan"), dtype=torch.float64, device=dev)
    got = torch.full((7,), float("nan"), dtype=torch.float64, device=dev)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    fizi.check(L.fizi_soft_bce(ctypes.c_void_p(frames.data_ptr()), ctypes.c_void_p(gt.data_ptr()), npx, p6,
                               ctypes.c_float(T), ctypes.c_void_p(ws.data_ptr()), ws_bytes,
                               ctypes.c_void_p(ref.data_ptr()), s))
    fizi.check(L.fizi_soft_bce_static(ctypes.c_void_p(frames.data_ptr()), ctypes.c_void_p(gt.data_ptr()), npx, p6,
                                      ctypes.c_float(T), ctypes.c_void_p(got.data_ptr()), s))
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("T", [0.5, 2.0])
def test_static_scratch_entry_matches_workspace_entry(T):
    from oracle import soft as osoft
    from paper_1907_04393_amd import fizi
    dev = need_gpu()
    L = fizi.lib()
    cases = [(8, 720, 0), (1, 37, 3)]          # 7.4 Mpx, then 47,363 px (a 3-pixel tail)
    for n_frames, rows, tail in cases:
        frames, gt = _inputs(n_frames, rows, tail)
        print("fizi_soft_bce_static", frames.shape[0], "px, T", T, flush=True)
        got, ref = _call_both(L, fizi, frames.to(dev), gt.to(dev), T, dev)
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref), (got, ref)
        g64 = osoft.grad_bce(frames.numpy(), gt.numpy(), P6, T)
        loss64 = osoft.bce_loss(frames.numpy(), gt.numpy(), P6, T)
        tol = 1e-4 * np.maximum(np.abs(g64), 1e-3 * np.abs(g64).max())
        assert np.all(np.abs(got[:6] - g64) <= tol), (got[:6], g64)
        assert abs(got[6] - loss64) <= 1e-6 * max(1.0, abs(loss64)), (got[6], loss64)
