"""GPU soft mask and hand-written adjoint against the FP64 oracle.

Tolerances: the mask is FP32 arithmetic on values of order 100 (chroma) and
10 (distance), so its absolute error is a few 1e-6 (bound used: 2e-5); the
gradients are compared as |g - g64| <= 1e-4 * max(|g64_i|, 1e-3 * max|g64|),
the stated relative tolerance of the calibration form."""
import numpy as np
import pytest
import torch

from helpers import need_gpu

pytestmark = pytest.mark.gpu


def _close(g, ref, rel=1e-4):
    g, ref = np.asarray(g, np.float64), np.asarray(ref, np.float64)
    tol = rel * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return np.all(np.abs(g - ref) <= tol), np.abs(g - ref) / np.maximum(np.abs(ref), 1e-300)


def _calib(n=32):
    from paper_1907_04393_amd import scene
    sc = scene.Scene(scene.calibration())
    f, gt = sc.hand_frames(0, n, with_gt=True)
    return f, gt.to(torch.uint8)


POINTS = [(102.0, 153.0, 208.3, 10.0, 133.3, 2.5), (108.0, 150.0, 260.0, -30.0, 170.0, 1.8)]


@pytest.mark.parametrize("T", [0.5, 2.0])
@pytest.mark.parametrize("p", POINTS)
def test_forward_and_adjoint_small(p, T):
    from oracle import soft as osoft
    from paper_1907_04393_amd import soft
    dev = need_gpu()
    f, gt = _calib(2)
    f = f[:, :200].contiguous()             # 2 x 200 x 1280 px, plus a 3-pixel tail
    flat = torch.cat([f.reshape(-1, 3), torch.tensor([[200, 120, 90], [90, 90, 90], [10, 200, 30]],
                                                     dtype=torch.uint8)]).contiguous()
    prm = torch.tensor(p, dtype=torch.float64)
    m = soft.soft_forward(flat.to(dev), prm, T)
    ref = osoft.mask(flat.numpy(), p, T)
    assert np.abs(m.cpu().numpy().astype(np.float64) - ref).max() < 2e-5
    rng = np.random.default_rng(4)
    dLdm = rng.normal(size=ref.size).astype(np.float32)
    g = soft.soft_backward(flat.to(dev), torch.from_numpy(dLdm).to(dev), prm, T).cpu().numpy()
    ok, rel = _close(g, osoft.grad_from_dm(flat.numpy(), dLdm.astype(np.float64), p, T))
    assert ok, rel


@pytest.mark.parametrize("T", [0.5, 2.0])
def test_zero_distance_pixels(T):
    """Black pixels sit exactly at mu = (128, 128) with S = I, in FP32 as in
    FP64: d = 0, m = sigmoid(theta / T) in closed form, and they add nothing
    to the mean and covariance gradients (the reading at d = 0); mixed with
    generic pixels, the whole gradient still matches the FP64 oracle."""
    from oracle import soft as osoft
    from paper_1907_04393_amd import soft
    dev = need_gpu()
    f, _ = _calib(1)
    black = torch.zeros((1000, 3), dtype=torch.uint8)
    flat = torch.cat([black, f[0, :64].reshape(-1, 3), black[:3]]).contiguous()
    p = (128.0, 128.0, 1.0, 0.0, 1.0, 1.3)
    prm = torch.tensor(p, dtype=torch.float64)
    closed = 1.0 / (1.0 + np.exp(-1.3 / T))
    m = soft.soft_forward(flat.to(dev), prm, T).cpu().numpy().astype(np.float64)
    ref = osoft.mask(flat.numpy(), p, T)
    assert np.abs(m[:1000] - closed).max() < 2e-5
    assert np.abs(m - ref).max() < 2e-5
    rng = np.random.default_rng(7)
    dLdm = rng.normal(size=ref.size).astype(np.float32)
    g = soft.soft_backward(flat.to(dev), torch.from_numpy(dLdm).to(dev), prm, T).cpu().numpy()
    ok, rel = _close(g, osoft.grad_from_dm(flat.numpy(), dLdm.astype(np.float64), p, T))
    assert ok, rel
    g0 = soft.soft_backward(black.to(dev), torch.from_numpy(dLdm[:1000]).to(dev), prm, T).cpu().numpy()
    assert np.all(g0[:5] == 0.0)
    dth = float(np.sum(dLdm[:1000].astype(np.float64)) * closed * (1.0 - closed) / T)
    assert abs(g0[5] - dth) <= 1e-4 * abs(dth)


@pytest.mark.parametrize("T", [0.5, 2.0])
def test_calibration_workload_full_size(T):
    """32 frames 1280x720 with ground-truth hand masks: the fused BCE pass and
    the autograd path (soft mask, torch BCE, hand-written backward) both
    match the FP64 oracle's loss and gradient."""
    from oracle import soft as osoft
    from paper_1907_04393_amd import soft
    dev = need_gpu()
    f, gt = _calib(32)
    p = POINTS[0]
    print("calibration 32x1280x720, T", T, flush=True)
    fd, gd = f.to(dev), gt.to(dev)
    prm = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    loss = soft.soft_bce(fd, gd, prm, T)
    loss.backward()
    g_fused = prm.grad.numpy().copy()
    fn, gn = f.numpy(), gt.numpy()
    ref_loss = osoft.bce_loss(fn, gn, p, T)
    ref_g = osoft.grad_bce(fn, gn, p, T)
    assert abs(loss.item() - ref_loss) <= 1e-4 * abs(ref_loss)
    ok, rel = _close(g_fused, ref_g)
    assert ok, rel
    # the autograd route: the FP32 soft mask, a loss taken in FP64 torch ops
    # over it, dL/dm handed back in FP32 to the hand-written adjoint
    prm2 = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    m = soft.SoftMask.apply(fd, prm2, T)
    l2 = torch.nn.functional.binary_cross_entropy(m.double(), gd.double())
    l2.backward()
    assert abs(l2.item() - ref_loss) <= 1e-4 * abs(ref_loss)
    ok, rel = _close(prm2.grad.numpy(), ref_g)
    assert ok, rel


def test_deterministic_and_calibrates():
    from paper_1907_04393_amd import soft
    dev = need_gpu()
    f, gt = _calib(4)
    fd, gd = f.to(dev), gt.to(dev)
    p0 = torch.tensor((115.0, 140.0, 200.0, 0.0, 150.0, 2.0), dtype=torch.float64)
    outs = []
    for _ in range(2):
        prm = p0.clone().requires_grad_(True)
        soft.soft_bce(fd, gd, prm, 1.0).backward()
        outs.append(prm.grad.numpy().copy())
    assert np.array_equal(outs[0], outs[1])
    prm = p0.clone().requires_grad_(True)
    opt = torch.optim.Adam([prm], lr=1.0)
    losses = []
    for _ in range(40):
        opt.zero_grad()
        loss = soft.soft_bce(fd, gd, prm, 1.0)
        loss.backward()
        opt.step()
        with torch.no_grad():            # keep the covariance positive definite
            prm[2].clamp_(min=5.0)
            prm[4].clamp_(min=5.0)
            lim = 0.95 * torch.sqrt(prm[2] * prm[4])
            prm[3].clamp_(-lim, lim)
        losses.append(loss.item())
    assert losses[-1] < 0.7 * losses[0], losses[::8]


def test_rejects_bad_parameters():
    from paper_1907_04393_amd import fizi, soft
    dev = need_gpu()
    f = torch.zeros((1, 8, 3), dtype=torch.uint8, device=dev)
    with pytest.raises(fizi.FiziError):
        soft.soft_forward(f, torch.tensor([100, 150, 1.0, 2.0, 1.0, 1.0]), 1.0)
    with pytest.raises(fizi.FiziError):
        soft.soft_forward(f, torch.tensor([100, 150, 1.0, 0.0, 1.0, 1.0]), 0.0)
