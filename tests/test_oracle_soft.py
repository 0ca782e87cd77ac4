"""Pins of the FP64 soft-mask oracle: central finite differences, torch's
float64 autograd as an independent derivative, and closed forms."""
import numpy as np
import pytest
import torch

from oracle import soft


def _frames(n=4096, seed=0):
    rng = np.random.default_rng(seed)
    # colours spread around the skin chroma box plus some far away
    y = rng.uniform(90, 190, n)
    cb = rng.uniform(60, 150, n)
    cr = rng.uniform(110, 190, n)
    r = y + 1.402 * (cr - 128)
    g = y - 0.344136 * (cb - 128) - 0.714136 * (cr - 128)
    b = y + 1.772 * (cb - 128)
    f = np.clip(np.rint(np.stack([r, g, b], 1)), 0, 255).astype(np.uint8)
    gt = (np.abs(cb - 102) < 25) & (np.abs(cr - 153) < 20)
    return f, gt.astype(np.uint8)


POINTS = [soft.CHECK_POINT, (110.0, 148.0, 300.0, -40.0, 150.0, 1.7), (95.0, 160.0, 180.0, 25.0, 120.0, 3.1)]


def test_chroma_closed_forms():
    grays = np.array([[v, v, v] for v in (0, 17, 128, 255)], np.uint8)
    cb, cr = soft.chroma(grays)
    assert np.allclose(cb, 128.0, atol=1e-12) and np.allclose(cr, 128.0, atol=1e-12)
    cb, cr = soft.chroma(np.array([[0, 0, 255], [255, 0, 0]], np.uint8))
    assert abs(cb[0] - 255.5) < 1e-9 and abs(cr[1] - 255.5) < 1e-9


@pytest.mark.parametrize("p", POINTS)
@pytest.mark.parametrize("T", [0.5, 2.0])
def test_gradient_vs_central_differences(p, T):
    f, gt = _frames()
    g = soft.grad_bce(f, gt, p, T)
    for i in range(6):
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = list(p), list(p)
        pp[i] += h
        pm[i] -= h
        fd = (soft.bce_loss(f, gt, pp, T) - soft.bce_loss(f, gt, pm, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.abs(g).max()), (i, fd, g[i])


@pytest.mark.parametrize("p", POINTS)
def test_gradient_vs_torch_autograd_float64(p):
    """torch float64 autograd of the same loss written in torch ops."""
    f, gt = _frames(seed=3)
    T = 0.5
    rng = np.random.default_rng(9)
    dLdm = rng.normal(size=f.shape[0])
    x = torch.tensor(f, dtype=torch.float64)
    prm = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    cb = 128.0 - 0.168736 * x[:, 0] - 0.331264 * x[:, 1] + 0.5 * x[:, 2]
    cr = 128.0 + 0.5 * x[:, 0] - 0.418688 * x[:, 1] - 0.081312 * x[:, 2]
    S = torch.stack([torch.stack([prm[2], prm[3]]), torch.stack([prm[3], prm[4]])])
    Sinv = torch.linalg.inv(S)
    dlt = torch.stack([cb - prm[0], cr - prm[1]], 1)
    q = torch.einsum("ni,ij,nj->n", dlt, Sinv, dlt)
    m = torch.sigmoid((prm[5] - torch.sqrt(q)) / T)
    (m * torch.tensor(dLdm)).sum().backward()
    assert np.allclose(soft.mask(f, p, T), m.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert np.allclose(soft.grad_from_dm(f, dLdm, p, T), prm.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_zero_distance_closed_form():
    """S = I and mu at the pixel's chroma: d = 0, m = sigmoid(theta / T), and
    only theta carries gradient."""
    f = np.array([[150, 100, 80]], np.uint8)
    cb, cr = soft.chroma(f)
    p = (cb[0], cr[0], 1.0, 0.0, 1.0, 1.3)
    for T in (0.5, 2.0):
        m = soft.mask(f, p, T)[0]
        assert abs(m - 1.0 / (1.0 + np.exp(-1.3 / T))) < 1e-15
        g = soft.grad_from_dm(f, [1.0], p, T)
        assert np.all(g[:5] == 0.0) and abs(g[5] - m * (1 - m) / T) < 1e-15


def test_low_temperature_approaches_hard_threshold():
    f, _ = _frames(seed=5)
    p = soft.CHECK_POINT
    P = soft._parts(f, p, 1.0)
    far = np.abs(P["d"] - p[5]) > 0.05
    m = soft.mask(f, p, 1e-4)
    assert np.array_equal(m[far] > 0.5, (P["d"] < p[5])[far])
    assert np.all((m[far] < 1e-6) | (m[far] > 1 - 1e-6))


def test_rejects_non_positive_definite():
    f, _ = _frames(n=8)
    with pytest.raises(ValueError):
        soft.mask(f, (100, 150, 1.0, 2.0, 1.0, 1.0), 1.0)
