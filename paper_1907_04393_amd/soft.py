"""Differentiable soft skin mask for calibration (binding of the HIP kernels).

SoftMask is a torch.autograd.Function: forward calls fizi_soft_forward,
backward calls the hand-written adjoint fizi_soft_backward. soft_bce is the
fused loss-and-gradient variant against a ground-truth mask. All arithmetic
runs in the HIP library; torch supplies memory, streams and the BCE of the
unfused path.
"""
from __future__ import annotations

import ctypes

import torch

from . import fizi

PARAM_NAMES = ("mu_b", "mu_r", "s_bb", "s_br", "s_rr", "theta")


def _p6(params: torch.Tensor):
    vals = [float(v) for v in params.detach().cpu().reshape(-1).tolist()]
    if len(vals) != 6:
        raise ValueError("params must hold 6 values")
    return (ctypes.c_float * 6)(*vals)


def _check_frames(frames):
    if frames.dtype != torch.uint8 or not frames.is_cuda or not frames.is_contiguous() or frames.shape[-1] != 3:
        raise fizi.FiziError(fizi.FIZI_EINVAL, "frames must be a contiguous (..., 3) uint8 CUDA tensor")


_ws = {}


def workspace(device, npx):
    n = int(fizi.lib().fizi_soft_workspace_bytes(int(npx)))
    key = (str(device), n)
    if key not in _ws:
        _ws[key] = torch.empty(n, dtype=torch.uint8, device=device)
    return _ws[key]


def soft_forward(frames: torch.Tensor, params: torch.Tensor, T: float, out: torch.Tensor = None):
    _check_frames(frames)
    npx = frames.numel() // 3
    if out is None:
        out = torch.empty(frames.shape[:-1], dtype=torch.float32, device=frames.device)
    fizi.check(fizi.lib().fizi_soft_forward(fizi._ptr(frames), npx, _p6(params), float(T), fizi._ptr(out),
                                            fizi._stream(None)))
    return out


def soft_backward(frames, dLdm, params, T):
    _check_frames(frames)
    npx = frames.numel() // 3
    dLdm = dLdm.contiguous().to(torch.float32)
    ws = workspace(frames.device, npx)
    g = torch.empty(6, dtype=torch.float64, device=frames.device)
    fizi.check(fizi.lib().fizi_soft_backward(fizi._ptr(frames), fizi._ptr(dLdm), npx, _p6(params), float(T),
                                             fizi._ptr(ws), ws.numel(), fizi._ptr(g), fizi._stream(None)))
    return g


class SoftMask(torch.autograd.Function):
    """m = sigmoid((theta - Mahalanobis distance in CbCr) / T)."""

    @staticmethod
    def forward(ctx, frames, params, T):
        ctx.save_for_backward(frames, params)
        ctx.T = float(T)
        return soft_forward(frames, params, T)

    @staticmethod
    def backward(ctx, grad_mask):
        frames, params = ctx.saved_tensors
        g = soft_backward(frames, grad_mask, params, ctx.T)
        return None, g.to(device=params.device, dtype=params.dtype), None


class _SoftBCE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, frames, gt, params, T):
        _check_frames(frames)
        npx = frames.numel() // 3
        if gt.dtype != torch.uint8 or gt.numel() != npx or not gt.is_contiguous():
            raise fizi.FiziError(fizi.FIZI_EINVAL, "gt must be a contiguous uint8 mask of one value per pixel")
        ws = workspace(frames.device, npx)
        out = torch.empty(7, dtype=torch.float64, device=frames.device)
        fizi.check(fizi.lib().fizi_soft_bce(fizi._ptr(frames), fizi._ptr(gt), npx, _p6(params), float(T),
                                            fizi._ptr(ws), ws.numel(), fizi._ptr(out), fizi._stream(None)))
        ctx.save_for_backward(out[:6].clone(), params)
        return out[6].clone()

    @staticmethod
    def backward(ctx, grad_loss):
        g, params = ctx.saved_tensors
        return None, None, (g * grad_loss.to(g.dtype).to(g.device)).to(device=params.device,
                                                                       dtype=params.dtype), None


STAGES = ("forward", "backward", "final")


def timing(enable=True):
    """Dispatch-event timing of the soft-mask kernels (process-wide)."""
    fizi.check(fizi.lib().fizi_soft_timing(int(bool(enable))))


def times() -> dict:
    """{kernel: (summed ms, launches)} since the last read; waits for them."""
    ms = (ctypes.c_double * 3)()
    n = (ctypes.c_int64 * 3)()
    fizi.check(fizi.lib().fizi_soft_times(ms, n))
    return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}


def soft_bce_static(frames, gt, params, T, out=None, stream=None):
    """The fused loss and gradient through the allocation-free entry point
    (its partial sums live in the library's static device array): returns
    the 7 doubles (6 gradients, then the loss) in `out` (a device float64
    tensor of 7, allocated here when not given)."""
    _check_frames(frames)
    npx = frames.numel() // 3
    if gt.dtype != torch.uint8 or gt.numel() != npx or not gt.is_contiguous():
        raise fizi.FiziError(fizi.FIZI_EINVAL, "gt must be a contiguous uint8 mask of one value per pixel")
    if out is None:
        out = torch.empty(7, dtype=torch.float64, device=frames.device)
    fizi.check(fizi.lib().fizi_soft_bce_static(fizi._ptr(frames), fizi._ptr(gt), npx, _p6(params), float(T),
                                               fizi._ptr(out), fizi._stream(stream)))
    return out


def soft_bce(frames, gt, params, T):
    """Mean BCE of the soft mask against gt, differentiable in params (one
    fused pass computes the loss and its gradient)."""
    return _SoftBCE.apply(frames, gt, params, T)
