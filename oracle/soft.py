"""FP64 oracle of the soft (sigmoid-relaxed) skin mask and its gradient.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).

This form is not in the paper, whose skin test is the hard hue interval of
Section 3.1 (iii); it is the calibration form that relaxes a chroma model to
a differentiable mask. Readings:
  * chroma: ITU-R BT.601 full-range Cb, Cr of the RGB pixel
        Cb = 128 - 0.168736 R - 0.331264 G + 0.5 B
        Cr = 128 + 0.5 R - 0.418688 G - 0.081312 B;
  * parameters p = (mu_b, mu_r, s_bb, s_br, s_rr, theta): the chroma mean, the
    three free entries of the symmetric covariance S = [[s_bb, s_br],
    [s_br, s_rr]] (positive definite), and the distance threshold;
  * d = sqrt(delta^T S^-1 delta) with delta = (Cb - mu_b, Cr - mu_r) (the
    Mahalanobis distance), z = (theta - d) / T, mask m = sigmoid(z);
  * loss = mean over pixels of the binary cross-entropy of m against the
    ground-truth mask y, written as max(z, 0) - z y + log1p(exp(-|z|));
  * where d = 0 the distance has no derivative; its contribution is taken as
    zero (a measure-zero set).
"""
from __future__ import annotations

import numpy as np


def chroma(frames):
    f = np.asarray(frames, dtype=np.float64).reshape(-1, 3)
    r, g, b = f[:, 0], f[:, 1], f[:, 2]
    cb = 128.0 - 0.168736 * r - 0.331264 * g + 0.5 * b
    cr = 128.0 + 0.5 * r - 0.418688 * g - 0.081312 * b
    return cb, cr


def _parts(frames, p, T):
    mu_b, mu_r, s_bb, s_br, s_rr, theta = [float(v) for v in p]
    cb, cr = chroma(frames)
    db, dr = cb - mu_b, cr - mu_r
    det = s_bb * s_rr - s_br * s_br
    if not (det > 0 and s_bb > 0):
        raise ValueError("covariance must be positive definite")
    # u = S^-1 delta
    ub = (s_rr * db - s_br * dr) / det
    ur = (-s_br * db + s_bb * dr) / det
    q = db * ub + dr * ur
    d = np.sqrt(np.maximum(q, 0.0))
    z = (theta - d) / T
    m = 1.0 / (1.0 + np.exp(-z))
    return dict(db=db, dr=dr, ub=ub, ur=ur, q=q, d=d, z=z, m=m)


def mask(frames, p, T):
    """Soft mask m in (0, 1), one value per pixel (flattened)."""
    return _parts(frames, p, T)["m"]


def bce_loss(frames, gt, p, T):
    z = _parts(frames, p, T)["z"]
    y = np.asarray(gt, dtype=np.float64).reshape(-1)
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def grad_from_dm(frames, dLdm, p, T):
    """Gradient of L with respect to p, given dL/dm per pixel."""
    P = _parts(frames, p, T)
    g = np.asarray(dLdm, dtype=np.float64).reshape(-1)
    gz = g * P["m"] * (1.0 - P["m"])              # dL/dz
    gtheta = np.sum(gz) / T
    gd = -gz / T                                   # dL/dd
    with np.errstate(divide="ignore", invalid="ignore"):
        gq = np.where(P["d"] > 0, gd / (2.0 * P["d"]), 0.0)   # dL/dq
    ub, ur = P["ub"], P["ur"]
    g_mu_b = np.sum(gq * (-2.0 * ub))
    g_mu_r = np.sum(gq * (-2.0 * ur))
    g_s_bb = np.sum(gq * (-ub * ub))
    g_s_br = np.sum(gq * (-2.0 * ub * ur))
    g_s_rr = np.sum(gq * (-ur * ur))
    return np.array([g_mu_b, g_mu_r, g_s_bb, g_s_br, g_s_rr, gtheta])


def grad_bce(frames, gt, p, T):
    """Gradient of the mean BCE loss: dL/dm folded into dL/dz = (m - y) / N."""
    P = _parts(frames, p, T)
    y = np.asarray(gt, dtype=np.float64).reshape(-1)
    m = P["m"]
    with np.errstate(divide="ignore", invalid="ignore"):
        dLdm = (m - y) / (m * (1.0 - m)) / y.size
    return grad_from_dm(frames, dLdm, p, T)


# the parameter point of the calibration workload: chroma box centre, box
# variances (50^2/12, 40^2/12) with a generic off-diagonal term, threshold
CHECK_POINT = (102.0, 153.0, 208.3, 10.0, 133.3, 2.5)
