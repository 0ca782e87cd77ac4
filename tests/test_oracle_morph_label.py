"""Pins of the oracle's erosion/dilation (Section 3.1, last paragraph) and of
the 8-connected labelling of the Mouse module (Section 2)."""
import numpy as np
import pytest
from scipy import ndimage

SQ = np.ones((3, 3), bool)


def _sc_erode(m):
    return ndimage.binary_erosion(m.astype(bool), structure=SQ, border_value=1).astype(np.uint8)


def _sc_dilate(m):
    return ndimage.binary_dilation(m.astype(bool), structure=SQ, border_value=0).astype(np.uint8)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (5, 1), (8, 8), (17, 33), (64, 64), (37, 100)])
def test_erode_dilate_vs_scipy(orc, shape):
    rng = np.random.default_rng(sum(shape))
    for density in (0.2, 0.5, 0.85):
        m = (rng.random(shape) < density).astype(np.uint8)
        assert (orc.erode(m) == _sc_erode(m)).all()
        assert (orc.dilate(m) == _sc_dilate(m)).all()


def test_all_4x4_masks_brute_force(orc):
    """Every 4x4 mask: opening-then-closing equals the composition of scipy's
    textbook operators."""
    for code in range(1 << 16):
        m = np.array([(code >> i) & 1 for i in range(16)], np.uint8).reshape(4, 4)
        want = _sc_erode(_sc_dilate(_sc_dilate(_sc_erode(m))))
        assert (orc.morph(m, 1, 1) == want).all(), code


def test_open_close_idempotent_and_iterations(orc):
    rng = np.random.default_rng(4)
    m = (rng.random((40, 64)) < 0.55).astype(np.uint8)
    o = orc.morph(m, 1, 0)
    assert (orc.morph(o, 1, 0) == o).all()
    c = orc.morph(m, 0, 1)
    assert (orc.morph(c, 0, 1) == c).all()
    for k in (2, 3):
        want = m
        for _ in range(k):
            want = _sc_erode(want)
        for _ in range(k):
            want = _sc_dilate(want)
        for _ in range(k):
            want = _sc_dilate(want)
        for _ in range(k):
            want = _sc_erode(want)
        assert (orc.morph(m, k, k) == want).all()


def test_opening_removes_small_objects(orc):
    m = np.zeros((32, 64), np.uint8)
    m[5, 5] = 1                 # isolated pixel
    m[10:12, 20:40] = 1         # 2-row bar: no 3x3 square fits
    m[20:25, 30:36] = 1         # survives
    out = orc.morph(m, 1, 0)
    assert out[:15].sum() == 0 and (out[20:25, 30:36] == 1).all()


def _partition(lab):
    """Canonical form of a labelling: each pixel's label renumbered by first
    raster appearance."""
    flat = lab.ravel()
    mapping = {}
    out = np.zeros_like(flat)
    for i, v in enumerate(flat):
        if v:
            out[i] = mapping.setdefault(v, len(mapping) + 1)
    return out.reshape(lab.shape)


@pytest.mark.parametrize("seed", range(6))
def test_label_vs_scipy(orc, seed):
    rng = np.random.default_rng(seed)
    shape = [(1, 64), (30, 1), (20, 20), (48, 64), (33, 70), (64, 128)][seed]
    m = (rng.random(shape) < 0.45).astype(np.uint8)
    lab, k = orc.label(m)
    sl, sk = ndimage.label(m, structure=SQ)
    assert k == sk
    assert (_partition(lab) == _partition(sl)).all()
