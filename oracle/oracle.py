"""ctypes wrapper of the CPU oracle (oracle/fizi_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg. The GPU library never imports, links or runs
anything under oracle/.

Masks here are byte images (one uint8 0/1 per pixel, H x W); frames are
H x W x 3 uint8 RGB. Beside the wrappers, one step is written here in plain
Python: the click debouncing of a tracked stream (ClickDebounce, reading R13:
Section 2, the Mouse module tracks the hand and reports its click state),
a state machine of two integers per stream.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fizi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Defaults of the readings (hue interval, margins, morphology, click, gain).
DEFAULTS = dict(alpha1_cdeg=33000, alpha2_cdeg=7500, gray_S=20, bg_delta=10,
                open_iters=1, close_iters=1, min_area=1, click_fill_permille=700,
                gain_row_stride=8, gain_lo_q16=32768, gain_hi_q16=131072, brightness_mode=0,
                click_debounce=0, track_radius=64, lum_hi=0)


class Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in DEFAULTS]


class Pointer(ctypes.Structure):
    _fields_ = [("present", ctypes.c_uint32), ("click", ctypes.c_uint32),
                ("area", ctypes.c_uint32), ("n_components", ctypes.c_uint32),
                ("inv_gain_q16", ctypes.c_uint32),
                ("x0", ctypes.c_uint32), ("y0", ctypes.c_uint32),
                ("x1", ctypes.c_uint32), ("y1", ctypes.c_uint32),
                ("sum_x", ctypes.c_uint64), ("sum_y", ctypes.c_uint64),
                ("frame_index", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no vectorisation pragmas)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u8p = P(ctypes.c_uint8)
        L.orc_hue_in.argtypes = [ctypes.c_int] * 5
        L.orc_hue_fraction.argtypes = [ctypes.c_int] * 3 + [P(ctypes.c_int64)] * 2
        L.orc_make_yref.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_uint16)]
        L.orc_gain.argtypes = [u8p, P(ctypes.c_uint16), ctypes.c_int, ctypes.c_int, P(Params)]
        L.orc_gain.restype = ctypes.c_uint32
        L.orc_correct_value.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.orc_correct.argtypes = [u8p, ctypes.c_uint32, ctypes.c_size_t, u8p]
        L.orc_learn.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(Params), ctypes.c_int,
                                u8p, u8p, P(ctypes.c_uint16), P(ctypes.c_uint32)]
        L.orc_relearn.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(Params), u8p, u8p,
                                  P(ctypes.c_uint16), P(ctypes.c_uint32)]
        L.orc_masks.argtypes = [u8p, u8p, u8p, ctypes.c_size_t, P(Params), u8p, u8p, u8p, u8p]
        L.orc_filtered_chroma.argtypes = [ctypes.c_int] * 4 + [P(ctypes.c_int64)] * 2
        L.orc_masks_scaled.argtypes = [u8p, u8p, u8p, ctypes.c_size_t, ctypes.c_uint32, P(Params),
                                       u8p, u8p, u8p, u8p]
        L.orc_erode.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int]
        L.orc_dilate.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int]
        L.orc_morph.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p]
        L.orc_label.argtypes = [u8p, ctypes.c_int, ctypes.c_int, P(ctypes.c_int32)]
        L.orc_pointer_of.argtypes = [u8p, ctypes.c_int, ctypes.c_int, P(Params), ctypes.c_uint32,
                                     ctypes.c_uint64, P(Pointer), u8p]
        L.orc_process.argtypes = [u8p, u8p, u8p, P(ctypes.c_uint16), ctypes.c_int, ctypes.c_int,
                                  P(Params), ctypes.c_uint64, P(Pointer), u8p, u8p, u8p]
        L.orc_process_track.argtypes = [u8p, u8p, u8p, P(ctypes.c_uint16), ctypes.c_int, ctypes.c_int,
                                        P(Params), ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                        P(Pointer), u8p, u8p, u8p]
        L.orc_pointer_track.argtypes = [u8p, ctypes.c_int, ctypes.c_int, P(Params), ctypes.c_uint32,
                                        ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, P(Pointer), u8p]
        _lib = L
    return _lib


def params(**kw) -> Params:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(k)
        d[k] = int(v)
    return Params(**d)


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


# -- the steps --------------------------------------------------------------
def hue_in(r, g, b, a1=DEFAULTS["alpha1_cdeg"], a2=DEFAULTS["alpha2_cdeg"]) -> bool:
    return bool(lib().orc_hue_in(int(r), int(g), int(b), int(a1), int(a2)))


def hue_fraction(r, g, b):
    hn, hd = ctypes.c_int64(), ctypes.c_int64()
    ok = lib().orc_hue_fraction(int(r), int(g), int(b), ctypes.byref(hn), ctypes.byref(hd))
    return (hn.value, hd.value) if ok else None


def filtered_chroma(r, g, b, lum_hi):
    """Chroma (units of 1/255) of the pixel after the over-exposure filter
    (R14), as an exact (numerator, denominator)."""
    n, d = ctypes.c_int64(), ctypes.c_int64()
    lib().orc_filtered_chroma(int(r), int(g), int(b), int(lum_hi), ctypes.byref(n), ctypes.byref(d))
    return n.value, d.value


def correct_value(v, inv) -> int:
    return int(lib().orc_correct_value(int(v), int(inv)))


def correct(frame, inv):
    f = _c(frame, np.uint8)
    out = np.empty_like(f)
    lib().orc_correct(_u8(f), int(inv), f.size, _u8(out))
    return out


def make_yref(frame0, p=None):
    p = p or params()
    f = _c(frame0, np.uint8)
    H, W = f.shape[:2]
    rows = (H + p.gain_row_stride - 1) // p.gain_row_stride
    yref = np.zeros((rows, W), np.uint16)
    lib().orc_make_yref(_u8(f), W, H, p.gain_row_stride,
                        yref.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)))
    return yref


def gain(frame, yref, p=None) -> int:
    p = p or params()
    f = _c(frame, np.uint8)
    H, W = f.shape[:2]
    y = _c(yref, np.uint16)
    return int(lib().orc_gain(_u8(f), y.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)), W, H,
                              ctypes.byref(p)))


class Model:
    """Background model: per-pixel, per-channel min/max plus the reference
    luminance rows."""

    def __init__(self, W, H, p=None):
        self.p = p or params()
        self.W, self.H = W, H
        rows = (H + self.p.gain_row_stride - 1) // self.p.gain_row_stride
        self.bgmin = np.full((H, W, 3), 255, np.uint8)
        self.bgmax = np.zeros((H, W, 3), np.uint8)
        self.yref = np.zeros((rows, W), np.uint16)
        self.learned = False

    def learn(self, frames, reset=True):
        f = _c(frames, np.uint8)
        n = f.shape[0]
        inv = np.zeros(max(n, 1), np.uint32)
        rc = lib().orc_learn(_u8(f), n, self.W, self.H, ctypes.byref(self.p), int(bool(reset)),
                             _u8(self.bgmin), _u8(self.bgmax),
                             self.yref.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                             inv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        if rc != 0:
            raise ValueError(f"orc_learn failed ({rc})")
        self.learned = True
        return inv[:n]

    def relearn(self, frames, fizi):
        """Partial re-learning (Section 3.3, reading R9): widen the model with
        frames (n, H, W, 3) at the pixels where fizi (n, H, W, 0/1) is 0."""
        if not self.learned:
            raise ValueError("relearn needs a learned model")
        f = _c(frames, np.uint8)
        m = _c((np.asarray(fizi) != 0).astype(np.uint8), np.uint8)
        n = f.shape[0]
        assert m.shape == (n, self.H, self.W)
        inv = np.zeros(max(n, 1), np.uint32)
        rc = lib().orc_relearn(_u8(f), _u8(m), n, self.W, self.H, ctypes.byref(self.p),
                               _u8(self.bgmin), _u8(self.bgmax),
                               self.yref.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                               inv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        if rc != 0:
            raise ValueError(f"orc_relearn failed ({rc})")
        return inv[:n]

    def process(self, frame, frame_index=0, want_raw=False, want_hand=False, track=None):
        """One running-phase frame. track: None (R7), or the previous frame's
        centroid pixel (x, y) for temporal tracking (R10)."""
        f = _c(frame, np.uint8)
        npx = self.W * self.H
        fizi = np.zeros((self.H, self.W), np.uint8)
        raw = np.zeros((self.H, self.W), np.uint8) if want_raw else None
        hand = np.zeros((self.H, self.W), np.uint8) if want_hand else None
        ptr = Pointer()
        null = ctypes.POINTER(ctypes.c_uint8)()
        tx, ty = track if track is not None else (-1, -1)
        rc = lib().orc_process_track(_u8(f), _u8(self.bgmin), _u8(self.bgmax),
                                     self.yref.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                     self.W, self.H, ctypes.byref(self.p), int(frame_index), int(tx), int(ty),
                                     ctypes.byref(ptr), _u8(raw) if raw is not None else null,
                                     _u8(fizi), _u8(hand) if hand is not None else null)
        if rc != 0:
            raise ValueError(f"orc_process failed ({rc})")
        assert fizi.size == npx
        out = dict(pointer=ptr.as_dict(), fizi=fizi)
        if want_raw:
            out["raw"] = raw
        if want_hand:
            out["hand"] = hand
        return out


def masks(frame_corrected, bgmin, bgmax, p=None):
    p = p or params()
    f = _c(frame_corrected, np.uint8)
    H, W = f.shape[:2]
    outs = [np.zeros((H, W), np.uint8) for _ in range(4)]
    lib().orc_masks(_u8(f), _u8(_c(bgmin, np.uint8)), _u8(_c(bgmax, np.uint8)), H * W,
                    ctypes.byref(p), *[_u8(o) for o in outs])
    return dict(r1=outs[0], r2=outs[1], r3=outs[2], raw=outs[3])


def masks_scaled(frame_raw, inv, bgmin, bgmax, p=None):
    """The three masks with the thresholds scaled to the frame's brightness
    (reading R12) instead of corrected pixels."""
    p = p or params()
    f = _c(frame_raw, np.uint8)
    H, W = f.shape[:2]
    outs = [np.zeros((H, W), np.uint8) for _ in range(4)]
    lib().orc_masks_scaled(_u8(f), _u8(_c(bgmin, np.uint8)), _u8(_c(bgmax, np.uint8)), H * W, int(inv),
                           ctypes.byref(p), *[_u8(o) for o in outs])
    return dict(r1=outs[0], r2=outs[1], r3=outs[2], raw=outs[3])


def erode(m):
    m = _c(m, np.uint8)
    out = np.empty_like(m)
    lib().orc_erode(_u8(m), _u8(out), m.shape[1], m.shape[0])
    return out


def dilate(m):
    m = _c(m, np.uint8)
    out = np.empty_like(m)
    lib().orc_dilate(_u8(m), _u8(out), m.shape[1], m.shape[0])
    return out


def morph(m, open_iters=1, close_iters=1):
    m = _c(m, np.uint8)
    out = np.empty_like(m)
    rc = lib().orc_morph(_u8(m), m.shape[1], m.shape[0], int(open_iters), int(close_iters), _u8(out))
    if rc != 0:
        raise MemoryError
    return out


def label(m):
    m = _c(m, np.uint8)
    lab = np.zeros(m.shape, np.int32)
    k = lib().orc_label(_u8(m), m.shape[1], m.shape[0], lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return lab, int(k)


def centroid_pixel(ptr):
    """The tracked pixel of a pointer (R10): floor of the coordinate sums over
    the area, or None without a hand."""
    if not ptr["present"]:
        return None
    return (ptr["sum_x"] // ptr["area"], ptr["sum_y"] // ptr["area"])


class ClickDebounce:
    """Click debouncing of a tracked stream (reading R13): the reported click
    changes only once D consecutive frames show the new state; a frame
    without a hand reports no click and clears the count. D <= 1 reports
    every frame's own click."""

    def __init__(self, D):
        self.D = int(D)
        self.click = 0   # the reported state
        self.count = 0   # consecutive frames that disagree with it

    def step(self, present, raw_click):
        if not present:
            self.click, self.count = 0, 0
            return 0
        if raw_click == self.click:
            self.count = 0
        else:
            self.count += 1
            if self.count >= self.D:
                self.click, self.count = raw_click, 0
        return self.click


class Tracker:
    """Temporal tracking over a frame sequence (R10): each frame's hand is
    the component (of area >= min_area) nearest to the previous frame's
    centroid pixel, within track_radius - the one covering it when there is
    one - else the largest; its click is debounced (R13)."""

    def __init__(self, model):
        self.m = model
        self.prev = None
        self.debounce = ClickDebounce(model.p.click_debounce)

    def process(self, frame, frame_index=0, want_hand=False):
        out = self.m.process(frame, frame_index, want_hand=want_hand, track=self.prev)
        ptr = out["pointer"]
        ptr["click"] = self.debounce.step(ptr["present"], ptr["click"])
        self.prev = centroid_pixel(ptr)
        return out


def pointer_of(fizi, p=None, inv=65536, frame_index=0, want_hand=False, track=None):
    p = p or params()
    m = _c(fizi, np.uint8)
    H, W = m.shape
    ptr = Pointer()
    hand = np.zeros((H, W), np.uint8) if want_hand else None
    tx, ty = track if track is not None else (-1, -1)
    rc = lib().orc_pointer_track(_u8(m), W, H, ctypes.byref(p), int(inv), int(frame_index), int(tx), int(ty),
                                 ctypes.byref(ptr),
                                 _u8(hand) if hand is not None else ctypes.POINTER(ctypes.c_uint8)())
    if rc != 0:
        raise MemoryError
    return (ptr.as_dict(), hand) if want_hand else ptr.as_dict()
