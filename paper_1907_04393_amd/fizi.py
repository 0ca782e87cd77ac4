"""Python binding of libfizi.so: argument marshalling only.

Every step of the pipeline runs in the HIP library; torch supplies device
memory (the state block, frames, outputs) and the stream. Names follow the C
ABI in include/fizi.h: learn_background, process_frames, get_pointer.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libfizi.so")

FIZI_OK, FIZI_EINVAL, FIZI_ESTATE, FIZI_ENOMEM, FIZI_EHIP, FIZI_ERANGE = 0, -1, -2, -3, -4, -5

PARAM_FIELDS = ("alpha1_cdeg", "alpha2_cdeg", "gray_S", "bg_delta", "open_iters", "close_iters",
                "min_area", "click_fill_permille", "gain_row_stride", "gain_lo_q16", "gain_hi_q16",
                "brightness_mode", "click_debounce", "track_radius", "lum_hi")


class Geom(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in PARAM_FIELDS]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k in PARAM_FIELDS}


class PointerC(ctypes.Structure):
    _fields_ = [("present", ctypes.c_uint8), ("click", ctypes.c_uint8),
                ("reserved", ctypes.c_uint16), ("area", ctypes.c_uint32),
                ("sum_x", ctypes.c_uint64), ("sum_y", ctypes.c_uint64),
                ("x0", ctypes.c_uint32), ("y0", ctypes.c_uint32),
                ("x1", ctypes.c_uint32), ("y1", ctypes.c_uint32),
                ("n_components", ctypes.c_uint32), ("inv_gain_q16", ctypes.c_uint32),
                ("frame_index", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("cls_iters", ctypes.c_int32), ("morph_rows", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("mode", ctypes.c_int32), ("short_bands", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Layout(ctypes.Structure):
    _fields_ = [("bgmin", ctypes.c_uint64), ("bgmax", ctypes.c_uint64), ("yref", ctypes.c_uint64),
                ("yref_rows", ctypes.c_uint64), ("total", ctypes.c_uint64)]


POINTER_DTYPE = np.dtype([("present", "u1"), ("click", "u1"), ("reserved", "<u2"), ("area", "<u4"),
                          ("sum_x", "<u8"), ("sum_y", "<u8"), ("x0", "<u4"), ("y0", "<u4"),
                          ("x1", "<u4"), ("y1", "<u4"), ("n_components", "<u4"),
                          ("inv_gain_q16", "<u4"), ("frame_index", "<u8")])
assert POINTER_DTYPE.itemsize == ctypes.sizeof(PointerC) == 56


class ZoneC(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("x0", "y0", "x1", "y1")]


class WheelC(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("cx", "cy", "r_min", "r_max", "dead_cdeg", "full_cdeg")]


DRIVE_FIELDS = ("on_wheel", "angle_cdeg", "steer_permille", "accelerate")


class FiziError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fizi error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, vp, i32, i64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.fizi_last_error.restype = ctypes.c_char_p
    L.fizi_default_params.argtypes = [P(Params)]
    L.fizi_validate.argtypes = [P(Geom), P(Params)]
    L.fizi_state_bytes.argtypes = [P(Geom), P(Params), i32]
    L.fizi_state_bytes.restype = ctypes.c_size_t
    L.fizi_state_layout.argtypes = [P(Geom), P(Params), i32, P(Layout)]
    L.fizi_create.argtypes = [P(Geom), P(Params), i32, vp, ctypes.c_size_t, vp, P(vp)]
    L.learn_background.argtypes = [vp, vp, i32, i32, vp]
    L.relearn_background.argtypes = [vp, vp, i32, vp, vp]
    L.fizi_set_tracking.argtypes = [vp, i32]
    L.fizi_set_pipelined.argtypes = [vp, i32]
    L.fizi_set_short_bands.argtypes = [vp, i32]
    L.fizi_flush.argtypes = [vp, vp]
    L.process_frames.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    L.get_pointer.argtypes = [vp, i64, P(PointerC)]
    L.fizi_destroy.argtypes = [vp]
    L.fizi_stage_timing.argtypes = [vp, i32]
    L.fizi_stage_times.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int64)]
    _extra_signatures(L)
    if hasattr(L, "fizi_zone_hit"):
        L.fizi_zone_hit.argtypes = [vp, i32, vp, i32, vp]
        L.fizi_drive_of.argtypes = [vp, i32, P(WheelC), vp]
    _lib = L
    return L


def _extra_signatures(L):
    """Signatures of the batched and soft-mask entry points, when present."""
    P, vp, i32, i64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    if hasattr(L, "fizi_batch_create"):
        L.fizi_batch_state_bytes.argtypes = [i32, P(Geom), P(Params)]
        L.fizi_batch_state_bytes.restype = ctypes.c_size_t
        L.fizi_batch_create.argtypes = [i32, P(Geom), P(Params), vp, ctypes.c_size_t, P(vp)]
        L.fizi_batch_learn.argtypes = [vp, i32, vp, i32, i32, vp]
        L.fizi_batch_relearn.argtypes = [vp, i32, vp, i32, vp, vp]
        L.fizi_batch_set_tracking.argtypes = [vp, i32, i32]
        L.fizi_batch_step.argtypes = [vp, P(vp), P(vp), vp, vp]
        L.fizi_batch_set_mode.argtypes = [vp, i32]
        L.fizi_batch_flush.argtypes = [vp, vp]
        L.fizi_batch_status.argtypes = [vp, P(ctypes.c_uint32)]
        L.fizi_batch_state_layout.argtypes = [vp, i32, P(Layout)]
        L.fizi_batch_stage_timing.argtypes = [vp, i32]
        L.fizi_batch_stage_times.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int64)]
        L.fizi_batch_destroy.argtypes = [vp]
        L.fizi_batch_get_tuning.argtypes = [vp, P(Tuning)]
        L.fizi_batch_set_tuning.argtypes = [vp, P(Tuning)]
        L.fizi_batch_autotune.argtypes = [vp, P(vp), vp, i32, vp, P(Tuning), P(ctypes.c_double)]
    if hasattr(L, "fizi_soft_forward"):
        L.fizi_soft_forward.argtypes = [vp, i64, P(ctypes.c_float), ctypes.c_float, vp, vp]
        L.fizi_soft_workspace_bytes.argtypes = [i64]
        L.fizi_soft_workspace_bytes.restype = ctypes.c_size_t
        L.fizi_soft_backward.argtypes = [vp, vp, i64, P(ctypes.c_float), ctypes.c_float, vp,
                                         ctypes.c_size_t, vp, vp]
        L.fizi_soft_bce.argtypes = [vp, vp, i64, P(ctypes.c_float), ctypes.c_float, vp,
                                    ctypes.c_size_t, vp, vp]
        L.fizi_soft_bce_static.argtypes = [vp, vp, i64, P(ctypes.c_float), ctypes.c_float, vp, vp]
        L.fizi_soft_timing.argtypes = [i32]
        L.fizi_soft_times.argtypes = [P(ctypes.c_double), P(ctypes.c_int64)]


def check(rc):
    if rc != FIZI_OK:
        raise FiziError(rc, lib().fizi_last_error().decode())
    return rc


def last_error() -> str:
    return lib().fizi_last_error().decode()


def default_params(**overrides) -> Params:
    p = Params()
    check(lib().fizi_default_params(ctypes.byref(p)))
    for k, v in overrides.items():
        if k not in PARAM_FIELDS:
            raise KeyError(k)
        setattr(p, k, int(v))
    return p


def state_bytes(width, height, params=None, chunk=16) -> int:
    params = params or default_params()
    return int(lib().fizi_state_bytes(ctypes.byref(Geom(width, height)), ctypes.byref(params), chunk))


def _device(device) -> torch.device:
    """A CUDA device with its index ("cuda" is the current device), so that it
    compares equal to the device of the tensors allocated on it."""
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def pointers_to_numpy(t: torch.Tensor) -> np.ndarray:
    """Device (n, 56) uint8 tensor of fizi_pointer -> structured numpy array."""
    return t.detach().cpu().numpy().reshape(-1).view(POINTER_DTYPE)


def pointer_dict(rec) -> dict:
    return {k: int(rec[k]) for k in POINTER_DTYPE.names if k != "reserved"}


class Context:
    """One camera stream: its learned model and scratch live in `self.state`."""

    def __init__(self, width, height, params=None, chunk=16, device="cuda", stream=None):
        L = lib()
        self.width, self.height = int(width), int(height)
        self.params = params or default_params()
        self.chunk = int(chunk)
        self.geom = Geom(self.width, self.height)
        nbytes = int(L.fizi_state_bytes(ctypes.byref(self.geom), ctypes.byref(self.params), self.chunk))
        if nbytes == 0:
            check(L.fizi_validate(ctypes.byref(self.geom), ctypes.byref(self.params)))
            raise FiziError(FIZI_EINVAL, "chunk must be in [1, 256]")
        self.device = _device(device)
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._pipelined = False
        # outputs a pipelined call is still writing (see set_pipelined)
        self._held = None
        self._h = ctypes.c_void_p()
        check(L.fizi_create(ctypes.byref(self.geom), ctypes.byref(self.params), self.chunk,
                            _ptr(self.state), nbytes, _stream(stream), ctypes.byref(self._h)))
        lay = Layout()
        check(L.fizi_state_layout(ctypes.byref(self.geom), ctypes.byref(self.params), self.chunk,
                                  ctypes.byref(lay)))
        self.layout = lay
        self.words = self.height * (self.width // 64)

    # -- the C ABI ------------------------------------------------------------
    def learn_background(self, frames: torch.Tensor, reset=True, stream=None):
        self._check_frames(frames)
        check(lib().learn_background(self._h, _ptr(frames), int(frames.shape[0]), int(bool(reset)),
                                     _stream(stream)))

    def relearn_background(self, frames: torch.Tensor, fizi_bits: torch.Tensor, stream=None):
        """Partial re-learning: widen the model with frames at the pixels
        whose bit in fizi_bits ((n, H, W/64) int64, as process_frames
        returns them) is 0."""
        self._check_frames(frames)
        self._check_bits(fizi_bits, int(frames.shape[0]))
        check(lib().relearn_background(self._h, _ptr(frames), int(frames.shape[0]), _ptr(fizi_bits),
                                       _stream(stream)))

    def set_tracking(self, enable=True):
        """Temporal tracking of the hand zone (see fizi_set_tracking)."""
        check(lib().fizi_set_tracking(self._h, int(bool(enable))))

    def set_pipelined(self, enable=True):
        """Pipelined calls (see fizi_set_pipelined): a call's outputs are
        complete once the next call, or flush(), has completed on its stream.
        Until then the context keeps a reference to them, so that their
        memory is not handed out while they are still being written."""
        check(lib().fizi_set_pipelined(self._h, int(bool(enable))))
        self._pipelined = bool(enable)
        self._held = None

    def set_short_bands(self, enable=True):
        """Short morphology bands for launches too small to fill the device
        (see fizi_set_short_bands); results do not depend on it."""
        check(lib().fizi_set_short_bands(self._h, int(bool(enable))))

    def flush(self, stream=None):
        """Completes every call's outputs on the stream."""
        check(lib().fizi_flush(self._h, _stream(stream)))
        self._held = None

    def _check_bits(self, bits, n):
        if (bits.dtype != torch.int64 or not bits.is_contiguous()
                or tuple(bits.shape) != (n, self.height, self.width // 64)):
            raise FiziError(FIZI_EINVAL, f"masks must be contiguous int64 ({n}, {self.height}, {self.width // 64})")

    def process_frames(self, frames: torch.Tensor, want_fizi=True, want_hand=False, stream=None):
        """Returns dict(pointers=(n,56) uint8, fizi=(n,H,W/64) int64 bits or
        None, hand=... or None); all device tensors, filled asynchronously."""
        self._check_frames(frames)
        n = int(frames.shape[0])
        shape = (n, self.height, self.width // 64)
        # the outputs are written on `stream`: allocated there, so that the
        # caching allocator does not hand their memory out before it is done
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(self.device)):
            fz = torch.empty(shape, dtype=torch.int64, device=self.device) if want_fizi else None
            hd = torch.empty(shape, dtype=torch.int64, device=self.device) if want_hand else None
            ptrs = torch.empty((n, 56), dtype=torch.uint8, device=self.device)
        check(lib().process_frames(self._h, _ptr(frames), n, _ptr(fz), _ptr(hd), _ptr(ptrs),
                                   _stream(stream)))
        if self._pipelined:
            self._held = (fz, hd, ptrs)
        return dict(pointers=ptrs, fizi=fz, hand=hd)

    def process_into(self, frames, n, fizi=None, hand=None, pointers=None, stream=None):
        """process_frames into caller tensors (no allocation)."""
        check(lib().process_frames(self._h, _ptr(frames), int(n), _ptr(fizi), _ptr(hand),
                                   _ptr(pointers), _stream(stream)))
        if self._pipelined:
            self._held = (fizi, hand, pointers)

    def get_pointer(self, frame_index: int) -> dict:
        out = PointerC()
        check(lib().get_pointer(self._h, int(frame_index), ctypes.byref(out)))
        return {k: int(getattr(out, k)) for k, _ in PointerC._fields_ if k != "reserved"}

    STAGES = ("gain", "classify", "morph", "resolve", "learn")

    def stage_timing(self, enable=True):
        check(lib().fizi_stage_timing(self._h, int(bool(enable))))

    def stage_times(self) -> dict:
        """{stage: (total ms, launches)} since the last read."""
        ms = (ctypes.c_double * 5)()
        n = (ctypes.c_int64 * 5)()
        check(lib().fizi_stage_times(self._h, ms, n))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(self.STAGES)}

    # -- helpers --------------------------------------------------------------
    def model(self):
        """Views of the learned model inside the state block."""
        L = self.layout
        px3 = self.width * self.height * 3
        bgmin = self.state[L.bgmin:L.bgmin + px3].view(self.height, self.width, 3)
        bgmax = self.state[L.bgmax:L.bgmax + px3].view(self.height, self.width, 3)
        ny = int(L.yref_rows) * self.width * 2
        yref = self.state[L.yref:L.yref + ny].view(torch.int16).view(int(L.yref_rows), self.width)
        return bgmin, bgmax, yref

    def _check_frames(self, frames):
        if frames.dtype != torch.uint8 or frames.device != self.device or not frames.is_contiguous():
            raise FiziError(FIZI_EINVAL, "frames must be a contiguous uint8 tensor on the context's device")
        if tuple(frames.shape[1:]) != (self.height, self.width, 3):
            raise FiziError(FIZI_EINVAL, f"frames must be (n, {self.height}, {self.width}, 3)")

    def close(self):
        if self._h:
            lib().fizi_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BATCH_DIRECT, BATCH_GRAPH, BATCH_PERSISTENT, BATCH_PERSISTENT_GRAPH = 0, 1, 2, 3
# software-pipelined across steps: a step's outputs are written by the next
# step or by flush()
BATCH_PIPELINED, BATCH_PIPELINED_GRAPH = 4, 5


class Batch:
    """Many camera streams, one pipeline pass over all active ones per step."""

    def __init__(self, geoms, params=None, device="cuda"):
        L = lib()
        self.n = len(geoms)
        self.geoms = [(int(w), int(h)) for w, h in geoms]
        if params is None or isinstance(params, Params):
            params = [params or default_params()] * self.n
        self.params = list(params)
        self._g = (Geom * self.n)(*[Geom(w, h) for w, h in self.geoms])
        self._p = (Params * self.n)(*self.params)
        nbytes = int(L.fizi_batch_state_bytes(self.n, self._g, self._p))
        if nbytes == 0:
            raise FiziError(FIZI_EINVAL, "invalid stream geometry or parameters")
        self.device = _device(device)
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        check(L.fizi_batch_create(self.n, self._g, self._p, _ptr(self.state), nbytes, ctypes.byref(self._h)))
        self._frames = (ctypes.c_void_p * self.n)()
        self._fizi = (ctypes.c_void_p * self.n)()
        self._shapes = [(h, w, 3) for w, h in self.geoms]
        # the last step's output tensors: in the pipelined modes they are
        # written by the next step or flush(), so they are kept alive until then
        self._held = None

    @staticmethod
    def stream_bytes(geom, params=None) -> int:
        """Device bytes one stream of this geometry adds to a batch (its
        model and its frame scratch)."""
        L = lib()
        p = params or default_params()
        g = Geom(int(geom[0]), int(geom[1]))
        one = int(L.fizi_batch_state_bytes(1, (Geom * 1)(g), (Params * 1)(p)))
        two = int(L.fizi_batch_state_bytes(2, (Geom * 2)(g, g), (Params * 2)(p, p)))
        return two - one

    def learn(self, stream_id, frames: torch.Tensor, reset=True, stream=None):
        w, h = self.geoms[stream_id]
        if frames.dtype != torch.uint8 or not frames.is_contiguous() or tuple(frames.shape[1:]) != (h, w, 3):
            raise FiziError(FIZI_EINVAL, f"frames must be contiguous uint8 (n, {h}, {w}, 3)")
        check(lib().fizi_batch_learn(self._h, int(stream_id), _ptr(frames), int(frames.shape[0]),
                                     int(bool(reset)), _stream(stream)))

    def set_tracking(self, stream_id, enable=True):
        check(lib().fizi_batch_set_tracking(self._h, int(stream_id), int(bool(enable))))

    def relearn(self, stream_id, frames: torch.Tensor, fizi_bits: torch.Tensor, stream=None):
        """Partial re-learning of one stream's model (see Context.relearn_background)."""
        w, h = self.geoms[stream_id]
        n = int(frames.shape[0])
        if frames.dtype != torch.uint8 or not frames.is_contiguous() or tuple(frames.shape[1:]) != (h, w, 3):
            raise FiziError(FIZI_EINVAL, f"frames must be contiguous uint8 (n, {h}, {w}, 3)")
        if fizi_bits.dtype != torch.int64 or not fizi_bits.is_contiguous() or tuple(fizi_bits.shape) != (n, h, w // 64):
            raise FiziError(FIZI_EINVAL, f"masks must be contiguous int64 ({n}, {h}, {w // 64})")
        check(lib().fizi_batch_relearn(self._h, int(stream_id), _ptr(frames), n, _ptr(fizi_bits),
                                       _stream(stream)))

    def _check_step(self, frames, pointers, fizi):
        """The library sees only device addresses: every argument of a step
        is checked against the batch's geometry here, before any is passed.
        Returns the frame address array, every entry set (NULL when idle).
        One pass per frame with cheap attribute tests: a step's host time is
        part of its latency."""
        if len(frames) != self.n:
            raise FiziError(FIZI_EINVAL, f"a step takes {self.n} frame entries, got {len(frames)}")
        arr, u8 = self._frames, torch.uint8
        dev = -1 if self.device.type == "cpu" else self.device.index
        for i, f in enumerate(frames):
            if f is None:
                arr[i] = None
                continue
            if (not isinstance(f, torch.Tensor) or f.dtype is not u8 or f.shape != self._shapes[i]
                    or f.get_device() != dev or not f.is_contiguous()):
                h, w, _ = self._shapes[i]
                raise FiziError(FIZI_EINVAL, f"frame {i} must be a contiguous uint8 ({h}, {w}, 3) "
                                             f"tensor on {self.device}")
            arr[i] = f.data_ptr()
        if (not isinstance(pointers, torch.Tensor) or pointers.dtype != torch.uint8
                or pointers.device != self.device or not pointers.is_contiguous()
                or tuple(pointers.shape) != (self.n, 56)):
            raise FiziError(FIZI_EINVAL, f"pointers must be a contiguous uint8 ({self.n}, 56) tensor "
                                         f"on {self.device}")
        if fizi is not None:
            if len(fizi) != self.n:
                raise FiziError(FIZI_EINVAL, f"a step takes {self.n} mask entries, got {len(fizi)}")
            for i, f in enumerate(fizi):
                if f is None:
                    continue
                w, h = self.geoms[i]
                if (not isinstance(f, torch.Tensor) or f.dtype != torch.int64 or f.device != self.device
                        or not f.is_contiguous() or tuple(f.shape) != (h, w // 64)):
                    raise FiziError(FIZI_EINVAL, f"mask {i} must be a contiguous int64 ({h}, {w // 64}) "
                                                 f"tensor on {self.device}")
        return arr

    def step(self, frames, pointers: torch.Tensor, fizi=None, stream=None):
        """frames: list of n device frames (H, W, 3) uint8 or None (idle);
        pointers: (n, 56) uint8 device tensor; fizi: optional list of n bit
        tensors (H, W/64) int64 (entries may be None)."""
        fr = self._check_step(frames, pointers, fizi)
        fz = None
        if fizi is not None:
            for i in range(self.n):
                f = fizi[i]
                self._fizi[i] = f.data_ptr() if f is not None else None
            fz = self._fizi
        check(lib().fizi_batch_step(self._h, fr, fz, _ptr(pointers), _stream(stream)))
        self._held = (pointers, None if fizi is None else list(fizi))

    def flush(self, stream=None):
        """Enqueues the pending half-step of the pipelined modes (after it
        completes on the stream, every step's outputs are written)."""
        check(lib().fizi_batch_flush(self._h, _stream(stream)))
        self._held = None

    def get_tuning(self) -> dict:
        t = Tuning()
        check(lib().fizi_batch_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning(**{**self.get_tuning(), **kw})
        check(lib().fizi_batch_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, frames, pointers, steps=5, stream=None):
        """Times candidate launch shapes on these frames; keeps the fastest.
        Returns (tuning dict, ms per step)."""
        fr = self._check_step(frames, pointers, None)
        t, ms = Tuning(), ctypes.c_double()
        check(lib().fizi_batch_autotune(self._h, fr, _ptr(pointers), int(steps), _stream(stream),
                                        ctypes.byref(t), ctypes.byref(ms)))
        return t.as_dict(), float(ms.value)

    def set_mode(self, mode: int):
        check(lib().fizi_batch_set_mode(self._h, int(mode)))

    def status(self) -> int:
        f = ctypes.c_uint32()
        check(lib().fizi_batch_status(self._h, ctypes.byref(f)))
        return int(f.value)

    def stage_timing(self, enable=True):
        check(lib().fizi_batch_stage_timing(self._h, int(bool(enable))))

    def stage_times(self) -> dict:
        ms = (ctypes.c_double * 5)()
        n = (ctypes.c_int64 * 5)()
        check(lib().fizi_batch_stage_times(self._h, ms, n))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(Context.STAGES)}

    def model(self, stream_id):
        lay = Layout()
        check(lib().fizi_batch_state_layout(self._h, int(stream_id), ctypes.byref(lay)))
        w, h = self.geoms[stream_id]
        px3 = w * h * 3
        bgmin = self.state[lay.bgmin:lay.bgmin + px3].view(h, w, 3)
        bgmax = self.state[lay.bgmax:lay.bgmax + px3].view(h, w, 3)
        ny = int(lay.yref_rows) * w * 2
        yref = self.state[lay.yref:lay.yref + ny].view(torch.int16).view(int(lay.yref_rows), w)
        return bgmin, bgmax, yref

    def close(self):
        if self._h:
            lib().fizi_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def learn_background(ctx: Context, frames, reset=True, stream=None):
    return ctx.learn_background(frames, reset, stream)


def process_frames(ctx: Context, frames, want_fizi=True, want_hand=False, stream=None):
    return ctx.process_frames(frames, want_fizi, want_hand, stream)


def get_pointer(ctx: Context, frame_index: int) -> dict:
    return ctx.get_pointer(frame_index)


def _host_pointers(pointers) -> np.ndarray:
    """fizi_pointer records as a contiguous host array: a structured array of
    POINTER_DTYPE, or an (n, 56) uint8 tensor (device or host)."""
    if isinstance(pointers, torch.Tensor):
        pointers = pointers_to_numpy(pointers)
    a = np.ascontiguousarray(pointers)
    if a.dtype != POINTER_DTYPE:
        raise TypeError("pointers must have the fizi_pointer layout")
    return a.reshape(-1)


def zone_hit(pointers, zones) -> np.ndarray:
    """Index of the first zone (x0, y0, x1, y1), inclusive, that holds each
    pointer's centroid pixel, or -1 (the Interface module, Section 2)."""
    p = _host_pointers(pointers)
    z = np.ascontiguousarray(np.asarray(zones, dtype=np.int32).reshape(-1, 4))
    out = np.empty(len(p), dtype=np.int32)
    check(lib().fizi_zone_hit(p.ctypes.data, len(p), z.ctypes.data, len(z), out.ctypes.data))
    return out


def drive_of(pointers, wheel) -> np.ndarray:
    """Virtual-wheel driving (Section 4) for each pointer; wheel =
    (cx, cy, r_min, r_max, dead_cdeg, full_cdeg). Returns an (n, 4) int32
    array with columns DRIVE_FIELDS."""
    p = _host_pointers(pointers)
    out = np.empty((len(p), 4), dtype=np.int32)
    w = WheelC(*[int(v) for v in wheel])
    check(lib().fizi_drive_of(p.ctypes.data, len(p), ctypes.byref(w), out.ctypes.data))
    return out


def pack_bits(mask, device=None) -> torch.Tensor:
    """(..., H, W) 0/1 array (W a multiple of 64) -> (..., H, W/64) int64
    LSB-first bit rows, the layout of I_FIZI masks."""
    m = np.ascontiguousarray(np.asarray(mask) != 0)
    b = np.packbits(m, axis=-1, bitorder="little")
    words = np.ascontiguousarray(b).view(np.uint64).view(np.int64)
    t = torch.from_numpy(words.copy())
    return t.to(device) if device is not None else t


def unpack_bits(words: torch.Tensor, width: int) -> np.ndarray:
    """(..., H, W/64) int64 LSB-first bit rows -> (..., H, W) uint8."""
    a = words.detach().cpu().numpy().view(np.uint64)
    b = a.view(np.uint8)   # little-endian: byte k of word j holds pixels 64j + 8k ..
    bits = np.unpackbits(b, axis=-1, bitorder="little")
    return bits[..., :width]
