"""The Python binding checks a batch step's arguments against the batch's
geometry before any device address reaches the library (the library cannot
see tensor shapes): wrong counts, shapes, dtypes, devices and layouts are
errors, and every entry of the reusable address arrays is set on each call."""
import pytest
import torch

from paper_1907_04393_amd import fizi


def _batch(geoms):
    """A Batch whose arguments can be checked without a GPU (no library
    object is created; the checks run before any library call)."""
    b = fizi.Batch.__new__(fizi.Batch)
    b.n = len(geoms)
    b.geoms = list(geoms)
    b.device = torch.device("cpu")
    b._h = None
    import ctypes
    b._frames = (ctypes.c_void_p * b.n)()
    b._fizi = (ctypes.c_void_p * b.n)()
    b._shapes = [(h, w, 3) for w, h in b.geoms]
    return b


GEOMS = [(64, 8), (128, 4)]


def _good():
    frames = [torch.zeros((8, 64, 3), dtype=torch.uint8), torch.zeros((4, 128, 3), dtype=torch.uint8)]
    ptrs = torch.zeros((2, 56), dtype=torch.uint8)
    fz = [torch.zeros((8, 1), dtype=torch.int64), torch.zeros((4, 2), dtype=torch.int64)]
    return frames, ptrs, fz


def test_good_arguments_pass():
    b = _batch(GEOMS)
    frames, ptrs, fz = _good()
    b._check_step(frames, ptrs, fz)
    b._check_step([None, frames[1]], ptrs, [None, None])


@pytest.mark.parametrize("case", ["short_frames", "long_frames", "wrong_shape", "wrong_dtype",
                                  "not_contiguous", "pointers_shape", "pointers_dtype", "short_fizi",
                                  "fizi_shape", "fizi_dtype"])
def test_bad_arguments_raise(case):
    b = _batch(GEOMS)
    frames, ptrs, fz = _good()
    if case == "short_frames":
        frames = frames[:1]
    elif case == "long_frames":
        frames = frames + [None]
    elif case == "wrong_shape":
        frames[0] = torch.zeros((8, 128, 3), dtype=torch.uint8)
    elif case == "wrong_dtype":
        frames[1] = torch.zeros((4, 128, 3), dtype=torch.int16)
    elif case == "not_contiguous":
        frames[0] = torch.zeros((64, 8, 3), dtype=torch.uint8).transpose(0, 1)
    elif case == "pointers_shape":
        ptrs = torch.zeros((1, 56), dtype=torch.uint8)
    elif case == "pointers_dtype":
        ptrs = torch.zeros((2, 14), dtype=torch.int32)
    elif case == "short_fizi":
        fz = fz[:1]
    elif case == "fizi_shape":
        fz[1] = torch.zeros((4, 1), dtype=torch.int64)
    elif case == "fizi_dtype":
        fz[0] = torch.zeros((8, 2), dtype=torch.int32)
    with pytest.raises(fizi.FiziError) as e:
        b.step(frames, ptrs, fizi=fz)
    assert e.value.code == fizi.FIZI_EINVAL


def test_every_entry_is_rewritten():
    """An idle stream's entry is NULL even when the previous step gave it a
    frame (no stale address survives from one step to the next)."""
    b = _batch(GEOMS)
    frames, ptrs, _ = _good()
    arr = b._check_step(frames, ptrs, None)
    assert arr[0] and arr[1]
    arr = b._check_step([None, frames[1]], ptrs, None)
    assert arr[0] is None and arr[1] == frames[1].data_ptr()
