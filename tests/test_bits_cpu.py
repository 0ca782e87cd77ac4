"""Host-side bit-mask helpers of the binding (no GPU)."""
import numpy as np

from paper_1907_04393_amd import fizi


def test_pack_unpack_round_trip():
    rng = np.random.default_rng(0)
    m = (rng.random((3, 5, 192)) < 0.4).astype(np.uint8)
    t = fizi.pack_bits(m)
    assert tuple(t.shape) == (3, 5, 3)
    assert np.array_equal(fizi.unpack_bits(t, 192), m)


def test_pack_bit_order():
    m = np.zeros((1, 128), np.uint8)
    m[0, 0] = 1      # bit 0 of word 0
    m[0, 65] = 1     # bit 1 of word 1
    m[0, 127] = 1    # bit 63 of word 1
    w = fizi.pack_bits(m).numpy().view(np.uint64)
    assert int(w[0, 0]) == 1
    assert int(w[0, 1]) == (1 << 1) | (1 << 63)
