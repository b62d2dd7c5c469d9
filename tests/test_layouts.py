"""CPU tests of the test-side layout codec and of the f32 mapping."""
import numpy as np

from tests import layouts


def test_bitsliced_roundtrip():
    rng = np.random.default_rng(1)
    for n in (1, 63, 64, 65, 1000):
        bits = rng.integers(0, 2, (n, 37), dtype=np.uint8)
        n_pad = (n + 63) // 64 * 64
        planes = layouts.to_bitsliced(bits, n_pad)
        assert planes.shape == (37, n_pad // 8)
        assert (layouts.from_bitsliced(planes, n) == bits).all()
        # instance i is bit i%8 of byte i/8 of its plane
        i = n - 1
        assert ((planes[:, i // 8] >> (i % 8)) & 1 == bits[i]).all()


def test_rowmajor_word_order():
    bits = np.zeros((2, 64), dtype=np.uint8)
    bits[0, 0] = 1       # first bit -> MSB of word 0
    bits[1, 63] = 1      # last bit -> LSB of word 1
    w = layouts.to_rowmajor_u32(bits)
    assert w[0, 0] == 0x80000000 and w[0, 1] == 0
    assert w[1, 0] == 0 and w[1, 1] == 1


def test_f32_mapping_exhaustive_top24():
    """Every 24-bit value maps to an exact float in [0, 1 - 2^-24], strictly increasing."""
    top = np.arange(1 << 24, dtype=np.uint32)
    f = layouts.u32_to_f32(top << np.uint32(8))
    assert f.dtype == np.float32
    assert f[0] == 0.0 and f[-1] == np.float32(1.0 - 2.0 ** -24)
    assert (np.diff(f.astype(np.float64)) == 2.0 ** -24).all()
    # the low 8 bits never matter
    assert (layouts.u32_to_f32((top << np.uint32(8)) | np.uint32(0xFF)) == f).all()
