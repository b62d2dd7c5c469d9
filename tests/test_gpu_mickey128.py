"""GPU parity of the bitsliced MICKEY-128 2.0 path (mickey128_* in libmickey.so) against
the bit-serial oracle (oracle/mickey128_ref.c), through the ctypes binding.

Every lane of the bitsliced output must equal its scalar instance bit for bit (paper
Sec. IV-D), across several workgroups of 64 slices and a ragged tail of pad instances,
IV lengths 0..128 (with 0, 1, 127 and 128 forced), odd and split generate lengths, and
the register planes after init and after generation; at the benchmark's size, sampled
instances at full length."""
import numpy as np
import pytest
import torch

from oracle import mickey128 as m128
from paper_1909_04750_amd import mickey, synth

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def inputs(seed, n, lengths=True):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    ivs = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    if not lengths:
        return keys, ivs, None
    ivb = rng.integers(0, 129, n, dtype=np.uint8)
    ivb[:4] = [0, 1, 127, 128]
    ivb[-4:] = [128, 127, 1, 0]
    return keys, ivs, ivb


def lane_bits(out, m, nbits, idx=None):
    """[n or len(idx), nbits] keystream bits of instances from bit-planes."""
    planes = out.cpu().numpy().reshape(nbits, m.pitch)
    if idx is not None:
        cols = planes[:, np.asarray(idx) // 8]
        return ((cols >> (np.asarray(idx) % 8).astype(np.uint8)) & 1).T
    return np.unpackbits(planes, axis=1, bitorder="little")[:, :m.n].T


def oracle_bits(keys, ivs, ivb, nbits, skip=0):
    rows = m128.generate_many(keys, ivs, ivb, nbits, skip=skip, threads=8)
    return np.unpackbits(rows, axis=1)[:, :nbits]


def test_ops_per_clock():
    assert mickey.mickey128_ops_per_clock() == 518


@pytest.mark.parametrize("n,nbits", [(2 * 2048 + 300, 777), (37, 64), (2048, 1)])
def test_full_parity_mixed_iv_lengths(n, nbits):
    keys, ivs, ivb = inputs(n + nbits, n)
    m = mickey.Mickey128(to_dev(keys), to_dev(ivs), to_dev(ivb))
    out = m.generate(nbits)
    m.sync()
    got = lane_bits(out, m, nbits)
    m.close()
    want = oracle_bits(keys, ivs, ivb, nbits)
    bad = np.flatnonzero((got != want).any(axis=1))
    assert bad.size == 0, "instances %s differ (iv lengths %s)" % (bad[:8], ivb[bad[:8]])


def test_default_iv_length_is_128():
    n, nbits = 3000, 200
    keys, ivs, _ = inputs(5, n, lengths=False)
    m = mickey.Mickey128(to_dev(keys), to_dev(ivs))
    out = m.generate(nbits)
    m.sync()
    got = lane_bits(out, m, nbits)
    m.close()
    assert (got == oracle_bits(keys, ivs, None, nbits)).all()


def test_split_generation_continues_the_stream():
    n = 2100
    keys, ivs, ivb = inputs(9, n)
    m = mickey.Mickey128(to_dev(keys), to_dev(ivs), to_dev(ivb))
    parts = []
    for nb in (1, 100, 333, 64):
        out = m.generate(nb)
        m.sync()
        parts.append(lane_bits(out, m, nb))
    assert m.bits_generated == 498
    m.close()
    assert (np.concatenate(parts, axis=1) == oracle_bits(keys, ivs, ivb, 498)).all()


def test_register_planes_match_oracle_state():
    n = 2048 + 5
    keys, ivs, ivb = inputs(13, n)
    m = mickey.Mickey128(to_dev(keys), to_dev(ivs), to_dev(ivb))
    after_init = m.export_planes().cpu().numpy().reshape(320, m.pitch)
    m.generate(129)
    after_gen = m.export_planes().cpu().numpy().reshape(320, m.pitch)
    m.sync()
    m.close()
    for planes, skip in ((after_init, 0), (after_gen, 129)):
        bits = np.unpackbits(planes, axis=1, bitorder="little")[:, :n].T  # [n, 320]
        for i in (0, 1, 2, 3, 777, n - 1):
            st = m128.State()
            st.init(keys[i].tobytes(), ivs[i].tobytes(), int(ivb[i]))
            st.generate(skip)
            assert (bits[i] == st.buf).all(), (i, skip)


def test_iv_length_over_128_is_refused():
    keys, ivs, ivb = inputs(17, 64)
    ivb[10] = 129
    with pytest.raises(mickey.MickeyError) as e:
        mickey.Mickey128(to_dev(keys), to_dev(ivs), to_dev(ivb))
    assert e.value.code == mickey.EINVAL


def test_benchmark_size_sampled_full_length():
    """The benchmark's workload (3 * 2^20 instances, 8192 bits) on sampled instances: all
    lanes of the first and last slice and seeded others, full length."""
    seed, n, nbits, _ = synth.workload("mickey128-3m")
    keys, ivs = synth.keys_ivs128(seed, n)
    m = mickey.Mickey128(to_dev(keys), to_dev(ivs))
    out = m.generate(nbits)
    m.sync()
    rng = np.random.default_rng(128)
    idx = np.unique(np.concatenate([np.arange(32), np.arange(n - 32, n), rng.choice(n, 192, replace=False)]))
    got = lane_bits(out, m, nbits, idx)
    m.close()
    del out
    want = oracle_bits(keys[idx], ivs[idx], None, nbits)
    bad = idx[(got != want).any(axis=1)]
    assert bad.size == 0, bad[:8]
