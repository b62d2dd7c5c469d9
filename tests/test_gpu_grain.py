"""GPU parity of the bitsliced Grain path (include/grain.h) against the Grain oracle, bit
for bit: the specification's known-answer vectors, ragged instance counts and clock
counts that exercise every loop of the kernels, row-major u32/f32 delivery, split
generation, state export/import, errors, and sampled instances of the 2^22-instance
workload the benchmark times."""
import numpy as np
import pytest
import torch

from oracle import grain as oracle_grain
from paper_1909_04750_amd import mickey, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def random_inputs(seed, n):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, (n, 10), dtype=np.uint8), rng.integers(0, 256, (n, 8), dtype=np.uint8)


def oracle_bits(keys, ivs, nbits, skip=0):
    """[n, nbits] keystream bits (oracle bytes are least significant bit first)."""
    rows = oracle_grain.generate_many(keys, ivs, nbits, skip=skip, threads=8)
    return np.unpackbits(rows, axis=1, bitorder="little")[:, :nbits]


def planes_to_bits(out, nbits, pitch, n):
    planes = out.cpu().numpy().reshape(nbits, pitch)
    return np.unpackbits(planes, axis=1, bitorder="little")[:, :n].T


def rowmajor_words(bits):
    """[n, nbits] -> uint32 [n, nbits/32]: bit b of word j is bit 32j + b."""
    n, nbits = bits.shape
    b = bits.reshape(n, nbits // 32, 32).astype(np.uint64)
    return (b << np.arange(32, dtype=np.uint64)).sum(axis=2).astype(np.uint32)


def test_known_answer_vectors_on_gpu():
    from tests.test_grain_oracle_pins import load_kats
    kats = load_kats()
    n = 70  # the vectors plus padding instances, across two 64-instance blocks
    keys, ivs = random_inputs(1, n)
    for i, (k, v, _) in enumerate(kats):
        keys[i] = np.frombuffer(k, dtype=np.uint8)
        ivs[i] = np.frombuffer(v, dtype=np.uint8)
        keys[66 + i] = keys[i]
        ivs[66 + i] = ivs[i]
    g = mickey.Grain(to_dev(keys), to_dev(ivs))
    bits = planes_to_bits(g.generate(80), 80, g.pitch, n)
    for i, (_, _, ks) in enumerate(kats):
        want = np.unpackbits(np.frombuffer(ks, dtype=np.uint8), bitorder="little")
        assert (bits[i] == want).all(), i
        assert (bits[66 + i] == want).all(), i
    g.close()


@pytest.mark.parametrize("n,nbits", [(1, 1), (33, 79), (100, 160), (1000, 1000), (2049, 257)])
def test_ragged_sizes_full_parity(n, nbits):
    """Instance counts off the 32/64 grid and clock counts that hit the two-ring loop,
    the single leftover ring and the shifting tail."""
    keys, ivs = random_inputs(n + nbits, n)
    g = mickey.Grain(to_dev(keys), to_dev(ivs))
    got = planes_to_bits(g.generate(nbits), nbits, g.pitch, n)
    assert (got == oracle_bits(keys, ivs, nbits)).all()
    assert g.bits_generated == nbits
    g.close()


def test_lane_position_invariance():
    keys, ivs = random_inputs(3, 256)
    perm = np.random.default_rng(4).permutation(256)
    a = mickey.Grain(to_dev(keys), to_dev(ivs))
    b = mickey.Grain(to_dev(keys[perm]), to_dev(ivs[perm]))
    ba = planes_to_bits(a.generate(300), 300, a.pitch, 256)
    bb = planes_to_bits(b.generate(300), 300, b.pitch, 256)
    assert (bb == ba[perm]).all()
    a.close()
    b.close()


def test_split_generation_continues_streams():
    n = 300
    keys, ivs = random_inputs(5, n)
    g = mickey.Grain(to_dev(keys), to_dev(ivs))
    parts = [planes_to_bits(g.generate(k), k, g.pitch, n) for k in (160, 37, 80, 3, 240)]
    assert (np.concatenate(parts, axis=1) == oracle_bits(keys, ivs, 520)).all()
    assert g.bits_generated == 520
    g.close()


@pytest.mark.parametrize("n,nbits", [(64, 32), (77, 32 * 17), (200, 32 * 10)])
def test_rowmajor_u32_f32(n, nbits):
    keys, ivs = random_inputs(6 + n, n)
    g = mickey.Grain(to_dev(keys), to_dev(ivs))
    g.generate(13)  # start at an offset that is not a ring boundary
    u, f = g.generate_rowmajor(nbits)
    want = rowmajor_words(oracle_bits(keys, ivs, nbits, skip=13))
    assert (u.cpu().numpy().view(np.uint32) == want).all()
    wf = ((want >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
    assert f.cpu().numpy().tobytes() == wf.tobytes()
    u2 = g.generate(64, mickey.ROWMAJOR_U32)  # and the stream continues from there
    want2 = rowmajor_words(oracle_bits(keys, ivs, 64, skip=13 + nbits))
    assert (u2.cpu().numpy().view(np.uint32) == want2).all()
    g.close()


def test_state_export_matches_oracle_and_resumes():
    n = 90
    keys, ivs = random_inputs(7, n)
    g = mickey.Grain(to_dev(keys), to_dev(ivs))
    g.generate(123)
    packed, bits = g.export_state()
    assert bits == 123
    pk = packed.cpu().numpy()
    for i in (0, 31, 32, 89):
        st = oracle_grain.State()
        st.init(keys[i].tobytes(), ivs[i].tobytes())
        st.generate(123)
        assert pk[i].tobytes() == st.packed(), i
    # resume in another state object created from unrelated keys
    k2, v2 = random_inputs(8, n)
    h = mickey.Grain(to_dev(k2), to_dev(v2))
    h.import_state(packed, bits)
    got = planes_to_bits(h.generate(200), 200, h.pitch, n)
    assert (got == oracle_bits(keys, ivs, 200, skip=123)).all()
    assert h.bits_generated == 323
    g.close()
    h.close()


def test_rekey_resets_streams():
    n = 50
    keys, ivs = random_inputs(9, n)
    k2, v2 = random_inputs(10, n)
    g = mickey.Grain(to_dev(keys), to_dev(ivs))
    g.generate(100)
    g.rekey(to_dev(k2), to_dev(v2))
    assert g.bits_generated == 0
    assert (planes_to_bits(g.generate(96), 96, g.pitch, n) == oracle_bits(k2, v2, 96)).all()
    g.close()


def test_error_paths():
    keys, ivs = random_inputs(11, 8)
    g = mickey.Grain(to_dev(keys), to_dev(ivs))
    with pytest.raises(mickey.MickeyError):
        g.generate(33, mickey.ROWMAJOR_U32, torch.empty(64, dtype=torch.int32, device=DEV))
    buf = torch.empty(64, dtype=torch.int32, device=DEV)
    assert mickey.load_library().grain_generate(g._h, 32, buf.data_ptr(), 7) == mickey.EINVAL
    assert g.bits_generated == 0  # failed calls change nothing
    big = torch.zeros(8 * 8 + 4, dtype=torch.uint8, device=DEV)
    with pytest.raises(mickey.MickeyError):
        mickey.Grain(to_dev(keys), big[4:])  # IVs not 8-byte aligned
    g.close()


def test_grain_4m_sampled_parity():
    """2^22 instances, 8192 bits, bitsliced: the launch configuration the benchmark
    times.  All lanes of the first and last slice plus seeded random instances."""
    seed, n, nbits, _ = synth.workload("grain-4m")
    keys, ivs = synth.grain_keys_ivs(seed, n)
    g = mickey.Grain(to_dev(keys), to_dev(ivs))
    out = g.generate(nbits)
    rng = np.random.default_rng(6)
    idx = np.unique(np.concatenate([np.arange(32), np.arange(n - 32, n), rng.choice(n, 320, replace=False)]))
    planes = out.view(nbits, g.pitch)
    sel = planes[:, torch.from_numpy(idx // 8).to(DEV)]
    got = ((sel >> torch.from_numpy(idx % 8).to(DEV).to(torch.uint8)) & 1).T.cpu().numpy()
    assert (got == oracle_bits(keys[idx], ivs[idx], nbits)).all()
    g.close()
