"""GPU parity of the bitsliced AES-128 counter-mode path (include/aes.h) against the AES
oracle, bit for bit: the standards' example vectors reproduced through the counter
layout, ragged stream counts, row-major u32/f32 delivery, continuation and seeking,
errors, and sampled streams of the 2^22-stream workload the benchmark times."""
import numpy as np
import pytest
import torch

from oracle import aes as oracle_aes
from paper_1909_04750_amd import mickey, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def counter_blocks(nonces, j0):
    """Initial counter blocks nonce_i || j0 (64-bit big-endian)."""
    low = np.array([j0], dtype=">u8").view(np.uint8)
    return np.concatenate([nonces, np.tile(low, (nonces.shape[0], 1))], axis=1)


def oracle_bits(key, nonces, j0, nblocks):
    ks = oracle_aes.ctr_many(bytes(key), counter_blocks(nonces, j0), nblocks, threads=8)
    return np.unpackbits(ks, axis=1)  # most significant bit first


def planes_to_bits(out, nbits, pitch, n):
    planes = out.cpu().numpy().reshape(nbits, pitch)
    return np.unpackbits(planes, axis=1, bitorder="little")[:, :n].T


def rowmajor_words(bits):
    n, nbits = bits.shape
    b = bits.reshape(n, nbits // 32, 32).astype(np.uint64)
    return (b << np.arange(31, -1, -1, dtype=np.uint64)).sum(axis=2).astype(np.uint32)


def random_inputs(seed, n):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, 16, dtype=np.uint8), rng.integers(0, 256, (n, 8), dtype=np.uint8)


def test_standard_vectors_through_the_counter_layout():
    from tests.test_aes_oracle_pins import load_kats
    blocks, ctrs = load_kats()
    # FIPS-197 C.1: the plaintext block is read as nonce || counter
    f = blocks[1]
    nonces = np.zeros((40, 8), dtype=np.uint8)
    nonces[5] = np.frombuffer(f["in"][:8], dtype=np.uint8)
    a = mickey.AesCtr(to_dev(np.frombuffer(f["key"], dtype=np.uint8).copy()), to_dev(nonces))
    a.seek(int.from_bytes(f["in"][8:], "big"))
    bits = planes_to_bits(a.generate(128), 128, a.pitch, 40)
    assert np.packbits(bits[5]).tobytes() == f["out"]
    a.close()
    # SP 800-38A F.5.1: four consecutive counter blocks from f0f1...fe ff
    c = ctrs[0]
    nonces = np.tile(np.frombuffer(c["t1"][:8], dtype=np.uint8), (3, 1))
    a = mickey.AesCtr(to_dev(np.frombuffer(c["key"], dtype=np.uint8).copy()), to_dev(nonces))
    a.seek(int.from_bytes(c["t1"][8:], "big"))
    u = a.generate(512, mickey.ROWMAJOR_U32)
    got = u.cpu().numpy().view(np.uint32).astype(">u4").tobytes()[:64]
    assert got == b"".join(c["o%d" % j] for j in range(1, 5))
    a.close()


@pytest.mark.parametrize("n,nblocks", [(1, 1), (33, 3), (100, 2), (2049, 1)])
def test_ragged_sizes_full_parity(n, nblocks):
    key, nonces = random_inputs(n + nblocks, n)
    a = mickey.AesCtr(to_dev(key), to_dev(nonces))
    got = planes_to_bits(a.generate(128 * nblocks), 128 * nblocks, a.pitch, n)
    assert (got == oracle_bits(key, nonces, 0, nblocks)).all()
    assert a.bits_generated == 128 * nblocks
    a.close()


def test_continuation_and_seek():
    n = 70
    key, nonces = random_inputs(3, n)
    a = mickey.AesCtr(to_dev(key), to_dev(nonces))
    parts = [planes_to_bits(a.generate(128 * k), 128 * k, a.pitch, n) for k in (1, 2)]
    assert (np.concatenate(parts, axis=1) == oracle_bits(key, nonces, 0, 3)).all()
    a.seek((1 << 64) - 3)  # the counter's last two usable blocks (it must stay below 2^64 - 1)
    assert (planes_to_bits(a.generate(256), 256, a.pitch, n) == oracle_bits(key, nonces, (1 << 64) - 3, 2)).all()
    with pytest.raises(mickey.MickeyError) as e:
        a.generate(128)  # would move the 64-bit block counter to 2^64 - 1
    assert e.value.code == mickey.ERANGE
    a.close()


@pytest.mark.parametrize("n,nblocks", [(64, 1), (77, 3)])
def test_rowmajor_u32_f32(n, nblocks):
    key, nonces = random_inputs(5 + n, n)
    a = mickey.AesCtr(to_dev(key), to_dev(nonces))
    a.seek(12345)
    u, f = a.generate_rowmajor(128 * nblocks)
    want = rowmajor_words(oracle_bits(key, nonces, 12345, nblocks))
    assert (u.cpu().numpy().view(np.uint32) == want).all()
    wf = ((want >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
    assert f.cpu().numpy().tobytes() == wf.tobytes()
    a.close()


def test_error_paths():
    key, nonces = random_inputs(7, 8)
    a = mickey.AesCtr(to_dev(key), to_dev(nonces))
    with pytest.raises(mickey.MickeyError):
        a.generate(64)  # not whole blocks
    buf = torch.empty(64, dtype=torch.int32, device=DEV)
    assert mickey.load_library().aes_ctr_generate(a._h, 128, buf.data_ptr(), 9) == mickey.EINVAL
    assert a.bits_generated == 0
    big = torch.zeros(8 * 8 + 4, dtype=torch.uint8, device=DEV)
    with pytest.raises(mickey.MickeyError):
        mickey.AesCtr(to_dev(key), big[4:].view(8, 8))  # nonces not 8-byte aligned
    a.close()


def test_aes_4m_sampled_parity():
    """2^22 streams, 8192 bits (64 blocks), bitsliced: the configuration the benchmark
    times.  All lanes of the first and last slice plus seeded random streams."""
    seed, n, nbits, _ = synth.workload("aes-4m")
    key, nonces = synth.aes_inputs(seed, n)
    a = mickey.AesCtr(to_dev(key), to_dev(nonces))
    out = a.generate(nbits)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([np.arange(32), np.arange(n - 32, n), rng.choice(n, 192, replace=False)]))
    planes = out.view(nbits, a.pitch)
    sel = planes[:, torch.from_numpy(idx // 8).to(DEV)]
    got = ((sel >> torch.from_numpy(idx % 8).to(DEV).to(torch.uint8)) & 1).T.cpu().numpy()
    assert (got == oracle_bits(key, nonces[idx], 0, nbits // 128)).all()
    a.close()
