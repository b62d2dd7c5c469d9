"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, bit for bit.

Every instance of the bitsliced generator must produce exactly the MICKEY 2.0 keystream
of its own key/IV (the paper's Sec. IV-D packs independent instances into bit lanes;
the output of each lane is the scalar cipher's).  The bar is bit-exact equality."""
import numpy as np
import pytest
import torch

import oracle
from paper_1909_04750_amd import mickey, synth
from tests import layouts

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def make(keys, ivs, ivb=None):
    return mickey.Mickey(to_dev(keys), to_dev(ivs), None if ivb is None else to_dev(ivb))


SCHEDULES = [mickey.SCHED_ONE_WAVE, mickey.SCHED_SPLIT, mickey.SCHED_SPLIT4]


def gpu_bitsliced(keys, ivs, ivb, nbits, word_bits=32, schedule=mickey.SCHED_AUTO):
    m = make(keys, ivs, ivb)
    if word_bits != 32:
        m.set_word_bits(word_bits)
    m.set_schedule(schedule)
    out = m.generate(nbits)
    torch.cuda.synchronize()
    planes = out.cpu().numpy().reshape(nbits, m.pitch)
    m.close()
    return planes


def oracle_bits(keys, ivs, ivb, nbits, skip=0):
    rows = oracle.generate_many(keys, ivs, ivb, nbits, skip=skip, threads=8)
    return layouts.bits_matrix(rows, nbits)


def random_inputs(seed, n, mixed=True):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivs = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivb = rng.integers(0, 81, n, dtype=np.uint8) if mixed else None
    if mixed:
        ivb[: min(n, 4)] = [0, 1, 79, 80][: min(n, 4)]
    return keys, ivs, ivb


def test_gpu_available():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    mickey.load_library()


def test_known_answer_vectors_on_gpu():
    from tests.test_oracle_pins import load_kats
    kats = load_kats()
    keys = np.zeros((len(kats), 10), dtype=np.uint8)
    ivs = np.zeros((len(kats), 10), dtype=np.uint8)
    ivb = np.zeros(len(kats), dtype=np.uint8)
    for i, (k, v, L, _) in enumerate(kats):
        keys[i] = np.frombuffer(k, dtype=np.uint8)
        ivs[i, : len(v)] = np.frombuffer(v, dtype=np.uint8)
        ivb[i] = L
    nbits = 128
    got = layouts.from_bitsliced(gpu_bitsliced(keys, ivs, ivb, nbits), len(kats))
    for i, (_, _, _, ks) in enumerate(kats):
        want = np.unpackbits(np.frombuffer(ks, dtype=np.uint8))
        assert (got[i, : want.size] == want).all(), i


def test_plain_1k_full_parity():
    """1024 instances (32 slices x 32 lanes), 80-bit IVs from splitmix64(seed 1), 4096
    keystream bits each, bitsliced layout: every bit against the oracle."""
    seed, n, nbits, _ = synth.workload("plain-1k")
    keys, ivs = synth.keys_ivs(seed, n)
    planes = gpu_bitsliced(keys, ivs, None, nbits)
    want = layouts.to_bitsliced(oracle_bits(keys, ivs, None, nbits), 1024)
    assert planes.shape == want.shape
    bad = np.nonzero(planes != want)
    assert bad[0].size == 0, "first mismatch at plane %d byte %d" % (bad[0][0], bad[1][0])


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("n,nbits", [(1, 1), (1, 37), (63, 130), (65, 257), (1000, 1003), (2113, 64)])
def test_ragged_sizes_mixed_iv_lengths(n, nbits, schedule):
    """Instance counts that leave lanes past the last slice (in the split schedule they
    run a copy of another slice) and clock counts off the unrolled loop."""
    keys, ivs, ivb = random_inputs(n * 7 + nbits, n)
    got = layouts.from_bitsliced(gpu_bitsliced(keys, ivs, ivb, nbits, schedule=schedule), n)
    want = oracle_bits(keys, ivs, ivb, nbits)
    assert (got == want).all()


def test_pad_lanes_run_zero_key():
    n = 5
    keys, ivs, _ = random_inputs(3, n, mixed=False)
    planes = gpu_bitsliced(keys, ivs, None, 96)
    pad = layouts.from_bitsliced(planes, 64)[n:]
    zero = oracle_bits(np.zeros((1, 10), np.uint8), np.zeros((1, 10), np.uint8), None, 96)[0]
    assert (pad == zero[None, :]).all()


def test_lane_position_invariance():
    """An instance's stream does not depend on which lane or slice carries it."""
    n = 256
    keys, ivs, ivb = random_inputs(21, n)
    perm = np.random.default_rng(5).permutation(n)
    a = layouts.from_bitsliced(gpu_bitsliced(keys, ivs, ivb, 200), n)
    b = layouts.from_bitsliced(gpu_bitsliced(keys[perm], ivs[perm], ivb[perm], 200), n)
    assert (b == a[perm]).all()


def test_word64_matches_word32_bytes():
    n = 4096 + 64
    keys, ivs, _ = random_inputs(8, n, mixed=False)
    a = gpu_bitsliced(keys, ivs, None, 515, word_bits=32)
    b = gpu_bitsliced(keys, ivs, None, 515, word_bits=64)
    assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_split_generation_and_counter(schedule):
    n = 300
    keys, ivs, ivb = random_inputs(4, n)
    m = make(keys, ivs, ivb)
    m.set_schedule(schedule)
    parts = [m.generate(nb) for nb in (1, 31, 100, 500)]
    torch.cuda.synchronize()
    assert m.bits_generated == 632
    got = np.concatenate([layouts.from_bitsliced(p.cpu().numpy().reshape(-1, m.pitch), n) for p in parts], axis=1)
    m.close()
    assert (got == oracle_bits(keys, ivs, ivb, 632)).all()


def test_state_export_matches_oracle_and_resumes():
    n = 130
    keys, ivs, ivb = random_inputs(12, n)
    m = make(keys, ivs, ivb)
    m.generate(77)
    packed, bits = m.export_state()
    torch.cuda.synchronize()
    assert bits == 77
    packed = packed.cpu().numpy()
    for i in range(0, n, 13):
        st = oracle.State()
        st.init(keys[i].tobytes(), ivs[i].tobytes(), int(ivb[i]))
        st.generate(77)
        assert packed[i].tobytes() == st.packed(), i
    # a second state with different keys resumes from the exported registers
    k2, v2, _ = random_inputs(99, n, mixed=False)
    m2 = make(k2, v2)
    m2.import_state(to_dev(packed), bits)
    out = m2.generate(64)
    torch.cuda.synchronize()
    assert m2.bits_generated == 77 + 64
    got = layouts.from_bitsliced(out.cpu().numpy().reshape(64, m2.pitch), n)
    assert (got == oracle_bits(keys, ivs, ivb, 64, skip=77)).all()
    m.close()
    m2.close()


@pytest.mark.parametrize("n,nbits", [(1, 32), (70, 96), (700, 1024)])
@pytest.mark.parametrize("transpose", [mickey.TRANSPOSE_FUSED, mickey.TRANSPOSE_STAGED])
@pytest.mark.parametrize("schedule", SCHEDULES)
def test_rowmajor_u32_f32(n, nbits, schedule, transpose):
    keys, ivs, ivb = random_inputs(n + 1, n)
    m = make(keys, ivs, ivb)
    m.set_schedule(schedule)
    m.set_transpose(transpose)
    u, f = m.generate_rowmajor(nbits)
    torch.cuda.synchronize()
    want = layouts.to_rowmajor_u32(oracle_bits(keys, ivs, ivb, nbits))
    got_u = u.cpu().numpy().view(np.uint32)
    assert (got_u == want).all()
    got_f = f.cpu().numpy()
    assert got_f.tobytes() == layouts.u32_to_f32(want).tobytes()
    # single-form layouts through mickey_generate, continuing the stream
    u2 = m.generate(64, mickey.ROWMAJOR_U32)
    f2 = m.generate(64, mickey.ROWMAJOR_F32)
    torch.cuda.synchronize()
    nxt = layouts.to_rowmajor_u32(oracle_bits(keys, ivs, ivb, 128, skip=nbits))
    assert (u2.cpu().numpy().view(np.uint32) == nxt[:, :2]).all()
    assert f2.cpu().numpy().tobytes() == layouts.u32_to_f32(nxt[:, 2:]).tobytes()
    m.close()


def test_staged_rowmajor_chunks_and_tiles():
    """The staged path across several chunk-buffer loads (the buffer holds up to 8192
    clocks here), a partial last transpose tile, a partial last slice tile (instance
    counts off 512), and a later call that needs a larger buffer than the first."""
    n = 600
    keys, ivs, ivb = random_inputs(77, n)
    m = make(keys, ivs, ivb)
    m.set_transpose(mickey.TRANSPOSE_STAGED)
    u1 = m.generate(96, mickey.ROWMAJOR_U32)                # buffer sized for one tile
    u2, f2 = m.generate_rowmajor(8192 + 1024 + 96)          # grows it; two chunk loads
    u3 = m.generate(2048 + 32, mickey.ROWMAJOR_U32)
    torch.cuda.synchronize()
    total = 96 + 9312 + 2080
    want = layouts.to_rowmajor_u32(oracle_bits(keys, ivs, ivb, total))
    assert (u1.cpu().numpy().view(np.uint32) == want[:, :3]).all()
    assert (u2.cpu().numpy().view(np.uint32) == want[:, 3:3 + 291]).all()
    assert f2.cpu().numpy().tobytes() == layouts.u32_to_f32(want[:, 3:3 + 291]).tobytes()
    assert (u3.cpu().numpy().view(np.uint32) == want[:, 294:]).all()
    assert m.bits_generated == total
    m.close()


def test_error_paths():
    keys, ivs, _ = random_inputs(1, 64, mixed=False)
    bad = np.full(64, 80, dtype=np.uint8)
    bad[17] = 81
    with pytest.raises(mickey.MickeyError) as e:
        make(keys, ivs, bad)
    assert e.value.code == mickey.EINVAL
    m = make(keys, ivs)
    with pytest.raises(mickey.MickeyError) as e:
        m.generate(0)
    assert e.value.code == mickey.EINVAL
    with pytest.raises(mickey.MickeyError) as e:
        m.generate(33, mickey.ROWMAJOR_U32)
    assert e.value.code == mickey.EINVAL
    with pytest.raises(mickey.MickeyError) as e:
        m.set_word_bits(16)
    assert e.value.code == mickey.ENOSYS
    with pytest.raises(mickey.MickeyError) as e:
        m.set_schedule(4)
    assert e.value.code == mickey.EINVAL
    with pytest.raises(mickey.MickeyError) as e:
        m.set_transpose(3)
    assert e.value.code == mickey.EINVAL
    m.set_schedule(mickey.SCHED_SPLIT)  # the split schedule keeps 32-bit words
    with pytest.raises(mickey.MickeyError) as e:
        m.set_word_bits(64)
    assert e.value.code == mickey.EINVAL
    m.set_schedule(mickey.SCHED_AUTO)
    m.set_word_bits(64)
    with pytest.raises(mickey.MickeyError) as e:
        m.set_schedule(mickey.SCHED_SPLIT)
    assert e.value.code == mickey.EINVAL
    m.set_word_bits(32)
    # the 2^40-bit budget per key/IV pair
    packed, _ = m.export_state()
    m.import_state(packed, mickey.MAX_BITS_PER_IV - 32)
    m.generate(32)
    with pytest.raises(mickey.MickeyError) as e:
        m.generate(1)
    assert e.value.code == mickey.ERANGE
    assert m.bits_generated == mickey.MAX_BITS_PER_IV
    m.close()


def sample_indices(n, k, seed):
    rng = np.random.default_rng(seed)
    idx = np.concatenate([np.arange(32), np.arange(n - 32, n), rng.choice(n, k - 64, replace=False)])
    return np.unique(idx)


def test_plain_4m_sampled_parity():
    """2^22 instances, 8192 bits, bitsliced, the launch configuration the benchmark times:
    all lanes of the first and last slice plus seeded random instances against the oracle;
    word widths 32 and 64 and the split schedules must give identical bytes."""
    seed, n, nbits, _ = synth.workload("plain-4m")
    keys, ivs = synth.keys_ivs(seed, n)
    m = make(keys, ivs)
    out = m.generate(nbits)
    idx = sample_indices(n, 384, 2)
    planes = out.view(nbits, m.pitch)
    sel = planes[:, torch.from_numpy(idx // 8).to(DEV)]
    got = ((sel >> torch.from_numpy(idx % 8).to(DEV).to(torch.uint8)) & 1).T.cpu().numpy()
    want = oracle_bits(keys[idx], ivs[idx], None, nbits)
    assert (got == want).all()
    m2 = make(keys, ivs)
    m2.set_word_bits(64)
    out2 = m2.generate(nbits)
    assert torch.equal(out, out2)
    m2.close()
    for sched in (mickey.SCHED_SPLIT, mickey.SCHED_SPLIT4):
        m3 = make(keys, ivs)
        m3.set_schedule(sched)
        out3 = m3.generate(nbits)
        assert torch.equal(out, out3), sched
        m3.close()
        del out3
    m.close()


def test_rowmajor_1m_sampled_parity():
    """2^20 instances, IV lengths in {0,32,64,80}, 65536 bits each, row-major u32 + f32:
    sampled instances at full length against the oracle."""
    seed, n, nbits, _ = synth.workload("rowmajor-1m")
    keys, ivs, ivb = synth.workload_inputs("rowmajor-1m")
    m = make(keys, ivs, ivb)
    u, f = m.generate_rowmajor(nbits)
    idx = sample_indices(n, 96, 3)
    ti = torch.from_numpy(idx).to(DEV)
    got_u = u[ti].cpu().numpy().view(np.uint32)
    got_f = f[ti].cpu().numpy()
    want = layouts.to_rowmajor_u32(oracle_bits(keys[idx], ivs[idx], ivb[idx], nbits))
    assert (got_u == want).all()
    assert got_f.tobytes() == layouts.u32_to_f32(want).tobytes()
    m.close()
    # the other schedule, and the fused transpose, give the same bytes for every instance
    m2 = make(keys, ivs, ivb)
    m2.set_schedule(mickey.SCHED_ONE_WAVE)
    m2.set_transpose(mickey.TRANSPOSE_FUSED)
    u2 = m2.generate(nbits, mickey.ROWMAJOR_U32)
    assert torch.equal(u, u2)
    m2.close()


@pytest.mark.parametrize("n", [64 * 33, 64 * 1024 + 96])
def test_schedules_agree_across_launch_shapes(n):
    """Every schedule, every instance, a few hundred clocks: one call per layout and
    a clock count that ends off the unrolled loop, at block counts that leave a
    partial last workgroup (lanes past the last slice)."""
    keys, ivs, ivb = random_inputs(n, n)
    outs = []
    for sched in SCHEDULES:
        m = make(keys, ivs, ivb)
        m.set_schedule(sched)
        a = m.generate(203)
        b = m.generate(96, mickey.ROWMAJOR_U32)
        exp, bits = m.export_state()
        outs.append((a, b, exp, bits))
        m.close()
    a0, b0, e0, n0 = outs[0]
    for a1, b1, e1, n1 in outs[1:]:
        assert torch.equal(a0, a1) and torch.equal(b0, b1) and torch.equal(e0, e1) and n0 == n1 == 299
    idx = sample_indices(n, 96, 9)
    want = oracle_bits(keys[idx], ivs[idx], ivb[idx], 299)
    ti = torch.from_numpy(idx).to(DEV)
    got = layouts.from_bitsliced(a0.view(203, -1).cpu().numpy(), n)[idx]
    assert (got == want[:, :203]).all()
    assert (b0[ti].cpu().numpy().view(np.uint32) == layouts.to_rowmajor_u32(want[:, 203:])).all()


def test_rekey_reuses_state():
    n = 200
    keys, ivs, ivb = random_inputs(31, n)
    k2, v2, b2 = random_inputs(32, n)
    m = make(keys, ivs, ivb)
    m.generate(64)
    m.rekey(to_dev(k2), to_dev(v2), to_dev(b2))
    assert m.bits_generated == 0
    out = m.generate(100)
    torch.cuda.synchronize()
    got = layouts.from_bitsliced(out.cpu().numpy().reshape(100, m.pitch), n)
    assert (got == oracle_bits(k2, v2, b2, 100)).all()
    m.close()
