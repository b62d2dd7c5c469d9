"""GPU tests of the C-ABI's state contract, through the ctypes binding:

- mickey_generate_batch: per-instance requests on an existing state (the paper's
  Sec. IV-D problem statement of independent instances), applied in array order per
  instance, bit-exact against the oracle continuing each instance's stream;
- a failed call leaves the registers and bit counters unchanged: a refused IV length in a
  re-key, and launch failures injected from the host (mickey_debug_fail_launch) in the
  middle of multi-launch calls;
- the host form of a state (mickey_state_export_host / _import_host) resumes exactly.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1909_04750_amd import mickey
from tests import layouts

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def inputs(seed, n):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivs = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivb = rng.integers(0, 81, n, dtype=np.uint8)
    ivb[:4] = [0, 1, 79, 80]
    return keys, ivs, ivb


def oracle_words(keys, ivs, ivb, idx, skip, nbits):
    """Row-major words of instances idx, from keystream bit `skip` on, nbits each."""
    rows = oracle.generate_many(keys[idx], ivs[idx], None if ivb is None else ivb[idx], nbits, skip=skip,
                                threads=8)
    return layouts.to_rowmajor_u32(layouts.bits_matrix(rows, nbits))


def stream_of(keys, ivs, ivb, i, skip, nbits):
    return oracle_words(keys, ivs, ivb, np.array([i]), skip, nbits)[0]


def run_requests(m, inst, nbits, layouts_):
    outs = [torch.zeros(max(int(b) // 32, 1), dtype=torch.int32, device="cuda") for b in nbits]
    m.generate_batch(inst, nbits, outs, layouts_)
    m.sync()
    return [o.cpu().numpy().view(np.uint32)[: int(b) // 32] for o, b in zip(outs, nbits)]


def check_requests(keys, ivs, ivb, base, inst, nbits, lays, got):
    """Every request against the oracle: instance i's requests follow each other in array
    order from its offset base[i]."""
    pos = dict(base)
    by_inst = {}
    for k, i in enumerate(inst):
        by_inst.setdefault(int(i), []).append(k)
    for i, ks in by_inst.items():
        total = int(sum(int(nbits[k]) for k in ks))
        if total == 0:
            continue
        want = stream_of(keys, ivs, ivb, i, pos[i], total)
        off = 0
        for k in ks:
            w = int(nbits[k]) // 32
            exp = want[off:off + w]
            if lays[k] == mickey.ROWMAJOR_U32:
                assert (got[k] == exp).all(), (k, i)
            else:
                assert got[k].view(np.float32).tobytes() == layouts.u32_to_f32(exp).tobytes(), (k, i)
            off += w
        pos[i] += total
    return pos


def test_generate_batch_matches_oracle_in_array_order():
    n = 3000
    keys, ivs, ivb = inputs(11, n)
    m = mickey.Mickey(to_dev(keys), to_dev(ivs), to_dev(ivb))
    m.generate(64, mickey.ROWMAJOR_U32)  # every instance at bit 64
    rng = np.random.default_rng(3)
    nreq = 700
    inst = rng.integers(0, n, nreq)
    inst[:6] = [5, 5, 5, 2999, 0, 5]  # repeated instances, first and last
    nbits = 32 * rng.integers(0, 128, nreq)
    nbits[:6] = [32, 0, 4096, 32 * 1000, 64, 96]
    long = rng.choice(nreq, 6, replace=False)  # latency-mode tasks (>= 2^14 bits)
    nbits[long] = 32 * rng.integers(1 << 9, 1 << 11, 6)
    lays = np.where(rng.random(nreq) < 0.3, mickey.ROWMAJOR_F32, mickey.ROWMAJOR_U32).astype(np.int32)
    got = run_requests(m, inst, nbits, lays)
    base = {i: 64 for i in range(n)}
    pos = check_requests(keys, ivs, ivb, base, inst, nbits, lays, got)
    for i in (5, 0, 2999, int(inst[long[0]]), 1):
        assert m.instance_bits(i) == pos[i], i
    assert m.bits_generated == 64
    # a second batch continues, then a whole-state generate moves every instance on from
    # where it stands
    inst2 = np.array([5, 1, 5, 7])
    nbits2 = np.array([64, 32, 32, 128])
    lays2 = np.full(4, mickey.ROWMAJOR_U32, dtype=np.int32)
    got2 = run_requests(m, inst2, nbits2, lays2)
    pos = check_requests(keys, ivs, ivb, pos, inst2, nbits2, lays2, got2)
    out = m.generate(96, mickey.ROWMAJOR_U32)
    torch.cuda.synchronize()
    words = out.cpu().numpy().view(np.uint32)
    for i in (0, 1, 5, 7, 2999, int(inst[long[1]]), 1234):
        assert (words[i] == stream_of(keys, ivs, ivb, i, pos[i], 96)).all(), i
    m.close()


def test_generate_batch_errors_leave_state_unchanged():
    n = 128
    keys, ivs, ivb = inputs(12, n)
    m = mickey.Mickey(to_dev(keys), to_dev(ivs), to_dev(ivb))
    buf = torch.zeros(64, dtype=torch.int32, device="cuda")
    cases = [
        (([n], [32], [buf]), mickey.EINVAL),                     # instance out of range
        (([1], [33], [buf]), mickey.EINVAL),                     # not whole words
        (([1], [32], [0]), mickey.EINVAL),                       # NULL output
    ]
    for (i_, b_, o_), code in cases:
        with pytest.raises(mickey.MickeyError) as e:
            m.generate_batch(i_, b_, o_)
        assert e.value.code == code
    with pytest.raises(mickey.MickeyError) as e:
        m.generate_batch([1], [32], [buf], mickey.BITSLICED)
    assert e.value.code == mickey.EINVAL
    # the 2^40 budget of one instance
    packed, _ = m.export_state()
    m.import_state(packed, mickey.MAX_BITS_PER_IV - 64)
    m.generate_batch([3], [64], [buf])
    with pytest.raises(mickey.MickeyError) as e:
        m.generate_batch([3, 4], [32, 32], [buf, buf])
    assert e.value.code == mickey.ERANGE
    assert m.instance_bits(3) == mickey.MAX_BITS_PER_IV and m.instance_bits(4) == mickey.MAX_BITS_PER_IV - 64
    with pytest.raises(mickey.MickeyError) as e:  # a whole-state call would take instance 3 past the limit
        m.generate(32)
    assert e.value.code == mickey.ERANGE
    m.close()


def test_rekey_with_a_refused_iv_length_keeps_the_old_state():
    n = 200
    keys, ivs, ivb = inputs(13, n)
    m = mickey.Mickey(to_dev(keys), to_dev(ivs), to_dev(ivb))
    m.generate(64, mickey.ROWMAJOR_U32)
    k2, v2, b2 = inputs(14, n)
    b2[77] = 81
    with pytest.raises(mickey.MickeyError) as e:
        m.rekey(to_dev(k2), to_dev(v2), to_dev(b2))
    assert e.value.code == mickey.EINVAL
    assert m.bits_generated == 64
    out = m.generate(128, mickey.ROWMAJOR_U32)
    torch.cuda.synchronize()
    want = oracle_words(keys, ivs, ivb, np.arange(n), 64, 128)
    assert (out.cpu().numpy().view(np.uint32) == want).all()
    m.close()


@pytest.mark.parametrize("fail_at", [1, 2, 3, 4, 5])
def test_injected_failure_in_staged_rowmajor_generate(fail_at):
    """A staged row-major call (snapshot, then generate / transpose per chunk) with the
    fail_at-th launch failing: the call reports MICKEY_EDEVICE, and the counter and the
    registers are those from before it."""
    n, nbits = 192, 3 * 8192  # three 8192-clock chunks
    keys, ivs, ivb = inputs(15, n)
    m = mickey.Mickey(to_dev(keys), to_dev(ivs), to_dev(ivb))
    m.set_transpose(mickey.TRANSPOSE_STAGED)
    m.generate(32, mickey.ROWMAJOR_U32)
    u = torch.empty((n, nbits // 32), dtype=torch.int32, device="cuda")
    mickey.debug_fail_launch(fail_at)
    try:
        with pytest.raises(mickey.MickeyError) as e:
            m.generate_rowmajor(nbits, u, None, want_f32=False)
    finally:
        mickey.debug_fail_launch(0)
    assert e.value.code == mickey.EDEVICE and "injected" in str(e.value)
    assert m.bits_generated == 32
    out = m.generate(256, mickey.ROWMAJOR_U32)
    torch.cuda.synchronize()
    want = oracle_words(keys, ivs, ivb, np.arange(n), 32, 256)
    assert (out.cpu().numpy().view(np.uint32) == want).all()
    m.close()


@pytest.mark.parametrize("fail_at", [1, 2, 3, 4])
def test_injected_failure_in_generate_batch(fail_at):
    """Launches of a batch with both kinds of task: pack, latency, bitsliced, scatter."""
    n = 100
    keys, ivs, ivb = inputs(16, n)
    m = mickey.Mickey(to_dev(keys), to_dev(ivs), to_dev(ivb))
    inst = [3, 9, 3]
    nbits = [1 << 15, 64, 96]
    outs = [torch.zeros(b // 32, dtype=torch.int32, device="cuda") for b in nbits]
    mickey.debug_fail_launch(fail_at)
    try:
        with pytest.raises(mickey.MickeyError) as e:
            m.generate_batch(inst, nbits, outs)
    finally:
        mickey.debug_fail_launch(0)
    assert e.value.code == mickey.EDEVICE
    assert m.instance_bits(3) == 0 and m.instance_bits(9) == 0
    got = run_requests(m, inst, nbits, [mickey.ROWMAJOR_U32] * 3)
    check_requests(keys, ivs, ivb, {i: 0 for i in range(n)}, inst, nbits, [mickey.ROWMAJOR_U32] * 3, got)
    m.close()


def test_injected_failure_in_plain_generate_and_rekey():
    n = 64
    keys, ivs, ivb = inputs(17, n)
    m = mickey.Mickey(to_dev(keys), to_dev(ivs), to_dev(ivb))
    m.generate(32)
    mickey.debug_fail_launch(1)
    with pytest.raises(mickey.MickeyError) as e:
        m.generate(64)
    assert e.value.code == mickey.EDEVICE and m.bits_generated == 32
    k2, v2, b2 = inputs(18, n)
    mickey.debug_fail_launch(2)  # the staging runs, the initialisation launch fails
    with pytest.raises(mickey.MickeyError) as e:
        m.rekey(to_dev(k2), to_dev(v2), to_dev(b2))
    mickey.debug_fail_launch(0)
    assert e.value.code == mickey.EDEVICE and m.bits_generated == 32
    out = m.generate(64, mickey.ROWMAJOR_U32)
    torch.cuda.synchronize()
    assert (out.cpu().numpy().view(np.uint32) == oracle_words(keys, ivs, ivb, np.arange(n), 32, 64)).all()
    m.close()


def test_host_export_import_resumes_exactly():
    n = 500
    keys, ivs, ivb = inputs(19, n)
    m = mickey.Mickey(to_dev(keys), to_dev(ivs), to_dev(ivb))
    m.generate(96, mickey.ROWMAJOR_U32)
    run_requests(m, [4, 4, 400], [64, 32, 1 << 15], [mickey.ROWMAJOR_U32] * 3)
    blob = m.export_host()
    assert len(blob) == 32 + 33 * n and blob[:8] == b"MICKEY2\0"
    counters = np.frombuffer(blob[32 + 25 * n:], dtype="<u8")
    assert counters[4] == 192 and counters[400] == 96 + (1 << 15) and counters[0] == 96
    # the packed registers are the oracle's state after that many clocks
    st = oracle.State()
    st.init(bytes(keys[4]), bytes(ivs[4]), int(ivb[4]))
    st.generate(192)
    assert blob[32 + 25 * 4: 32 + 25 * 5] == st.packed()
    k2, v2, b2 = inputs(20, n)
    m2 = mickey.Mickey(to_dev(k2), to_dev(v2), to_dev(b2))
    bad = bytearray(blob)
    bad[0] ^= 1
    for b, code in ((bytes(bad), mickey.EINVAL), (blob[:-1], mickey.EINVAL)):
        with pytest.raises(mickey.MickeyError) as e:
            m2.import_host(b)
        assert e.value.code == code
    big = bytearray(blob)
    big[32 + 25 * n: 32 + 25 * n + 8] = ((1 << 40) + 1).to_bytes(8, "little")
    with pytest.raises(mickey.MickeyError) as e:
        m2.import_host(bytes(big))
    assert e.value.code == mickey.ERANGE
    assert m2.bits_generated == 0
    m2.import_host(blob)
    assert m2.instance_bits(400) == 96 + (1 << 15) and m2.instance_bits(4) == 192
    a = m.generate(128, mickey.ROWMAJOR_U32)
    b = m2.generate(128, mickey.ROWMAJOR_U32)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    small = mickey.Mickey(to_dev(keys[:10]), to_dev(ivs[:10]), to_dev(ivb[:10]))
    with pytest.raises(mickey.MickeyError) as e:
        small.import_host(blob)
    assert e.value.code == mickey.EINVAL
    small.close()
    m.close()
    m2.close()
