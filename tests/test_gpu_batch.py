"""GPU parity of the batched path: many fresh requests of uneven keystream and IV
lengths in one persistent, graph-captured launch, each bit-exact against the oracle and
identical alone and in the mix."""
import numpy as np
import pytest
import torch

import oracle
from paper_1909_04750_amd import mickey, synth
from tests import layouts

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def random_requests(seed, n, max_words):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivs = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivb = rng.integers(0, 81, n, dtype=np.uint8)
    nbits = 32 * rng.integers(0, max_words + 1, n).astype(np.uint64)
    return keys, ivs, ivb, nbits


def arena_for(nbits):
    words = (np.asarray(nbits, dtype=np.uint64) // 32).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(words)])
    arena = torch.zeros(int(max(offs[-1], 1)), dtype=torch.int32, device="cuda")
    ptrs = [arena.data_ptr() + 4 * int(o) for o in offs[:-1]]
    return arena, offs, ptrs


def run_batch(keys, ivs, ivb, nbits, params=None, batch=None):
    b = batch or mickey.Batch(len(nbits))
    arena, offs, ptrs = arena_for(nbits)
    dk, dv = to_dev(keys), to_dev(ivs)
    db = None if ivb is None else to_dev(ivb)
    b.set(dk, dv, db, nbits, ptrs)
    if params:
        b.set_params(*params)
    torch.cuda.synchronize()
    b.run()
    b.sync()
    words = arena.cpu().numpy().view(np.uint32)
    return [words[offs[i]:offs[i + 1]] for i in range(len(nbits))], b


def oracle_words(keys, ivs, ivb, nbits):
    out = []
    for i in range(len(nbits)):
        nb = int(nbits[i])
        if nb == 0:
            out.append(np.zeros(0, dtype=np.uint32))
            continue
        rows = oracle.generate_many(keys[i:i + 1], ivs[i:i + 1], None if ivb is None else ivb[i:i + 1], nb)
        out.append(layouts.to_rowmajor_u32(layouts.bits_matrix(rows, nb))[0])
    return out


def test_batch_matches_oracle_uneven_lengths():
    keys, ivs, ivb, nbits = random_requests(1, 300, 96)
    nbits[:3] = [0, 32, 96 * 32]
    got, b = run_batch(keys, ivs, ivb, nbits)
    want = oracle_words(keys, ivs, ivb, nbits)
    for i in range(len(nbits)):
        assert (got[i] == want[i]).all(), i
    b.close()


def test_request_alone_equals_in_mix():
    keys, ivs, ivb, nbits = random_requests(2, 2100, 40)  # more than one task of 2048 requests
    got, b = run_batch(keys, ivs, ivb, nbits)
    b.close()
    for i in (0, 5, 777, 2099):
        alone, b1 = run_batch(keys[i:i + 1], ivs[i:i + 1], ivb[i:i + 1], nbits[i:i + 1])
        b1.close()
        assert (alone[0] == got[i]).all(), i
    sample = [0, 1, 63, 64, 2047, 2048, 2099]
    want = oracle_words(keys[sample], ivs[sample], ivb[sample], nbits[sample])
    for k, i in enumerate(sample):
        assert (got[i] == want[k]).all(), i


def test_all_kernel_variants_agree():
    keys, ivs, ivb, nbits = random_requests(3, 200, 20)
    ref = None
    for u in (2, 4, 8):
        for w in (1, 2, 4):
            got, b = run_batch(keys, ivs, ivb, nbits, params=(u, w))
            assert b.get_params() == (u, w)
            b.close()
            flat = np.concatenate(got)
            if ref is None:
                ref = flat
                want = np.concatenate(oracle_words(keys, ivs, ivb, nbits))
                assert (ref == want).all()
            assert (flat == ref).all(), (u, w)


def test_graph_replays_with_eager_work_between():
    keys, ivs, ivb, nbits = random_requests(4, 150, 30)
    want = np.concatenate(oracle_words(keys, ivs, ivb, nbits))
    b = mickey.Batch(150)
    arena, offs, ptrs = arena_for(nbits)
    b.set(to_dev(keys), to_dev(ivs), to_dev(ivb), nbits, ptrs)
    k2, v2, _, _ = random_requests(5, 64, 1)
    for rep in range(4):
        arena.zero_()
        torch.cuda.synchronize()
        b.run()
        b.sync()
        assert (arena.cpu().numpy().view(np.uint32)[: len(want)] == want).all(), rep
        # eager work of the program between replays
        m = mickey.Mickey(to_dev(k2), to_dev(v2))
        m.generate(64 * (rep + 1))
        x = torch.arange(1 << 16, device="cuda", dtype=torch.float32).sum()
        torch.cuda.synchronize()
        m.close()
        assert float(x) > 0
    b.close()


def test_autotune_and_cache(tmp_path):
    keys, ivs, ivb, nbits = random_requests(6, 100, 50)
    want = np.concatenate(oracle_words(keys, ivs, ivb, nbits))
    b = mickey.Batch(100)
    arena, offs, ptrs = arena_for(nbits)
    b.set(to_dev(keys), to_dev(ivs), to_dev(ivb), nbits, ptrs)
    cache = tmp_path / "batch_tune.json"
    params = b.autotune(256, cache)
    assert params[0] in (2, 4, 8) and params[1] in (1, 2, 4)
    text = cache.read_text()
    assert '"unroll": %d' % params[0] in text and "timings_ms" in text
    b.run()
    b.sync()
    assert (arena.cpu().numpy().view(np.uint32)[: len(want)] == want).all()
    b.close()
    b2 = mickey.Batch(100)
    b2.set(to_dev(keys), to_dev(ivs), to_dev(ivb), nbits, ptrs)
    assert b2.autotune(256, cache) == params  # read back from the cache
    b2.close()


def test_batch_errors():
    keys, ivs, ivb, nbits = random_requests(7, 10, 4)
    b = mickey.Batch(10)
    arena, offs, ptrs = arena_for(nbits)
    bad = nbits.copy()
    bad[3] = 33
    with pytest.raises(mickey.MickeyError) as e:
        b.set(to_dev(keys), to_dev(ivs), to_dev(ivb), bad, ptrs)
    assert e.value.code == mickey.EINVAL
    badl = ivb.copy()
    badl[2] = 81
    with pytest.raises(mickey.MickeyError) as e:
        b.set(to_dev(keys), to_dev(ivs), to_dev(badl), nbits, ptrs)
    assert e.value.code == mickey.EINVAL
    with pytest.raises(mickey.MickeyError) as e:
        b.run()  # nothing set yet
    assert e.value.code == mickey.EINVAL
    big = np.zeros((11, 10), dtype=np.uint8)
    with pytest.raises(mickey.MickeyError):
        b.set(to_dev(big), to_dev(big), None, np.zeros(11, np.uint64), [0] * 11)
    b.close()


def test_batch_10k_recipe_capped_sampled_parity():
    """The 10,000-request batched workload (seed 4) with lengths log-uniform up to 2^16
    bits instead of 2^24 (same recipe, shorter tail) in one launch; sampled requests
    against the oracle."""
    keys, ivs, ivb, nbits = synth.batch_requests(4, 10000, max_log2=16.0)
    got, b = run_batch(keys, ivs, ivb, nbits)
    b.close()
    rng = np.random.default_rng(9)
    order = np.argsort(-nbits.astype(np.int64), kind="stable")
    sample = np.unique(np.concatenate([order[:8], order[-8:], rng.choice(10000, 48, replace=False)]))
    want = oracle_words(keys[sample], ivs[sample], ivb[sample], nbits[sample])
    for k, i in enumerate(sample):
        assert (got[i] == want[k]).all(), int(i)


def test_latency_mode_matches_bitsliced_and_oracle():
    keys, ivs, ivb, nbits = random_requests(8, 260, 120)
    nbits[:4] = [0, 32, 120 * 32, 64]
    b = mickey.Batch(len(nbits))
    arena, offs, ptrs = arena_for(nbits)
    b.set(to_dev(keys), to_dev(ivs), to_dev(ivb), nbits, ptrs)
    outs = {}
    for th in (mickey.Batch.LATENCY_OFF, 1, 32 * 60, 0):
        b.set_latency_threshold(th)
        arena.zero_()
        torch.cuda.synchronize()
        b.run()
        b.sync()
        outs[th] = arena.cpu().numpy().view(np.uint32).copy()
        t, nlat, ratio = b.routing()
        if th == mickey.Batch.LATENCY_OFF:
            assert t is None and nlat == 0
        elif th == 1:
            assert nlat == int((nbits > 0).sum())  # every non-empty request in latency mode
        elif th == 32 * 60:
            assert nlat == int((nbits >= th).sum()) and 0 < nlat < len(nbits)
    for th, o in outs.items():
        assert (o == outs[mickey.Batch.LATENCY_OFF]).all(), th
    want = np.concatenate(oracle_words(keys, ivs, ivb, nbits))
    assert (outs[1][: len(want)] == want).all()
    b.close()


def test_batch_10k_full_lengths_sampled_parity():
    """The batched workload at its configured lengths (seed 4: 10,000 requests, log-uniform
    up to 2^24 bits, IV lengths 0..80), one launch with size-aware routing: the 8 longest
    requests (latency mode) and 24 seeded others against the oracle, full length."""
    keys, ivs, ivb, nbits = synth.batch_requests(4, 10000)
    arena, offs, ptrs = arena_for(nbits)
    b = mickey.Batch(len(nbits))
    b.set(to_dev(keys), to_dev(ivs), to_dev(ivb), nbits, ptrs)
    b.run()
    b.sync()
    threshold, nlat, _ = b.routing()
    b.close()
    order = np.argsort(-nbits.astype(np.int64), kind="stable")
    rng = np.random.default_rng(9)
    pick = np.concatenate([order[:8], rng.choice(order[8:], 24, replace=False)])
    assert nlat > 0 and all(int(nbits[i]) >= threshold for i in order[:8])
    from concurrent.futures import ThreadPoolExecutor

    def want(i):  # one instance per job: ctypes releases the GIL while the oracle runs
        return oracle.generate_many(keys[i:i + 1], ivs[i:i + 1], ivb[i:i + 1], int(nbits[i]))[0].tobytes()
    with ThreadPoolExecutor(8) as pool:
        wants = list(pool.map(want, pick))
    for i, wb in zip(pick, wants):
        w = int(nbits[i]) // 32
        got = arena[int(offs[i]):int(offs[i]) + w].cpu().numpy().view(np.uint32)
        assert got.astype(">u4").tobytes() == wb, (int(i), int(nbits[i]))
