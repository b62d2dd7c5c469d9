"""GPU tests of the served path: resident states resumed by requests, continuous
batching, admission by output budget.  Every returned stream must equal the oracle
continuing that state from where its previous request stopped, and each result must be
the same alone and in the mix."""
import numpy as np
import pytest
import torch

import oracle
from paper_1909_04750_amd import mickey
from tests import layouts

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_pool(seed, n, mixed=True):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivs = rng.integers(0, 256, (n, 10), dtype=np.uint8)
    ivb = rng.integers(0, 81, n, dtype=np.uint8) if mixed else None
    init = mickey.Mickey(to_dev(keys), to_dev(ivs), None if ivb is None else to_dev(ivb))
    return keys, ivs, ivb, init


# (schedule, transpose) of the quantum kernels: the fused one-wave kernel, and the staged
# kernels (bit-planes, then a tiled transpose into the requests) with each schedule
KERNELS = [(mickey.SCHED_ONE_WAVE, mickey.TRANSPOSE_FUSED), (mickey.SCHED_ONE_WAVE, mickey.TRANSPOSE_STAGED),
           (mickey.SCHED_SPLIT, mickey.TRANSPOSE_STAGED), (mickey.SCHED_SPLIT4, mickey.TRANSPOSE_STAGED)]
KERNEL_IDS = ["fused", "staged-one-wave", "staged-split", "staged-split4"]


def server(init, kernel, **kw):
    srv = mickey.Server(init, **kw)
    srv.set_kernel(*kernel)
    return srv


def drain(srv, max_steps=100000):
    done = []
    for _ in range(max_steps):
        st = srv.stats()
        if st["waiting"] == 0 and st["running"] == 0:
            break
        srv.step()
        done += srv.poll().tolist()
    done += srv.poll().tolist()
    return done


def fetch(srv, rid, nbits):
    buf = torch.empty(nbits // 32, dtype=torch.int32, device="cuda")
    srv.copy(rid, buf, nbits // 32)
    return buf.cpu().numpy().view(np.uint32)


def oracle_history(keys, ivs, ivb, sid, lengths):
    """Row-major words of consecutive requests of `lengths` bits on state sid."""
    total = int(sum(lengths))
    rows = oracle.generate_many(keys[sid:sid + 1], ivs[sid:sid + 1], None if ivb is None else ivb[sid:sid + 1], total)
    words = layouts.to_rowmajor_u32(layouts.bits_matrix(rows, total))[0]
    out, w = [], 0
    for nb in lengths:
        out.append(words[w:w + nb // 32])
        w += nb // 32
    return out


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_served_streams_continue_states(kernel):
    keys, ivs, ivb, init = make_pool(1, 300)
    srv = server(init, kernel, nslices=64, quantum_clocks=64, budget_bytes=1 << 20)
    init.close()
    rng = np.random.default_rng(2)
    sids = rng.integers(0, 300, 400)
    sids[:6] = [7, 7, 7, 8, 8, 299]  # several requests on one state
    lengths = 32 * rng.integers(1, 40, 400)
    ids = [srv.submit(int(s), int(nb)) for s, nb in zip(sids, lengths)]
    done = drain(srv)
    assert sorted(done) == sorted(ids)
    hist = {}
    for rid, s, nb in zip(ids, sids, lengths):
        hist.setdefault(int(s), []).append((rid, int(nb)))
    for s in list(hist)[:60] + [7, 8, 299]:
        reqs = hist[s]
        want = oracle_history(keys, ivs, ivb, s, [nb for _, nb in reqs])
        for (rid, nb), w in zip(reqs, want):
            assert (fetch(srv, rid, nb) == w).all(), (s, rid)
        assert srv.state_bits(s) == sum(nb for _, nb in reqs)
    # per-state order: requests on state 7 completed in submission order
    t = [srv.times(r)[2] for r, _ in hist[7]]
    assert t == sorted(t)
    srv.close()


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_request_alone_equals_in_mix(kernel):
    keys, ivs, ivb, init = make_pool(3, 200)
    srv = server(init, kernel, nslices=64, quantum_clocks=96, budget_bytes=1 << 20)
    rng = np.random.default_rng(4)
    sids = rng.permutation(200)[:150]  # first request on each state
    lengths = 32 * rng.integers(1, 60, 150)
    ids = [srv.submit(int(s), int(nb)) for s, nb in zip(sids, lengths)]
    drain(srv)
    mixed = {k: fetch(srv, ids[k], int(lengths[k])) for k in (0, 17, 149)}
    srv.close()
    for k, w in mixed.items():
        alone = server(init, kernel, nslices=64, quantum_clocks=96, budget_bytes=1 << 20)
        rid = alone.submit(int(sids[k]), int(lengths[k]))
        drain(alone)
        assert (fetch(alone, rid, int(lengths[k])) == w).all(), k
        alone.close()
    init.close()


def test_budget_admission_and_overlap():
    keys, ivs, ivb, init = make_pool(5, 100, mixed=False)
    # budget of 2 requests of 4096 bits: the rest wait for space
    srv = mickey.Server(init, nslices=64, quantum_clocks=32, budget_bytes=2 * 4096 // 8)
    init.close()
    first = [srv.submit(s, 4096) for s in range(4)]
    srv.step()
    st = srv.stats()
    assert st["running"] == 2 and st["waiting"] == 2
    # requests arriving while others run are admitted as budget frees up
    for _ in range(2000):
        srv.step()
        for rid in srv.poll().tolist():
            srv.release(rid)
        st = srv.stats()
        if st["running"] + st["waiting"] == 0:
            break
    assert srv.stats()["finished"] == 4
    late = srv.submit(50, 64)
    long = srv.submit(51, 32 * 200)  # 800 bytes: fits next to `later` in the 1 KiB budget
    srv.step()
    later = srv.submit(52, 64)  # arrives while `long` runs
    done = drain(srv)
    assert set(done) >= {late, long, later}
    a_later = srv.times(later)[1]
    assert a_later < srv.times(long)[2]  # admitted before `long` finished: they overlapped
    want = oracle_history(keys, ivs, None, 52, [64])[0]
    assert (fetch(srv, later, 64) == want).all()
    # device time of the quanta: positive, and within the launch-to-retirement time
    st = srv.stats()
    assert 0 < st["gpu_ns"] <= st["quantum_ns"]
    srv.close()


def test_submit_errors_and_2p40_limit():
    keys, ivs, ivb, init = make_pool(6, 10, mixed=False)
    packed, _ = init.export_state()
    init.import_state(packed, mickey.MAX_BITS_PER_IV - 64)
    srv = mickey.Server(init, nslices=64, quantum_clocks=32, budget_bytes=1 << 16)
    init.close()
    with pytest.raises(mickey.MickeyError):
        srv.submit(10, 32)  # no such state
    with pytest.raises(mickey.MickeyError):
        srv.submit(0, 33)
    ok = srv.submit(0, 64)
    over = srv.submit(0, 32)
    drain(srv)
    assert len(fetch(srv, ok, 64)) == 2
    with pytest.raises(mickey.MickeyError) as e:
        srv.times(over)
    assert e.value.code == mickey.ERANGE
    srv.close()


@pytest.mark.parametrize("latency", [False, True], ids=["bit-lanes", "latency-streams"])
@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_chunked_delivery_continues_states_exactly(kernel, latency):
    keys, ivs, ivb, init = make_pool(7, 120)
    # budget 4 KiB: far smaller than several requests below, which stream through it
    srv = server(init, kernel, nslices=64, quantum_clocks=64, budget_bytes=4096)
    if latency:  # what is left of requests of 100+ words takes one of 8 latency streams
        srv.set_latency(8, threshold_bits=32 * 100, clocks_per_quantum=32 * 3)
    init.close()
    rng = np.random.default_rng(8)
    plan = []  # (state, bits, chunk bytes)
    for k in range(150):
        chunk = int(rng.choice([0, 96, 1024]))
        nb = 32 * int(rng.integers(1, 1024 if chunk else 64))
        plan.append((int(rng.integers(0, 120)), nb, chunk))
    plan[:5] = [(3, 32 * 3000, 96), (3, 64, 0), (3, 32 * 2500, 1024), (4, 32 * 8000, 96), (3, 32, 96)]
    ids = []
    for sid, nb, chunk in plan:
        srv.set_chunk(chunk)
        ids.append(srv.submit(sid, nb))
    got = {}
    done = []
    whole = {}
    for _ in range(200000):
        srv.step()
        ch = srv.poll_chunks()
        for c in ch:
            buf = torch.empty(int(c["words"]), dtype=torch.int32, device="cuda")
            srv.copy_chunk(int(c["handle"]), buf, int(c["words"]))
            got.setdefault(int(c["request"]), []).append(
                (int(c["offset"]), int(c["last"]), buf.cpu().numpy().view(np.uint32)))
        if len(ch):
            srv.release_chunks(ch["handle"])
        for rid in srv.poll().tolist():
            done.append(rid)
            sid, nb, chunk = plan[rid]
            if not chunk:
                whole[rid] = fetch(srv, rid, nb)
                srv.release(rid)
        st = srv.stats()
        if st["waiting"] == 0 and st["running"] == 0 and not len(ch):
            break
    assert sorted(done) == sorted(ids)
    assert srv.stats()["free_budget_words"] == 1024  # everything given back
    hist = {}
    for rid, (sid, nb, chunk) in zip(ids, plan):
        hist.setdefault(sid, []).append((rid, nb, chunk))
    for sid in [3, 4] + sorted(hist)[:40]:
        reqs = hist[sid]
        want = oracle_history(keys, ivs, ivb, sid, [nb for _, nb, _ in reqs])
        for (rid, nb, chunk), w in zip(reqs, want):
            if not chunk:
                assert rid not in got
                assert (whole[rid] == w).all(), (sid, rid)
                continue
            parts = sorted(got[rid], key=lambda t: t[0])
            sizes = [len(p[2]) for p in parts]
            assert all(z == chunk // 4 for z in sizes[:-1]) and 0 < sizes[-1] <= chunk // 4, (rid, sizes)
            assert [p[0] for p in parts] == list(np.cumsum([0] + sizes[:-1])), rid
            assert [p[1] for p in parts] == [0] * (len(parts) - 1) + [1], rid
            assert (np.concatenate([p[2] for p in parts]) == w).all(), (sid, rid)
        assert srv.state_bits(sid) == sum(nb for _, nb, _ in reqs)
    # per-state order across whole and chunked requests on state 3
    t = srv.times_many([r for r, _, _ in hist[3]])[:, 2].tolist()
    assert t == sorted(t)
    srv.close()


def test_chunked_delivery_errors():
    keys, ivs, ivb, init = make_pool(9, 4, mixed=False)
    srv = mickey.Server(init, nslices=64, quantum_clocks=32, budget_bytes=1024)
    init.close()
    with pytest.raises(mickey.MickeyError):
        srv.set_chunk(6)  # not whole words
    with pytest.raises(mickey.MickeyError):
        srv.set_chunk(2048)  # larger than the budget
    with pytest.raises(mickey.MickeyError):
        srv.submit(0, 32 * 1024)  # whole delivery: larger than the budget
    srv.set_chunk(256)
    rid = srv.submit(0, 32 * 1024)  # 4 KiB through a 1 KiB budget
    seen = []
    for _ in range(10000):
        srv.step()
        ch = srv.poll_chunks()
        seen += ch.tolist()
        if len(ch):
            srv.release_chunks(ch["handle"])
            with pytest.raises(mickey.MickeyError):
                srv.release_chunks(ch["handle"][:1])  # already given back
        if srv.poll().tolist() == [rid]:
            break
    assert len(seen) == 16
    with pytest.raises(mickey.MickeyError):
        srv.release(rid)  # chunked requests are released chunk by chunk
    with pytest.raises(mickey.MickeyError):
        srv.copy(rid, torch.empty(8, dtype=torch.int32, device="cuda"), 8)
    assert srv.times(rid)[2] > 0
    srv.close()


@pytest.mark.parametrize("schedule", [mickey.SCHED_ONE_WAVE, mickey.SCHED_SPLIT, mickey.SCHED_SPLIT4])
def test_staged_quantum_in_several_launches(schedule):
    """2^17 slices: one 1024-clock launch of planes fills the 512 MiB staging buffer, so a
    quantum of 2144 clocks runs as launches of 1024, 1024 and 96 clocks; requests that end
    inside each launch, and idle slices (their tiles are skipped), between busy ones."""
    keys, ivs, ivb, init = make_pool(10, 300)
    srv = mickey.Server(init, nslices=1 << 17, quantum_clocks=2144, budget_bytes=1 << 22)
    srv.set_kernel(schedule, mickey.TRANSPOSE_STAGED)
    init.close()
    rng = np.random.default_rng(11)
    sids = rng.permutation(300)[:200]
    lengths = 32 * rng.integers(1, 200, 200)
    lengths[:4] = [32 * 32, 32 * 33, 32 * 64, 32 * 67]  # ends at and next to launch edges
    ids = [srv.submit(int(s), int(nb)) for s, nb in zip(sids, lengths)]
    assert sorted(drain(srv)) == sorted(ids)
    for k in list(range(8)) + list(range(190, 200)):
        want = oracle_history(keys, ivs, ivb, int(sids[k]), [int(lengths[k])])[0]
        assert (fetch(srv, ids[k], int(lengths[k])) == want).all(), k
    srv.close()


def test_set_kernel_errors():
    keys, ivs, ivb, init = make_pool(12, 8, mixed=False)
    srv = mickey.Server(init, nslices=64, quantum_clocks=32, budget_bytes=1 << 12)
    init.close()
    for sched, tp in ((4, mickey.TRANSPOSE_AUTO), (mickey.SCHED_AUTO, 3),
                      (mickey.SCHED_SPLIT, mickey.TRANSPOSE_FUSED), (mickey.SCHED_SPLIT4, mickey.TRANSPOSE_FUSED)):
        with pytest.raises(mickey.MickeyError) as e:
            srv.set_kernel(sched, tp)
        assert e.value.code == mickey.EINVAL
    srv.close()


@pytest.mark.parametrize("streams", [5, 4096])
def test_latency_streams_continue_states(streams):
    """Size-aware routing: requests with at least 20 words left run on latency streams
    (5 of them, so many overflow to bit lanes, or 4096, so none do); a state's successive
    requests alternate between the two kinds of lane and must still continue exactly."""
    keys, ivs, ivb, init = make_pool(21, 300)
    srv = mickey.Server(init, nslices=64, quantum_clocks=64, budget_bytes=1 << 22)
    srv.set_latency(streams, threshold_bits=32 * 20, clocks_per_quantum=32 * 5)
    init.close()
    rng = np.random.default_rng(22)
    sids = rng.integers(0, 300, 400)
    sids[:8] = [7, 7, 7, 7, 8, 8, 8, 299]
    lengths = 32 * rng.integers(1, 120, 400)
    lengths[:8] = [32 * 30, 32 * 3, 32 * 45, 32 * 1, 32 * 21, 32 * 20, 32 * 19, 32 * 100]
    ids = [srv.submit(int(s), int(nb)) for s, nb in zip(sids, lengths)]
    assert sorted(drain(srv)) == sorted(ids)
    hist = {}
    for rid, s, nb in zip(ids, sids, lengths):
        hist.setdefault(int(s), []).append((rid, int(nb)))
    for s in list(hist)[:80] + [7, 8, 299]:
        reqs = hist[s]
        want = oracle_history(keys, ivs, ivb, s, [nb for _, nb in reqs])
        for (rid, nb), w in zip(reqs, want):
            assert (fetch(srv, rid, nb) == w).all(), (s, rid)
        assert srv.state_bits(s) == sum(nb for _, nb in reqs)
    t = [srv.times(r)[2] for r, _ in hist[7]]
    assert t == sorted(t)
    srv.close()


def test_set_latency_errors():
    keys, ivs, ivb, init = make_pool(23, 8, mixed=False)
    srv = mickey.Server(init, nslices=64, quantum_clocks=32, budget_bytes=1 << 16)
    init.close()
    L = mickey.load_library()
    assert L.mickey_server_set_latency(srv._h, 16385, 1 << 20, 256) == mickey.EINVAL  # too many streams
    assert L.mickey_server_set_latency(srv._h, 8, 1 << 20, 33) == mickey.EINVAL     # not whole words
    assert L.mickey_server_set_latency(srv._h, 8, 1 << 20, 0) == mickey.EINVAL
    srv.set_latency(8, threshold_bits=64, clocks_per_quantum=64)
    rid = srv.submit(0, 32 * 50)
    srv.step()  # now a latency stream is busy
    assert L.mickey_server_set_latency(srv._h, 0, 0, 0) == mickey.EINVAL
    drain(srv)
    srv.wait()
    srv.set_latency(0)  # off: everything takes bit lanes
    rid2 = srv.submit(0, 32 * 50)
    drain(srv)
    want = oracle_history(keys, ivs, None, 0, [32 * 50, 32 * 50])
    assert (fetch(srv, rid, 32 * 50) == want[0]).all() and (fetch(srv, rid2, 32 * 50) == want[1]).all()
    srv.close()
