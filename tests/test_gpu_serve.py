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


def test_served_streams_continue_states():
    keys, ivs, ivb, init = make_pool(1, 300)
    srv = mickey.Server(init, nslices=64, quantum_clocks=64, budget_bytes=1 << 20)
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


def test_request_alone_equals_in_mix():
    keys, ivs, ivb, init = make_pool(3, 200)
    srv = mickey.Server(init, nslices=64, quantum_clocks=96, budget_bytes=1 << 20)
    rng = np.random.default_rng(4)
    sids = rng.permutation(200)[:150]  # first request on each state
    lengths = 32 * rng.integers(1, 60, 150)
    ids = [srv.submit(int(s), int(nb)) for s, nb in zip(sids, lengths)]
    drain(srv)
    mixed = {k: fetch(srv, ids[k], int(lengths[k])) for k in (0, 17, 149)}
    srv.close()
    for k, w in mixed.items():
        alone = mickey.Server(init, nslices=64, quantum_clocks=96, budget_bytes=1 << 20)
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
