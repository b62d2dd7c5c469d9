#!/usr/bin/env python3
"""Benchmark: bitsliced MICKEY 2.0 keystream generation on one MI355X.

One step = the whole hot path over one batch: input staging and initialisation of
2^22 instances (80-bit keys and IVs from splitmix64 seed 2, already resident in HBM),
then 8192 keystream clocks per instance with the bit-plane store of every clock and the
state write-back.  Prints one JSON line (value = keystream Gbit/s of the whole step).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-word64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "keystream Gbit/s on 1 MI355X (bit-exact vs oracle); served p50/p99 latency"
WORKLOAD = "plain-4m"
# 32-bit VALU lane-ops: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.64 T/s (the published fp32
# vector peak, 157.3 TFLOP/s, counted as 2 flops per FMA lane-op)
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


HEADLINE_SYMBOL = "_ZN12_GLOBAL__N_120gen_bitsliced_kernelILi1EEEvPjjjmS1_"  # gen_bitsliced_kernel<1>


def kernel_code_hash() -> str:
    """Hash of the headline kernel's machine code in the built library."""
    from paper_1909_04750_amd import codeobj
    from paper_1909_04750_amd.build import LIB_PATH
    return codeobj.kernel_code_hash(LIB_PATH, HEADLINE_SYMBOL) or "missing"


def traffic_record(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the kernel's current machine code; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, WORKLOAD))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("code_hash") != kernel_code_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def oracle_threads() -> int:
    """Host threads the oracle may use: the CPUs this process may run on, at most 16 (the
    host's share for one GPU)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - non-Linux
        avail = os.cpu_count() or 1
    return max(1, min(avail, 16))


class OracleRuns:
    """cpu_baseline leg: the oracle (plain bit-serial C) run on host threads beside the GPU
    legs, one instance per job, from its initialisation.  Its outputs also check sampled
    GPU results of the batched and served configurations bit for bit; its thread time gives
    the oracle's rate on those configurations."""

    def __init__(self, threads: int):
        import threading
        from concurrent.futures import ThreadPoolExecutor
        import oracle
        self.oracle = oracle
        self.threads = threads
        self.pool = ThreadPoolExecutor(max_workers=threads)
        self.lock = threading.Lock()
        self.stats = {}  # tag -> [jobs, bits, thread seconds]

    def stream(self, tag: str, key, iv, iv_bits, nbits: int):
        """Future of instance (key, iv, iv_bits)'s first nbits keystream bits (MSB-first bytes)."""
        def job():
            t0 = time.perf_counter()
            rows = self.oracle.generate_many(key[None, :], iv[None, :],
                                             None if iv_bits is None else np.array([iv_bits], dtype=np.uint8),
                                             int(nbits))
            dt = time.perf_counter() - t0
            with self.lock:
                st = self.stats.setdefault(tag, [0, 0, 0.0])
                st[0] += 1
                st[1] += int(nbits)
                st[2] += dt
            return rows[0].tobytes()
        return self.pool.submit(job)

    def rate(self, tag: str):
        jobs, bits, ts = self.stats.get(tag, [0, 0, 0.0])
        return {"instances": jobs, "bits": bits, "thread_s": round(ts, 2),
                "gbit_s_per_core": round(bits / ts / 1e9, 6) if ts else None}

    def close(self):
        self.pool.shutdown(wait=True)


def warm_up(torch, fn, seconds: float = 0.5):
    """Run fn until `seconds` of wall time have passed (at least twice), so that a leg is
    timed at the engine clock the device settles at under that kernel, not at the clock
    it idled at before."""
    t0 = time.perf_counter()
    k = 0
    while k < 2 or time.perf_counter() - t0 < seconds:
        fn()
        torch.cuda.synchronize()
        k += 1


def words_be_bytes(words: np.ndarray) -> bytes:
    """Row-major words as the oracle's MSB-first byte stream (bit 31-b of word j is bit
    32j+b, so a word's big-endian bytes are 4 consecutive stream bytes)."""
    return np.ascontiguousarray(words, dtype=np.uint32).astype(">u4").tobytes()


def cpu_baseline(keys, ivs, nbits, gpu_sample_bits, sample_idx, threads):
    """The oracle (plain bit-serial C) on a bounded sample of the same workload."""
    import oracle
    k, v = keys[sample_idx], ivs[sample_idx]
    t0 = time.perf_counter()
    rows = oracle.generate_many(k, v, None, nbits, threads=threads)
    dt = time.perf_counter() - t0
    bits = np.unpackbits(rows, axis=1)[:, :nbits]
    match = bool((bits == gpu_sample_bits).all())
    return {
        "value": round(len(sample_idx) * nbits / dt / 1e9, 6),
        "unit": "Gbit/s",
        "cores": threads,
        "host_cores": os.cpu_count(),
        "kind": "oracle",
        "sample": "%d of the %d instances (init + %d keystream bits each), %.1f s wall on %d threads "
                  "(the host's CPU share for one GPU; os.cpu_count() gives the machine's)"
                  % (len(sample_idx), keys.shape[0], nbits, dt, threads),
        "sample_bit_exact_vs_gpu": match,
    }


def cpu_baseline_c1(torch, mickey, synth, threads):
    """The small configuration in full: 1024 instances x 4096 bits on the GPU (bit-planes)
    and on the oracle, compared bit for bit, with the oracle's time."""
    import oracle
    seed, n, nbits, _ = synth.workload("plain-1k")
    keys, ivs = synth.keys_ivs(seed, n)
    m = mickey.Mickey(torch.from_numpy(keys).cuda(), torch.from_numpy(ivs).cuda())
    out = m.generate(nbits)
    torch.cuda.synchronize()
    planes = out.cpu().numpy().reshape(nbits, m.pitch)
    m.close()
    got = np.unpackbits(planes, axis=1, bitorder="little")[:, :n].T
    t0 = time.perf_counter()
    rows = oracle.generate_many(keys, ivs, None, nbits, threads=threads)
    dt = time.perf_counter() - t0
    want = np.unpackbits(rows, axis=1)[:, :nbits]
    return {"workload": "plain-1k: 1024 instances (seed 1), full init, 4096 bits each", "instances": n,
            "bits": n * nbits, "oracle_s": round(dt, 3), "gbit_s": round(n * nbits / dt / 1e9, 6),
            "threads": threads, "bit_exact_vs_gpu": bool((got == want).all())}


def bench_rowmajor(torch, mickey, synth, reps: int = 3):
    """2^20 instances, IV lengths in {0,32,64,80}, 65536 bits each, transposed to
    row-major u32 plus exact f32 (16 GiB of output).  2^20 instances are 512 waves at 32
    instances per lane, a quarter of the device's two-per-SIMD wave slots: the default
    (automatic) schedule splits each slice over four waves (halves of R and S), and the
    row-major words come from bit-plane chunks through a tiled transpose.  The two-wave
    split and the fused in-kernel transpose are timed beside it."""
    seed, n, nbits, _ = synth.workload("rowmajor-1m")
    keys, ivs, ivb = synth.workload_inputs("rowmajor-1m")
    dk, dv, db = (torch.from_numpy(a).cuda() for a in (keys, ivs, ivb))
    stream = torch.cuda.current_stream()
    u = torch.empty((n, nbits // 32), dtype=torch.int32, device="cuda")
    f = torch.empty((n, nbits // 32), dtype=torch.float32, device="cuda")
    bits = n * nbits
    res = {"workload": "2^20 instances, IV lengths {0,32,64,80}, 65536 bits each, row-major u32 + f32"}
    legs = (("auto", mickey.SCHED_AUTO, mickey.TRANSPOSE_AUTO),
            ("split2_staged", mickey.SCHED_SPLIT, mickey.TRANSPOSE_STAGED),
            ("split2_fused", mickey.SCHED_SPLIT, mickey.TRANSPOSE_FUSED),
            ("one_wave_fused", mickey.SCHED_ONE_WAVE, mickey.TRANSPOSE_FUSED))
    for name, sched, tp in legs:
        m = mickey.Mickey(dk, dv, db, stream=stream)
        m.set_schedule(sched)
        m.set_transpose(tp)
        m.generate_rowmajor(nbits, u, f)  # warm-up
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        t_init, t_gen = [], []
        for _ in range(reps):
            ev[0].record(stream)
            m.rekey(dk, dv, db)
            ev[1].record(stream)
            m.generate_rowmajor(nbits, u, f)
            ev[2].record(stream)
            torch.cuda.synchronize()
            t_init.append(ev[0].elapsed_time(ev[1]))
            t_gen.append(ev[1].elapsed_time(ev[2]))
        m.close()
        ti, tg = float(np.mean(t_init)), float(np.mean(t_gen))
        ops = mickey.ops_per_clock() * (n // 32) * nbits
        print("# rowmajor-1m %s: init %.3f ms, generate %.3f ms" % (name, ti, tg), file=sys.stderr, flush=True)
        leg = {"gbit_s": round(bits / ((ti + tg) * 1e-3) / 1e9, 3), "init_ms": round(ti, 4),
               "generate_ms": round(tg, 4), "generate_gbit_s": round(bits / (tg * 1e-3) / 1e9, 3),
               "valu_frac": round(ops / (tg * 1e-3) / (VALU_PEAK_TOPS * 1e12), 4)}
        if name == "auto":
            res.update(leg)
            res["path"] = ("four-wave split schedule (%d waves) into 2048-clock bit-plane chunks (two 256 MiB "
                           "buffers); each chunk's tiled transpose to u32 + f32 rows runs on a second stream beside "
                           "the next chunk's generation" % (4 * (n // 32 // 64)))
        else:
            res[name] = leg
    return res


def bench_grain(torch, mickey, synth, reps: int = 5):
    """Bitsliced Grain v1: 2^22 instances (splitmix64 seed 6 keys and 64-bit IVs), 8192
    bits each into bit-planes (4 GiB), init and generate timed separately.  At 36 VALU
    ops per clock for 32 instances the kernel writes faster than it computes, so its
    roofline is the HBM write bandwidth."""
    seed, n, nbits, _ = synth.workload("grain-4m")
    keys, ivs = synth.grain_keys_ivs(seed, n)
    dk, dv = torch.from_numpy(keys).cuda(), torch.from_numpy(ivs).cuda()
    stream = torch.cuda.current_stream()
    g = mickey.Grain(dk, dv, stream=stream)
    out = torch.empty(nbits * g.pitch, dtype=torch.uint8, device="cuda")
    warm_up(torch, lambda: g.generate(nbits, mickey.BITSLICED, out))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_init, t_gen = [], []
    for _ in range(reps):
        ev[0].record(stream)
        g.rekey(dk, dv)
        ev[1].record(stream)
        g.generate(nbits, mickey.BITSLICED, out)
        ev[2].record(stream)
        torch.cuda.synchronize()
        t_init.append(ev[0].elapsed_time(ev[1]))
        t_gen.append(ev[1].elapsed_time(ev[2]))
    g.close()
    ti, tg = float(np.mean(t_init)), float(np.mean(t_gen))
    bits = n * nbits
    ops = mickey.grain_ops_per_clock() * (n // 32) * nbits
    wbytes = bits / 8 + 2 * 20 * n  # keystream planes, plus the 160 state planes read and written
    print("# grain-4m: init %.3f ms, generate %.3f ms" % (ti, tg), file=sys.stderr, flush=True)
    return {"workload": "grain-4m: 2^22 Grain v1 instances, 80-bit keys, 64-bit IVs (splitmix64 seed 6), "
                        "8192 bits each, bitsliced planes",
            "gbit_s": round(bits / ((ti + tg) * 1e-3) / 1e9, 3), "init_ms": round(ti, 4),
            "generate_ms": round(tg, 4), "generate_gbit_s": round(bits / (tg * 1e-3) / 1e9, 3),
            "hbm_gb_s": round(wbytes / (tg * 1e-3) / 1e9, 1), "hbm_frac": round(wbytes / (tg * 1e-3) / 8e12, 4),
            "valu_frac": round(ops / (tg * 1e-3) / 78.6432e12, 4),
            "ops_per_clock_per_32": mickey.grain_ops_per_clock()}


def bench_aes(torch, mickey, synth, reps: int = 3):
    """Bitsliced AES-128-CTR: one key, 2^22 streams (splitmix64 seed 7 key and 64-bit
    nonces), 8192 bits (64 blocks) each into bit-planes (4 GiB).  VALU-bound: about 4.2
    lane-ops per keystream bit, mostly the S-box circuit."""
    seed, n, nbits, _ = synth.workload("aes-4m")
    key, nonces = synth.aes_inputs(seed, n)
    dk, dn = torch.from_numpy(key).cuda(), torch.from_numpy(nonces).cuda()
    stream = torch.cuda.current_stream()
    a = mickey.AesCtr(dk, dn, stream=stream)
    out = torch.empty(nbits * a.pitch, dtype=torch.uint8, device="cuda")
    warm_up(torch, lambda: a.generate(nbits, mickey.BITSLICED, out))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t_gen = []
    for _ in range(reps):
        a.seek(0)
        ev[0].record(stream)
        a.generate(nbits, mickey.BITSLICED, out)
        ev[1].record(stream)
        torch.cuda.synchronize()
        t_gen.append(ev[0].elapsed_time(ev[1]))
    a.close()
    tg = float(np.mean(t_gen))
    bits = n * nbits
    ops = mickey.aes_ops_per_block() * (n // 32) * (nbits // 128)
    print("# aes-4m: generate %.3f ms" % tg, file=sys.stderr, flush=True)
    return {"workload": "aes-4m: AES-128-CTR, one key, 2^22 streams with 64-bit nonces (splitmix64 seed 7), "
                        "8192 bits (64 blocks) each, bitsliced planes",
            "generate_ms": round(tg, 4), "generate_gbit_s": round(bits / (tg * 1e-3) / 1e9, 3),
            "valu_frac": round(ops / (tg * 1e-3) / 78.6432e12, 4),
            "ops_per_block_per_32": mickey.aes_ops_per_block(),
            "hbm_frac": round(bits / 8 / (tg * 1e-3) / 8e12, 4)}


def bench_mickey128(torch, mickey, synth, reps: int = 5, ncheck: int = 16):
    """Bitsliced MICKEY-128 2.0: 3 * 2^20 instances (splitmix64 seed 8, 128-bit keys and
    IVs), 8192 bits each into bit-planes (3 GiB); the R and S waves of each 64 slices run
    three waves per SIMD.  VALU-bound at 518 ops per clock for 32 instances.  ncheck
    seeded instances are compared with the oracle at full length."""
    from oracle import mickey128 as m128_oracle
    seed, n, nbits, _ = synth.workload("mickey128-3m")
    keys, ivs = synth.keys_ivs128(seed, n)
    dk, dv = torch.from_numpy(keys).cuda(), torch.from_numpy(ivs).cuda()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    m = mickey.Mickey128(dk, dv, stream=stream)
    m.sync()
    init_wall = time.perf_counter() - t0
    out = torch.empty(nbits * m.pitch, dtype=torch.uint8, device="cuda")
    warm_up(torch, lambda: m.generate(nbits, out))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for k in range(reps):
        m.generate(nbits, out)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    tg = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]))
    # the output holds each stream's last nbits clocks
    skip = m.bits_generated - nbits
    rng = np.random.default_rng(1280)
    idx = np.sort(rng.choice(n, ncheck, replace=False))
    planes = out.view(nbits, m.pitch)
    ti = torch.from_numpy(idx // 8).cuda()
    sh = torch.from_numpy(idx % 8).cuda().to(torch.uint8)
    got = ((planes[:, ti] >> sh) & 1).T.cpu().numpy()
    m.close()
    del out
    rows = m128_oracle.generate_many(keys[idx], ivs[idx], None, nbits, skip=skip, threads=8)
    want = np.unpackbits(rows, axis=1)[:, :nbits]
    mism = int((got != want).any(axis=1).sum())
    bits = n * nbits
    ops = mickey.mickey128_ops_per_clock() * (n // 32) * nbits
    print("# mickey128-3m: generate %.3f ms, oracle check %d/%d" % (tg, ncheck - mism, ncheck), file=sys.stderr,
          flush=True)
    return {"workload": "mickey128-3m: 3*2^20 MICKEY-128 2.0 instances (stand-in S tables), 128-bit keys and "
                        "IVs (splitmix64 seed 8), 8192 bits each, bitsliced planes",
            "generate_ms": round(tg, 4), "generate_gbit_s": round(bits / (tg * 1e-3) / 1e9, 3),
            "init_wall_ms": round(init_wall * 1e3, 2),
            "valu_frac": round(ops / (tg * 1e-3) / 78.6432e12, 4),
            "ops_per_clock_per_32": mickey.mickey128_ops_per_clock(),
            "oracle_check": {"instances": ncheck, "bits_each": nbits, "mismatches": mism}}


def bench_batch(torch, mickey, synth, oracle_runs=None, tune_cap_bits: int = 4096, nsample: int = 12,
                n_longest: int = 16, n_other: int = 48):
    """10,000 fresh requests (seed 4): IV lengths 0..80, lengths log-uniform in
    [2^8, 2^24) bits; one persistent work-queue launch replayed from a HIP graph,
    autotuned; compared with per-request plain launches (timed on a sample of requests
    and extrapolated linearly in length) and with the critical path: the longest request
    alone in latency mode.  With oracle_runs, the n_longest longest requests (all routed to
    latency mode) and n_other seeded others are checked bit for bit against the oracle,
    which runs on host threads while the GPU works, after both the routed and the
    all-bitsliced run."""
    import tempfile
    keys, ivs, ivb, nbits = synth.batch_requests(4, 10000)
    n = len(nbits)
    check = None
    if oracle_runs is not None:
        order = np.argsort(-nbits.astype(np.int64), kind="stable")
        rng = np.random.default_rng(404)
        check = np.concatenate([order[:n_longest], rng.choice(order[n_longest:], n_other, replace=False)])
        want = {int(i): oracle_runs.stream("batch", keys[i], ivs[i], int(ivb[i]), int(nbits[i])) for i in check}
    dk, dv, db = (torch.from_numpy(a).cuda() for a in (keys, ivs, ivb))
    words = (nbits // 32).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(words)])
    arena = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    ptrs = [arena.data_ptr() + 4 * int(o) for o in offs[:-1]]
    b = mickey.Batch(n)
    b.set(dk, dv, db, nbits, ptrs)
    with tempfile.TemporaryDirectory() as td:
        params = b.autotune(tune_cap_bits, os.path.join(td, "batch_tune.json"))
        tune = json.load(open(os.path.join(td, "batch_tune.json")))
    bs = torch.cuda.ExternalStream(b.stream_handle)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed_run():
        torch.cuda.synchronize()
        e0.record(bs)
        b.run()
        e1.record(bs)
        b.sync()
        return e0.elapsed_time(e1)
    def sample_words():
        return {} if check is None else {int(i): arena[int(offs[i]):int(offs[i + 1])].cpu().numpy().view(np.uint32)
                                         for i in check}
    arena.zero_()
    batch_ms = timed_run()  # size-aware routing (automatic threshold)
    got_routed = sample_words()
    routing = b.routing()
    b.set_latency_threshold(mickey.Batch.LATENCY_OFF)
    arena.zero_()
    bs_only_ms = timed_run()  # every request bitsliced
    got_bs = sample_words()
    b.close()
    del arena
    total_bits = int(nbits.sum())
    print("# batch-10k: %.1f ms routed (%s), %.1f ms all bitsliced (params %s)" % (batch_ms, routing, bs_only_ms, params),
          file=sys.stderr, flush=True)
    # per-request plain launches (mickey_init with n = 1, then row-major generate) on a
    # sample of requests up to 2^16 bits, fitted as a + b * nbits
    stream = torch.cuda.current_stream()
    order = np.argsort(nbits.astype(np.int64))
    short = order[nbits[order] <= (1 << 16)]
    pick = short[np.linspace(0, len(short) - 1, nsample).astype(int)]
    ts, ls = [], []
    out1 = torch.empty(1 << 11, dtype=torch.int32, device="cuda")
    for k, i in enumerate(pick):
        e0.record(stream)
        m = mickey.Mickey(dk[i:i + 1], dv[i:i + 1], db[i:i + 1], stream=stream)
        m.generate(int(nbits[i]), mickey.ROWMAJOR_U32, out1)
        e1.record(stream)
        torch.cuda.synchronize()
        m.close()
        if k:  # first one warms up
            ts.append(e0.elapsed_time(e1))
            ls.append(float(nbits[i]))
    slope, icpt = np.polyfit(np.array(ls), np.array(ts), 1)
    serial_ms = float(np.sum(icpt + slope * nbits.astype(np.float64)))
    lmax = int(nbits.max())
    bound_ms = float(icpt + slope * lmax)  # one lane running the longest request alone
    # the longest request alone in latency mode (a batch of one, routed there): the
    # critical path of any schedule of this batch on this engine.  Alone, one wave keeps
    # the device nearly idle and it runs at a lower clock than under the batch's load, so
    # the batch can finish somewhat below this time.
    il = int(np.argmax(nbits))
    b1 = mickey.Batch(1)
    buf1 = torch.empty(lmax // 32, dtype=torch.int32, device="cuda")
    b1.set(dk[il:il + 1], dv[il:il + 1], db[il:il + 1], nbits[il:il + 1], [buf1.data_ptr()])
    b1.set_latency_threshold(1)
    bs1 = torch.cuda.ExternalStream(b1.stream_handle)
    lat_alone = []
    for _ in range(3):
        torch.cuda.synchronize()
        e0.record(bs1)
        b1.run()
        e1.record(bs1)
        b1.sync()
        lat_alone.append(e0.elapsed_time(e1))
    b1.close()
    lat_bound_ms = float(min(lat_alone[1:]))  # the first run builds the graph
    verified = None
    if check is not None:
        mism = 0
        lat_checked = 0
        for i in check:
            w = want[int(i)].result()
            ok_r = words_be_bytes(got_routed[int(i)]) == w
            ok_b = words_be_bytes(got_bs[int(i)]) == w
            mism += int(not ok_r) + int(not ok_b)
            lat_checked += int(routing[0] is not None and int(nbits[i]) >= routing[0])
        verified = {"requests": int(len(check)), "outputs_compared": int(2 * len(check)), "mismatches": mism,
                    "latency_mode_requests": lat_checked,
                    "bits_per_run": int(nbits[check].sum()),
                    "sample": "the %d longest requests (%d..%d bits) and %d seeded others, full length, after "
                              "the routed run and after the all-bitsliced run, against the oracle"
                              % (n_longest, int(nbits[check[n_longest - 1]]), int(nbits[check[0]]), n_other)}
        print("# batch-10k oracle check: %d outputs, %d mismatches" % (2 * len(check), mism), file=sys.stderr,
              flush=True)
    return {"workload": "10,000 fresh requests (splitmix64 seed 4), IV lengths 0..80, lengths log-uniform in "
                        "[2^8, 2^24) bits, row-major u32 outputs, one persistent launch (HIP graph)",
            "requests": n, "total_bits": total_bits, "batch_ms": round(batch_ms, 2),
            "gbit_s": round(total_bits / (batch_ms * 1e-3) / 1e9, 3),
            "params": {"unroll": params[0], "waves_per_block": params[1], "word_bits": 32,
                       "tune_timings_ms": tune.get("timings_ms")},
            "routing": {"latency_threshold_bits": routing[0], "latency_requests": routing[1],
                        "latency_clock_ratio": round(routing[2], 4),
                        "bitsliced_only_ms": round(bs_only_ms, 2)},
            "critical_path": {"longest_bits": lmax,
                              "bitsliced_bound_ms": round(bound_ms, 2),
                              "bitsliced_only_over_bound": round(bs_only_ms / bound_ms, 4),
                              "longest_alone_latency_mode_ms": round(lat_bound_ms, 2),
                              "batch_over_longest_alone": round(batch_ms / lat_bound_ms, 4),
                              "clock_ns_single_bitsliced_lane": round(slope * 1e6, 2),
                              "clock_ns_single_latency_request": round(lat_bound_ms * 1e6 / lmax, 2),
                              "clock_ns_longest_in_batch_at_most": round(batch_ms * 1e6 / lmax, 2),
                              "note": "alone, the one busy wave leaves the device at a lower clock than the "
                                      "batch's load does, so the batch can end below the lone run"},
            "per_request_plain": {"sampled": len(ts), "fit_ms": [round(icpt, 4), round(slope * 1e6, 4)],
                                  "fit_units": ["ms", "ns per bit"], "extrapolated_serial_ms": round(serial_ms, 1),
                                  "batch_speedup": round(serial_ms / batch_ms, 1)},
            "oracle_check": verified}


def serve_check_states(sids, nbits, lat_bits: int, n_resumed: int = 48, n_long: int = 16,
                       resumed_cap_bits: int = 16 << 23, long_cap_bits: int = 24 << 23, seed: int = 505):
    """States of the served trace whose complete request histories the oracle replays:
    n_resumed seeded states with at least two requests (a history of at most
    resumed_cap_bits), and n_long seeded states with a request of at least lat_bits (one
    that may take a latency stream; a history of at most long_cap_bits)."""
    order = np.argsort(sids, kind="stable")
    ss = sids[order]
    starts = np.flatnonzero(np.r_[True, ss[1:] != ss[:-1]])
    ends = np.r_[starts[1:], len(ss)]
    total = np.add.reduceat(nbits[order].astype(np.int64), starts)
    biggest = np.maximum.reduceat(nbits[order].astype(np.int64), starts)
    count = ends - starts
    rng = np.random.default_rng(seed)
    res = np.flatnonzero((count >= 2) & (total <= resumed_cap_bits) & (biggest < lat_bits))
    lng = np.flatnonzero((biggest >= lat_bits) & (total <= long_cap_bits))
    pick = np.concatenate([rng.choice(res, min(n_resumed, len(res)), replace=False),
                           rng.choice(lng, min(n_long, len(lng)), replace=False)])
    return {int(ss[starts[g]]): order[starts[g]:ends[g]] for g in pick}  # state -> request ids in arrival order


def bench_serve(torch, mickey, synth, duration: float, max_bytes: int, drain: float, qclocks: int = 8192,
                lat_ratio: int = 4,
                lat_streams: int = 16384, lat_threshold: int = 1 << 26, rate: float = 20000.0,
                nstates: int = 10 ** 6, budget: int = 64 << 30, chunk: int = 64 << 10, sat_seconds: float = 3.0,
                oracle_runs=None):
    """Served generation over 10^6 resident states (splitmix64 seed 5 keys and 80-bit
    IVs, initialised).  Open loop: Poisson arrivals at `rate`/s for `duration` s, state
    uniform, size log-uniform in [4 KiB, max_bytes], delivered in `chunk`-byte chunks
    through a `budget`-byte output budget; latency = completion of the last chunk -
    scheduled arrival.  The run stops when every request is done or `drain` s after the
    last arrival; requests still running then are censored (their latency is only known
    to exceed the time they have waited).  With oracle_runs, the complete request
    histories of sampled states (serve_check_states) are replayed by the oracle on host
    threads during the run and compared with the delivered chunks by digest.  Closed loop
    (saturation): every state keeps one request of the same size distribution in flight,
    chunked through the same budget, for sat_seconds, with its per-request latency and
    per-chunk delivery gaps; compared with the plain kernel on the same 10^6 instances."""
    import hashlib
    keys, ivs = synth.keys_ivs(5, nstates)
    dk, dv = torch.from_numpy(keys).cuda(), torch.from_numpy(ivs).cuda()
    init = mickey.Mickey(dk, dv)
    init.sync()
    out = {}
    # -- open loop
    t_arr, sids, nbits = synth.serve_requests(5, nstates, rate, duration, 4096, max_bytes)
    n = len(t_arr)
    hist = serve_check_states(sids, nbits, lat_threshold) if oracle_runs is not None else {}
    want = {}  # request id -> future of its oracle digest

    def digests(fut, ids):
        data = fut.result()
        res, off = {}, 0
        for r in ids:
            nb = int(nbits[r]) // 8
            res[int(r)] = hashlib.blake2b(data[off:off + nb], digest_size=16).digest()
            off += nb
        return res
    hist_futs = []
    for sid, ids in hist.items():
        f = oracle_runs.stream("serve", keys[sid], ivs[sid], None, int(nbits[ids].sum()))
        hist_futs.append((f, ids))
    vreq = {int(r): sid for sid, ids in hist.items() for r in ids}
    hashers = {r: hashlib.blake2b(digest_size=16) for r in vreq}
    next_word = {r: 0 for r in vreq}
    order_ok = True
    nslices = 32768
    srv = mickey.Server(init, nslices=nslices, quantum_clocks=qclocks, budget_bytes=budget)
    srv.set_chunk(chunk)
    # size-aware routing: what is left of a request of lat_threshold bits or more takes one
    # of lat_streams latency streams (one request per four lanes), lat_ratio x the quantum
    # per step
    srv.set_latency(lat_streams, threshold_bits=lat_threshold, clocks_per_quantum=lat_ratio * qclocks)
    lat = np.full(n, np.inf)
    run_s = np.zeros(n)  # admission to completion
    t0 = time.monotonic_ns()
    i = done_n = 0
    last_done = t0
    nchunks = 0
    peak_running = 0
    t_stop = duration + drain
    next_note = 5.0
    vkeys = np.array(sorted(vreq), dtype=np.uint64)
    while done_n < n:
        now = (time.monotonic_ns() - t0) * 1e-9
        if now > t_stop:
            break
        if now > next_note:
            print("#   serve open loop t=%.0f s: %d/%d done" % (now, done_n, n), file=sys.stderr, flush=True)
            next_note += 5.0
        k = int(np.searchsorted(t_arr, now, side="right"))
        if k > i:
            srv.submit_many(sids[i:k], nbits[i:k])  # ids are assigned in arrival order
            i = k
        srv.step()
        ch = srv.poll_chunks(1 << 16)
        if len(ch):
            nchunks += len(ch)
            if len(vkeys):
                for c in ch[np.isin(ch["request"], vkeys)]:
                    r, w = int(c["request"]), int(c["words"])
                    buf = torch.empty(w, dtype=torch.int32, device="cuda")
                    srv.copy_chunk(int(c["handle"]), buf, w)
                    order_ok &= int(c["offset"]) == next_word[r]
                    next_word[r] += w
                    hashers[r].update(words_be_bytes(buf.cpu().numpy().view(np.uint32)))
            srv.release_chunks(ch["handle"])  # the consumer has taken the chunk
        ids = srv.poll(1 << 16)
        if len(ids):
            tm = srv.times_many(ids)
            lat[ids] = (tm[:, 2].astype(np.float64) - t0) * 1e-9 - t_arr[ids]
            run_s[ids] = (tm[:, 2].astype(np.float64) - tm[:, 1].astype(np.float64)) * 1e-9
            last_done = max(last_done, int(tm[:, 2].max()))
            done_n += len(ids)
        st = srv.stats()
        peak_running = max(peak_running, st["running"])
        if not len(ch) and not len(ids) and i == n and st["running"] == 0 and st["waiting"] == 0:
            srv.wait()
    t_end = time.monotonic_ns()
    st = srv.stats()
    lat_words = srv.latency_words_many(vkeys) if len(vkeys) else np.zeros(0, dtype=np.uint64)
    srv.close()
    span = (t_end - t0) * 1e-9
    done = np.isfinite(lat)
    cens = np.where(done, lat, span - t_arr)  # a censored request has waited at least this long

    def pct(q):
        v = float(np.percentile(lat, q))
        return (round(v, 4) if np.isfinite(v) else None), round(float(np.percentile(cens, q)), 4)
    p50, p50_lb = pct(50)
    p99, p99_lb = pct(99)
    # per-request stream rate (bits / (completion - admission)) of completed requests of >= 1 MiB
    big = done & (nbits >= 8 * (1 << 20))
    rate_mbit = round(float(np.median(nbits[big] / run_s[big])) / 1e6, 3) if big.any() else None
    verified = None
    if hist:
        t_wait = time.perf_counter()
        want = {}
        for f, ids in hist_futs:
            want.update(digests(f, ids))
        wait_s = time.perf_counter() - t_wait
        lw = {int(r): int(v) for r, v in zip(vkeys, lat_words)}
        checked = mism = resumed = on_lat = 0
        for sid, ids in hist.items():
            for pos, r in enumerate(ids):
                r = int(r)
                if not done[r]:
                    break  # later requests of the state wait for this one
                checked += 1
                resumed += int(pos > 0)
                on_lat += int(lw[r] > 0)
                mism += int(hashers[r].digest() != want[r])
        verified = {"states": len(hist), "requests_checked": checked, "mismatches": mism,
                    "resumed_requests": resumed, "latency_stream_requests": on_lat,
                    "chunks_in_order": bool(order_ok), "bits_replayed": int(sum(int(nbits[ids].sum())
                                                                              for ids in hist.values())),
                    "oracle_wait_after_run_s": round(wait_s, 2),
                    "sample": "complete request histories of %d seeded states (%d with two or more requests, "
                              "%d with a request of >= %d KiB), replayed by the oracle on host threads during "
                              "the run; each completed request's delivered words compared with the oracle's by "
                              "a 128-bit BLAKE2b digest" % (len(hist), sum(1 for v in hist.values() if len(v) > 1),
                                                             sum(1 for v in hist.values()
                                                                 if int(nbits[v].max()) >= lat_threshold),
                                                             lat_threshold >> 13)}
        print("# serve open loop oracle check: %d requests (%d resumed, %d on latency streams), %d mismatches"
              % (checked, resumed, on_lat, mism), file=sys.stderr, flush=True)
    out["open_loop"] = {
        "workload": "10^6 resident states; Poisson arrivals %.0f/s for %.1f s; state uniform; size log-uniform "
                    "4 KiB..%d KiB; row-major u32 output delivered in %d KiB chunks; 64 GiB output budget; "
                    "%d slots x 32 lanes; quantum %d clocks; requests with >= %d KiB left routed to %d "
                    "latency streams (%d clocks per quantum) while the bit lanes are at most half busy; stopped "
                    "%.0f s after the last arrival" % (rate, duration, max_bytes >> 10, chunk >> 10, nslices, qclocks,
                                                       lat_threshold >> 13, lat_streams, lat_ratio * qclocks, drain),
        "requests": n, "completed": int(done.sum()), "completed_fraction": round(float(done.mean()), 4),
        "bits_offered": int(nbits.sum()), "bits_delivered": st["bits_delivered"], "span_s": round(span, 3),
        "served_gbit_s": round(st["bits_delivered"] / span / 1e9, 3),
        "offered_gbit_s": round(float(nbits.sum()) / duration / 1e9, 3),
        "latency_s": {"p50": p50, "p99": p99, "p50_lower_bound": p50_lb, "p99_lower_bound": p99_lb,
                      "max_completed": round(float(lat[done].max()), 4) if done.any() else None},
        "stream_rate_mbit_s_per_request": rate_mbit,
        "host_s": {"blocked_on_gpu": round(st["host_wait_ns"] * 1e-9, 3),
                   "retiring": round(st["host_retire_ns"] * 1e-9, 3),
                   "admitting": round(st["host_admit_ns"] * 1e-9, 3)},
        "chunks": nchunks, "peak_running": peak_running, "steps": st["steps"],
        "mean_quantum_ms": round(st["quantum_ns"] / max(st["steps"], 1) / 1e6, 3),
        "oracle_check": verified,
    }
    print("# serve open loop: %d/%d requests done, p50 %s s p99 %s s (lower bound %.1f s)" % (
        int(done.sum()), n, p50, p99, p99_lb), file=sys.stderr, flush=True)
    # -- closed loop: every state always has a request in flight (saturation)
    srng = np.random.default_rng(55)
    lo, hi = np.log2(4096), np.log2(max_bytes)

    def sizes(k):  # bits: log-uniform 4 KiB .. max_bytes, whole 32-bit words
        return (32 * np.floor(2.0 ** (lo + (hi - lo) * srng.random(k)) / 4)).astype(np.uint64)
    nsl = (nstates + 31) // 32
    qclk = 8192
    phases = (chunk * 8) // qclk  # quanta per chunk

    def closed_loop(stagger: bool):
        """Served rate with every state busy.  stagger: the first requests are submitted over
        the first `phases` steps (1/phases of the states per step), so that the lanes' chunk
        boundaries fall in different quanta, as in a server that has been running; without
        it every lane starts in the same quantum and all of them finish a chunk together."""
        srv = mickey.Server(init, nslices=nsl, quantum_clocks=qclk, budget_bytes=budget)
        srv.set_chunk(chunk)
        all_s = np.arange(nstates, dtype=np.uint32)
        sid_of = np.zeros(1 << 23, dtype=np.uint32)  # request id -> state id
        groups = np.array_split(all_s, phases if stagger else 1)
        t_start = time.monotonic_ns()
        b0 = tb0 = st0 = c0 = None
        nchunks = 0
        k = 0
        last_t = np.zeros(len(sid_of), dtype=np.int64)  # request id -> when its last chunk was polled
        gaps, req_lat = [], []
        while True:
            if k < len(groups):
                new = srv.submit_many(groups[k], sizes(len(groups[k])))
                sid_of[new] = groups[k]
                k += 1
            srv.step()
            ch = srv.poll_chunks(1 << 20)
            t_poll = time.monotonic_ns()
            if len(ch):
                nchunks += len(ch)
                r = ch["request"].astype(np.int64)
                if b0 is not None:  # delivery gaps between consecutive chunks of a request
                    prev = last_t[r]
                    gaps.append((t_poll - prev[prev > 0]) * 1e-9)
                last_t[r] = t_poll
                srv.release_chunks(ch["handle"])  # the consumer has taken the chunk
            ids = srv.poll(1 << 20)
            if len(ids):
                if b0 is not None:  # submission to completion of the last chunk
                    tm = srv.times_many(ids)
                    req_lat.append((tm[:, 2].astype(np.float64) - tm[:, 0].astype(np.float64)) * 1e-9)
                again = sid_of[ids]
                new = srv.submit_many(again, sizes(len(again)))
                if new.max() >= len(sid_of):
                    sid_of = np.concatenate([sid_of, np.zeros_like(sid_of)])
                    last_t = np.concatenate([last_t, np.zeros_like(last_t)])
                sid_of[new] = again
            el = (time.monotonic_ns() - t_start) * 1e-9
            st = srv.stats()
            if b0 is None and el > 2.0 and st["steps"] >= 40 + len(groups):  # warm-up
                b0, tb0, st0, c0 = st["bits_delivered"], time.monotonic_ns(), st, nchunks
            if b0 is not None and (time.monotonic_ns() - tb0) * 1e-9 > sat_seconds:
                break
        b1, tb1, st1 = st["bits_delivered"], time.monotonic_ns(), st
        srv.close()
        win = (tb1 - tb0) * 1e-9

        def d(key):
            return (st1[key] - st0[key]) * 1e-9
        g = np.concatenate(gaps) if gaps else np.zeros(0)
        rl = np.concatenate(req_lat) if req_lat else np.zeros(0)

        def q(a, p):
            return round(float(np.percentile(a, p)), 4) if len(a) else None
        return {"served_gbit_s": round((b1 - b0) / win / 1e9, 3), "window_s": round(win, 3),
                "latency_s": {"chunk_gap_p50": q(g, 50), "chunk_gap_p99": q(g, 99), "chunk_gaps": int(len(g)),
                              "request_p50": q(rl, 50), "request_p99": q(rl, 99), "requests_completed": int(len(rl)),
                              "note": "chunk gap: time between deliveries of consecutive 64 KiB chunks of a "
                                      "request (the stream's latency under load); request: submission to last "
                                      "chunk, for requests completed in the window"},
                "chunks_per_s": round((nchunks - c0) / win), "steps_in_window": st1["steps"] - st0["steps"],
                "device_s_in_window": round(d("gpu_ns"), 3),
                "host_s_in_window": {"blocked_on_gpu": round(d("host_wait_ns"), 3),
                                     "retiring": round(d("host_retire_ns"), 3),
                                     "admitting": round(d("host_admit_ns"), 3),
                                     "client_and_other": round(win - d("host_wait_ns") - d("host_retire_ns")
                                                               - d("host_admit_ns"), 3)}}
    steady = closed_loop(True)
    sync = closed_loop(False)
    served = steady["served_gbit_s"]
    # plain kernel on the same 10^6 instances, row-major
    pbits = 65536
    stream = torch.cuda.current_stream()
    buf = torch.empty((nstates, pbits // 32), dtype=torch.int32, device="cuda")
    init.generate(pbits, mickey.ROWMAJOR_U32, buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    init.generate(pbits, mickey.ROWMAJOR_U32, buf)
    e1.record(stream)
    torch.cuda.synchronize()
    plain = nstates * pbits / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del buf
    init.close()
    out["closed_loop"] = dict(
        workload="every one of the 10^6 states keeps one request in flight (resubmitted on completion), size "
                 "log-uniform 4 KiB..%d KiB, %d KiB chunks through the 64 GiB budget, %d slots x 32 lanes, "
                 "quantum %d clocks; the first requests submitted over the first %d steps (one chunk's worth "
                 "of quanta) so that chunk boundaries are spread over the quanta; measured over %.1f s after a "
                 "2 s warm-up" % (max_bytes >> 10, chunk >> 10, nsl, qclk, phases, steady["window_s"]),
        plain_same_instances_gbit_s=round(plain, 3), served_over_plain=round(served / plain, 4), **steady)
    out["closed_loop"]["synchronized_start"] = {
        "note": "the same loop with every first request submitted at once: all lanes finish their 64 KiB "
                "chunks in the same quanta, and the host's retirement of those bursts idles the device",
        "served_gbit_s": sync["served_gbit_s"], "served_over_plain": round(sync["served_gbit_s"] / plain, 4),
        "device_s_in_window": sync["device_s_in_window"], "window_s": sync["window_s"],
        "latency_s": sync["latency_s"]}
    print("# serve closed loop: %.1f Gbit/s served vs %.1f plain (synchronized start: %.1f)" % (
        served, plain, sync["served_gbit_s"]), file=sys.stderr, flush=True)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-word64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=131072,
                    help="instances the oracle runs for cpu_baseline (~10-15 s on 16 host threads)")
    ap.add_argument("--no-rowmajor", action="store_true", help="skip the row-major 2^20 x 65536 measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the 10,000-request batched measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the served measurements")
    ap.add_argument("--no-grain", action="store_true", help="skip the bitsliced Grain leg")
    ap.add_argument("--no-aes", action="store_true", help="skip the bitsliced AES-CTR leg")
    ap.add_argument("--no-mickey128", action="store_true", help="skip the bitsliced MICKEY-128 2.0 leg")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="Poisson arrival window of the served run")
    ap.add_argument("--serve-max-kib", type=int, default=64 << 10, help="largest served request (KiB)")
    ap.add_argument("--serve-drain", type=float, default=90.0,
                    help="seconds the open-loop served run continues after the last arrival")
    ap.add_argument("--serve-quantum", type=int, default=8192, help="open loop: clocks per quantum (multiple of 32)")
    ap.add_argument("--serve-lat-ratio", type=int, default=4,
                    help="open loop: latency-stream clocks per quantum, as a multiple of the quantum")
    ap.add_argument("--serve-lat-streams", type=int, default=16384, help="open loop: latency streams (0: off)")
    ap.add_argument("--serve-lat-kib", type=int, default=8192,
                    help="open loop: requests with at least this many KiB left take latency streams")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--code-hash", action="store_true", help="print the headline kernel's code hash and exit")
    args = ap.parse_args()
    if args.code_hash:
        print(kernel_code_hash())
        return 0
    if args.copy_calib:
        import torch
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")  # 1 GiB
        a.fill_(7)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4, "launches": 3}))
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU only: the instances are independent, so more GPUs "
              "would only partition them (no collectives); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_1909_04750_amd import mickey, synth

    assert torch.cuda.is_available(), "needs a HIP GPU"
    mickey.load_library()
    seed, n, nbits, _ = synth.workload(WORKLOAD)
    keys, ivs = synth.keys_ivs(seed, n)
    dkeys = torch.from_numpy(keys).cuda()
    divs = torch.from_numpy(ivs).cuda()
    stream = torch.cuda.current_stream()
    m = mickey.Mickey(dkeys, divs, None, stream=stream)
    out = torch.empty(nbits * m.pitch, dtype=torch.uint8, device="cuda")
    print("# workload %s: n=%d nbits=%d output %.2f GiB" % (WORKLOAD, n, nbits, out.numel() / 2**30),
          file=sys.stderr, flush=True)

    def step(ev):
        ev[0].record(stream)
        m.rekey(dkeys, divs)
        ev[1].record(stream)
        m.generate(nbits, mickey.BITSLICED, out)
        ev[2].record(stream)

    for _ in range(args.warmup):
        step([torch.cuda.Event(enable_timing=True) for _ in range(3)])
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    init_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    gen_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    ms_per_step = wall * 1e3 / args.steps
    bits_per_step = n * nbits
    value = bits_per_step / (ms_per_step * 1e-3) / 1e9
    print("# step %.3f ms (init %.3f ms, generate %.3f ms)" % (ms_per_step, init_ms, gen_ms),
          file=sys.stderr, flush=True)

    ops = mickey.ops_per_clock()
    n_pad = m.pitch * 8
    gen_ops = ops * (n_pad // 32) * nbits
    achieved = gen_ops / (gen_ms * 1e-3) / 1e12
    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "plain-4m: 2^22 MICKEY 2.0 instances, 80-bit keys and IVs from "
                        "splitmix64(seed=2), full init, 8192 keystream bits each, bitsliced "
                        "column-major output (4 GiB), uint32 slicing words",
            "instances": n,
            "bits_per_instance": nbits,
            "layout": "bitsliced",
            "word_bits": 32,
        },
        "init_ms": round(init_ms, 4),
        "generate_ms": round(gen_ms, 4),
        "generate_gbit_s": round(bits_per_step / (gen_ms * 1e-3) / 1e9, 3),
        "roofline": {
            "bound": "alu",
            "kernel": "gen_bitsliced_kernel<1>",
            "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 3),
            "unit": "TOP/s (32-bit VALU lane-ops)",
            "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "ops_per_launch": gen_ops,
            "traffic": traffic_record("gen_bitsliced"),
            "hbm_write_gbs": round(nbits * m.pitch / (gen_ms * 1e-3) / 1e9, 1),
            "hbm_write_frac": round(nbits * m.pitch / (gen_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
    }

    if not args.no_word64:
        m.set_word_bits(64)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        m.generate(nbits, mickey.BITSLICED, out)  # warm
        ev[0].record(stream)
        reps = 2
        for _ in range(reps):
            m.generate(nbits, mickey.BITSLICED, out)
        ev[1].record(stream)
        torch.cuda.synchronize()
        g64 = ev[0].elapsed_time(ev[1]) / reps
        res["word64"] = {"generate_ms": round(g64, 4),
                         "generate_gbit_s": round(bits_per_step / (g64 * 1e-3) / 1e9, 3)}
        m.set_word_bits(32)

    if not args.no_cpu_baseline:
        # GPU bits of the sample from the last step's output (same keys, rekeyed each step)
        m.rekey(dkeys, divs)
        m.generate(nbits, mickey.BITSLICED, out)
        rng = np.random.default_rng(0)
        sample_idx = np.sort(rng.choice(n, args.cpu_sample, replace=False))
        planes = out.view(nbits, m.pitch)
        ti = torch.from_numpy(sample_idx // 8).cuda()
        sh = torch.from_numpy(sample_idx % 8).cuda().to(torch.uint8)
        gpu_bits = ((planes[:, ti] >> sh) & 1).T.cpu().numpy()
        threads = oracle_threads()
        res["cpu_baseline"] = cpu_baseline(keys, ivs, nbits, gpu_bits, sample_idx, threads)
        res["cpu_baseline"]["c1_full"] = cpu_baseline_c1(torch, mickey, synth, threads)

    m.close()
    del out
    torch.cuda.empty_cache()
    if not args.no_rowmajor:
        res["rowmajor_1m"] = bench_rowmajor(torch, mickey, synth)
    if not args.no_grain:
        res["grain_4m"] = bench_grain(torch, mickey, synth)
    if not args.no_aes:
        res["aes_4m"] = bench_aes(torch, mickey, synth)
    if not args.no_mickey128:
        res["mickey128_3m"] = bench_mickey128(torch, mickey, synth)
    # the oracle's runs on sampled batched and served requests (part of the cpu_baseline leg)
    # go on host threads while the GPU works; they also check those requests' outputs
    # (half the host threads: the server's host loop and the GPU runtime need the rest)
    oruns = None if args.no_cpu_baseline else OracleRuns(max(1, oracle_threads() // 2))
    if not args.no_batch:
        res["batch_10k"] = bench_batch(torch, mickey, synth, oracle_runs=oruns)
    if not args.no_serve:
        res["serve"] = bench_serve(torch, mickey, synth, args.serve_seconds, args.serve_max_kib << 10,
                                   args.serve_drain, args.serve_quantum, args.serve_lat_ratio, args.serve_lat_streams,
                                   args.serve_lat_kib << 13, oracle_runs=oruns)
    if oruns is not None:
        oruns.close()
        if "cpu_baseline" in res:
            res["cpu_baseline"]["batch_10k_sample"] = oruns.rate("batch")
            res["cpu_baseline"]["serve_sample"] = oruns.rate("serve")
            res["cpu_baseline"]["sample_threads"] = oruns.threads
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
