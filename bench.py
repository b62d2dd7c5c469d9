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
import hashlib
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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("csrc/mickey_bitslice.h", "csrc/mickey_kernels.hip"):
        h.update(open(os.path.join(ROOT, "paper_1909_04750_amd", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, WORKLOAD))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


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
        "kind": "oracle",
        "sample": "%d of the %d instances (init + %d keystream bits each), %.1f s wall"
                  % (len(sample_idx), keys.shape[0], nbits, dt),
        "sample_bit_exact_vs_gpu": match,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-word64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2048)
    args = ap.parse_args()
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
        threads = min(os.cpu_count() or 1, 16)
        res["cpu_baseline"] = cpu_baseline(keys, ivs, nbits, gpu_bits, sample_idx, threads)

    m.close()
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
