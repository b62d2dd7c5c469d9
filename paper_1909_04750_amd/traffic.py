"""Turn rocprofv3 FETCH_SIZE / WRITE_SIZE counter CSVs into HBM bytes per launch.

Usage (from the repository root, after the two counter runs named in the summary):
  python -m paper_1909_04750_amd.traffic FETCH.csv WRITE.csv CALIB_FETCH.csv CALIB_WRITE.csv \\
      --kernel gen_bitsliced_kernel<1> --calib-kernel <copy kernel name part> --out profiles/x.json

Each counter is summed per dispatch (KiB), averaged over the dispatches of the kernel,
and scaled by bytes / counter of a plain copy kernel of known size (1 GiB read, 1 GiB
written per launch).  The record carries the hash of the kernel's machine code in the built
library, which bench.py checks.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import subprocess
import sys
from collections import defaultdict


def per_dispatch(path: str, counter: str, name_part: str):
    vals = defaultdict(float)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]:
            vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
    return list(vals.values())


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch")
    ap.add_argument("write")
    ap.add_argument("calib_fetch")
    ap.add_argument("calib_write")
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--calib-kernel", required=True)
    ap.add_argument("--calib-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    f = per_dispatch(a.fetch, "FETCH_SIZE", a.kernel)
    w = per_dispatch(a.write, "WRITE_SIZE", a.kernel)
    cf = per_dispatch(a.calib_fetch, "FETCH_SIZE", a.calib_kernel)
    cw = per_dispatch(a.calib_write, "WRITE_SIZE", a.calib_kernel)
    if not (f and w and cf and cw):
        print("missing dispatches", len(f), len(w), len(cf), len(cw), file=sys.stderr)
        return 1
    kf = a.calib_bytes / (max(cf) * 1024.0)  # bytes per counted byte (calibration: largest copy dispatch)
    kw = a.calib_bytes / (max(cw) * 1024.0)
    fetch = sum(f) / len(f) * 1024.0 * kf
    write = sum(w) / len(w) * 1024.0 * kw
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    h = subprocess.check_output([sys.executable, os.path.join(root, "bench.py"), "--code-hash"]).decode().strip()
    rec = {"kernel": a.kernel, "code_hash": h, "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "hbm_bytes_per_launch": fetch + write, "calibration_factor": {"fetch": kf, "write": kw},
           "dispatches": {"fetch": len(f), "write": len(w)}}
    json.dump(rec, open(a.out, "w"), indent=1)
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
