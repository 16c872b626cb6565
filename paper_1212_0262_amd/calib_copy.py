"""Calibration run for HBM-traffic counters: a plain device copy of known size.

Run under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``): the elementwise
kernel reads exactly ``--mib`` MiB and writes the same amount, so the counter
value per dispatch divided by that size is the factor that converts the counter
into bytes for the kernels of libmd measured the same way.

Usage: python -m paper_1212_0262_amd.calib_copy [--mib 512] [--reps 3]
"""
from __future__ import annotations

import argparse
import sys


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=512)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    n = args.mib * (1 << 20) // 4
    src = torch.rand(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        torch.mul(src, 1.0, out=dst)   # one read and one write of n float32 values
    torch.cuda.synchronize()
    print(f"copied {args.mib} MiB x {args.reps} (read {args.mib} MiB, wrote {args.mib} MiB per dispatch)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
