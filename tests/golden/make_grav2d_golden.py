#!/usr/bin/env python3
"""Writes the oracle's energies along the 2D self-gravitating benchmark run.

The 2D model of Sec. 2 (eq. 3: V = (1/N) sum_{i<j} log(|r_i - r_j|^2 + eps)),
integrated by the fourth-order Yoshida composition of Sec. 3 (eq. 4), from the
benchmark's seeded state: positions uniform in the unit disk, momenta Gaussian
with sigma = 0.5 and zero mean (seed 3), eps = 1e-3, dt = 0.01.  Sec. 4 judges
a run by its relative energy error |E(t) - E0| / |E0|; the file written here
holds the FP64 oracle's K, V and E at every report time, plus the positions and
momenta of a fixed sample of particles, so that the GPU runs can be compared
with the oracle at each report time without repeating the O(N^2) CPU run.

Only the oracle (oracle/) and the seeded input generator are called.  The JSON
written holds every float as Python's shortest round-trip repr.

Usage:
    python tests/golden/make_grav2d_golden.py --n 65536 --steps 100 --every 10
    python tests/golden/make_grav2d_golden.py --n 262144 --steps 100 --every 10 \\
        --checkpoint /tmp/grav2d_262144.npz
With --checkpoint the state after each report time is saved there and an
interrupted run resumes from it (the same steps, so the same numbers).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1212_0262_amd import inputs  # noqa: E402

SEED, SIGMA, EPS, DT = 3, 0.5, 1e-3, 0.01
N_SAMPLE = 32


def golden_path(n: int) -> str:
    return os.path.join(HERE, f"grav2d_disk_seed3_n{n}.json")


def sample_rows(n: int) -> list:
    rows = np.random.default_rng([SEED, n]).choice(n, size=min(N_SAMPLE, n), replace=False)
    return sorted(int(r) for r in rows)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--threads", type=int, default=0, help="oracle OpenMP threads (0: all)")
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.threads > 0:
        oracle.set_threads(args.threads)
    n = args.n
    out = args.out or golden_path(n)
    rows = sample_rows(n)
    q, p = inputs.grav2d_disk(n, seed=SEED, sigma=SIGMA)
    rec = {
        "what": "FP64 oracle energies along the 2D self-gravitating run (Sec. 2 eq. 3, Sec. 3 eq. 4, "
                "relative energy error of Sec. 4)",
        "written_by": "tests/golden/make_grav2d_golden.py",
        "command": f"python tests/golden/make_grav2d_golden.py --n {n} --steps {args.steps} --every {args.every}",
        "recipe": "inputs.grav2d_disk(n, seed=3, sigma=0.5): r = sqrt(U(0,1)), phi = U(0, 2 pi), "
                  "p ~ N(0, 0.5) minus its mean",
        "n": n, "seed": SEED, "sigma": SIGMA, "eps": EPS, "dt": DT, "every": args.every,
        "sample_rows": rows, "steps": [], "K": [], "V": [], "E": [], "q_sample": [], "p_sample": [],
        "oracle_threads": oracle.get_threads(), "seconds": 0.0,
    }
    step0 = 0
    f = None
    if args.checkpoint and os.path.exists(args.checkpoint):
        ck = np.load(args.checkpoint)
        q, p, f, step0 = ck["q"], ck["p"], ck["f"], int(ck["step"])
        with open(out) as fh:
            rec = json.load(fh)
        keep = sum(1 for s in rec["steps"] if s <= step0)  # entries written after the checkpoint go
        for key in ("steps", "K", "V", "E", "q_sample", "p_sample"):
            rec[key] = rec[key][:keep]
        print(f"resuming at step {step0}", flush=True)
    t_start = time.perf_counter() - rec["seconds"]

    def record(step, q, p):
        e = oracle.energy(oracle.GRAV2D, q, p, EPS)
        rec["steps"].append(step)
        rec["K"].append(float(e[0]))
        rec["V"].append(float(e[1]))
        rec["E"].append(float(e[2]))
        rec["q_sample"].append(q[:, rows].tolist())
        rec["p_sample"].append(p[:, rows].tolist())
        rec["seconds"] = time.perf_counter() - t_start
        with open(out + ".tmp", "w") as fh:
            json.dump(rec, fh, indent=1)
        os.replace(out + ".tmp", out)
        print(f"step {step}: K={e[0]!r} V={e[1]!r} E={e[2]!r} ({rec['seconds']:.0f} s)", flush=True)

    if f is None:
        record(0, q, p)
        f = oracle.force(oracle.GRAV2D, q, EPS)
    step = step0
    while step < args.steps:
        k = min(args.every, args.steps - step)
        q, p, f = oracle.step(oracle.GRAV2D, q, p, f, DT, k, EPS)
        step += k
        record(step, q, p)
        if args.checkpoint:
            np.savez(args.checkpoint + ".tmp.npz", q=q, p=p, f=f, step=step)
            os.replace(args.checkpoint + ".tmp.npz", args.checkpoint)
    return 0


if __name__ == "__main__":
    sys.exit(main())
