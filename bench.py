#!/usr/bin/env python3
"""Benchmark: pair-interaction throughput of the 2D self-gravitating model.

Workload: N = 262,144 particles, eps = 1e-3, positions uniform in the unit disk,
momenta Gaussian (sigma = 0.5) with zero total momentum (seed 3), dt = 0.01.
A step is one fourth-order Yoshida step (three all-pairs force evaluations);
the timed region is `--steps` consecutive steps in one md_step call, with the
state resident in HBM.  Throughput = 3 N^2 pair interactions per step (self
pairs included, as in the paper's tiles) / elapsed time.

The headline line is the mixed form (FP32 pair arithmetic, FP32 partials folded
into FP64) in md_step's automatic launch form, which at this N is the symmetric
one (each pair evaluated once for both particles); the staged form (every ordered
pair evaluated) is timed beside it.  The FP64 form is timed on the same steps, and
the relative energy error |E - E0| / |E0| (and the better conditioned
|E - E0| / (K0 + |V0|)) is reported for both; the mixed figure counts only if
its error is <= 1e-5.

Also reported: the pair kernel's fraction of the FP32 vector peak (roofline: its
own launches timed by the library with HIP events on its stream, and the interactions
one launch covers), the SIMD cycles it spends per pair and wavefront, and
the FP64 CPU oracle's pair throughput on a bounded sample of force rows of the
same configuration (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 2] [--no-fp64] [--no-cpu] [--no-variants]
                       [--launch auto|staged|symmetric]
       python bench.py --workload ring|hmf|ensemble|adjoint|paper_errors   (the other workloads)
       python bench.py --workload copy_calibration   (a plain copy of known size, for the traffic counters)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gpair-interactions/s (2D gravity N=262144), mixed vs FP64 at dE/E<=1e-5"
N = 262_144
EPS = 1e-3
DT = 0.01
SEED = 3
SIGMA = 0.5
FLOPS_PER_PAIR = 10          # 2 sub, 2 FMA (r^2 + eps), 2 FMA (accumulate); plus one reciprocal
VALU_PER_PAIR = 6            # the same six instructions, FP32, non-transcendental
TRANS_PER_PAIR = 1           # v_rcp_f32
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (FMA = 2 flops)
PEAK_FP64_TFLOPS = 78.6
SIMD_CYCLES_PER_S = 256 * 4 * 2.4e9   # 1024 SIMDs at 2.4 GHz
LAUNCH_NAMES = {1: "staged", 2: "fused", 3: "symmetric"}
ENS_SYM_TILE = 512           # particles per tile of the ensembles' symmetric form (md_get_sym_tile)


def sym_counts(n, tile):
    """Tile pairs' and diagonal tiles' evaluations of one symmetric launch over n
    particles in tiles of `tile` (n padded to a multiple of 1024)."""
    nt = -(-n // 1024) * 1024 // tile
    return nt * (nt - 1) // 2 * tile ** 2, nt * tile ** 2
SYM_FLOPS_PER_EVAL = 14      # symmetric form, per pair evaluated: 2 sub, 2 FMA (r^2), 2 FMA (i side), 2 FMA (j side)
PAIR_KERNEL_SRCS = [os.path.join(ROOT, "paper_1212_0262_amd", "csrc", f) for f in ("pair.hip", "pair_terms.h", "device.h")]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "grav2d_pair_mixed_n262144_pmc.txt")
HMF_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hmf_pass_n1e7_pmc.txt")
HMF_KERNEL_SRCS = [os.path.join(ROOT, "paper_1212_0262_amd", "csrc", f) for f in ("hmf.hip", "device.h")]
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
GATE_BAR = {"mixed": 1e-5, "fp64": 1e-6}   # |E - E_oracle| / |E0| at every report time


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def source_hash(srcs) -> str:
    """Hash of the sources a kernel is compiled from (the counter summaries record it)."""
    h = hashlib.sha256()
    for fn in srcs:
        with open(fn, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hmf_traffic_from_profile():
    """HBM bytes of one FP64 stage pass (the median dispatch) from the committed counter
    summary, if it was taken on the current source of the pass kernel; else None."""
    try:
        txt = open(HMF_TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not (m and b) or m.group(1) != source_hash(HMF_KERNEL_SRCS):
        return None
    return float(b.group(1))


def traffic_from_profile(launch, tiles):
    """HBM bytes per launch of the dominant pair kernel from the committed counter
    summary, if it was taken on the current kernel source in the same launch form
    (and, for the staged form, the same tiles); else None."""
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    f = re.search(r"launch:\s*(\w+)", txt)
    t = re.search(r"tiles_ipl_waves_jsplit_jtile:\s*([0-9, ]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not (m and f and t and b) or m.group(1) != source_hash(PAIR_KERNEL_SRCS) or f.group(1) != launch:
        return None
    if launch == "staged" and [int(x) for x in t.group(1).replace(" ", "").split(",") if x] != list(tiles):
        return None
    return float(b.group(1))


def run_variant(md, torch, prec, q0, p0, steps, warmup, launch=None):
    """Time `steps` Yoshida steps of one precision form (and launch form, if given);
    returns a result dict."""
    stream = torch.cuda.current_stream()
    ctx = md.md_init(md.GRAV2D, prec, N, EPS, stream=stream)
    if launch is not None:
        md.md_set_launch(ctx, launch)
    q = torch.from_numpy(q0).cuda()
    p = torch.from_numpy(p0).cuda()
    f = torch.empty_like(q)
    e0 = md.md_energy(ctx, q, p).cpu().numpy()
    md.md_force(ctx, q, f)
    if warmup > 0:  # warm up on a copy so the timed run starts from the initial state
        qw, pw, fw = q.clone(), p.clone(), f.clone()
        md.md_step(ctx, qw, pw, fw, DT, warmup)
        del qw, pw, fw
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # the library brackets each launch of its pair kernel with HIP events on the same stream
    md.md_timing_begin(ctx, 3 * steps + 4)
    t0 = time.perf_counter()
    ev0.record(stream)
    md.md_step(ctx, q, p, f, DT, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    kernel_ms, kernel_launches, kernel_name = md.md_timing_end(ctx)
    e1 = md.md_energy(ctx, q, p).cpu().numpy()
    tiles = md.md_get_tiles(ctx)
    launch = LAUNCH_NAMES[md.md_get_launch(ctx)]
    sym_tile = md.md_get_sym_tile(ctx)
    ctx.close()
    pairs = 3.0 * N * N * steps
    return {
        "ms_total": ms, "wall_s": wall, "ms_per_step": ms / steps,
        "gpairs_per_s": pairs / (ms * 1e-3) / 1e9,
        "pair_launches": 3 * steps,
        "pair_ms_avg": ms / (3 * steps),  # one force evaluation: every kernel of it, and the gaps
        "kernel_ms_avg": kernel_ms / max(kernel_launches, 1), "kernel_launches": kernel_launches,
        "kernel_name": kernel_name,
        "E0": e0.tolist(), "E1": e1.tolist(),
        "dE_E": abs(e1[2] - e0[2]) / abs(e0[2]),
        "dE_KV": abs(e1[2] - e0[2]) / (abs(e0[0]) + abs(e0[1])),
        "tiles": list(tiles), "launch": launch, "sym_tile": sym_tile, "final_q": q, "final_p": p,
    }


def oracle_golden(n):
    """The FP64 oracle's energies along this run (tests/golden, written by
    tests/golden/make_grav2d_golden.py from the oracle alone), or None."""
    path = os.path.join(GOLDEN_DIR, f"grav2d_disk_seed3_n{n}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        g = json.load(fh)
    if g["n"] != n or g["seed"] != SEED or g["eps"] != EPS or g["dt"] != DT or g["sigma"] != SIGMA:
        return None
    return g


def gate_run(md, torch, prec, q0, p0, golden):
    """Untimed: the run from the initial state in chunks of the golden's report
    interval, md_energy at every report time; returns the energies [times][K, V, E]."""
    import numpy as np
    ctx = md.md_init(md.GRAV2D, prec, N, EPS)
    q, p = torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda()
    f = torch.empty_like(q)
    md.md_force(ctx, q, f)
    E = [md.md_energy(ctx, q, p).cpu().numpy()]
    for s0, s1 in zip(golden["steps"][:-1], golden["steps"][1:]):
        md.md_step(ctx, q, p, f, DT, s1 - s0)
        E.append(md.md_energy(ctx, q, p).cpu().numpy())
    ctx.close()
    return np.array(E)


def oracle_gate(md, torch, q0, p0, golden, precs):
    """Energies of each precision form against the oracle's at every report time
    (relative energy error of Sec. 4, against |E0| and against K0 + |V0|)."""
    import numpy as np
    Eo = np.array([golden["K"], golden["V"], golden["E"]]).T
    E0, KV0 = abs(Eo[0, 2]), abs(Eo[0, 0]) + abs(Eo[0, 1])
    out = {"report_steps": golden["steps"], "oracle_E0": Eo[0].tolist(),
           "oracle_max_dE_E0": float(np.abs(Eo[:, 2] - Eo[0, 2]).max() / E0)}
    for name, prec in precs:
        log(f"bench: oracle gate {name} ({golden['steps'][-1]} steps, energies every {golden['every']})")
        E = gate_run(md, torch, prec, q0, p0, golden)
        d = np.abs(E[:, 2] - Eo[:, 2])
        out[name] = {"max_dE_vs_oracle_over_absE0": float(d.max() / E0),
                     "max_dE_vs_oracle_over_K0_plus_absV0": float(d.max() / KV0),
                     "E0_vs_oracle_over_K0_plus_absV0": float(np.abs(E[0] - Eo[0]).max() / KV0),
                     "max_dE_E0": float(np.abs(E[:, 2] - E[0, 2]).max() / E0),
                     "bar": GATE_BAR[name], "pass": bool(d.max() <= GATE_BAR[name] * E0)}
        log(f"bench: {name} vs oracle: max |E - E_oracle| / |E0| = {d.max() / E0:.2e} "
            f"(bar {GATE_BAR[name]:.0e}), / (K0+|V0|) = {d.max() / KV0:.2e}")
    return out


def cpu_baseline(q0, target_s: float = 10.0):
    """FP64 oracle pair throughput on sampled force rows of the same configuration."""
    import numpy as np

    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    oracle.set_threads(threads)
    used = oracle.get_threads()
    rng = np.random.default_rng(0)
    rows = rng.choice(N, size=32, replace=False)
    t0 = time.perf_counter()
    oracle.force_rows(oracle.GRAV2D, q0, rows, EPS)
    dt = time.perf_counter() - t0
    nrows = int(min(N, max(32, 32 * target_s / max(dt, 1e-6))))
    rows = rng.choice(N, size=nrows, replace=False)
    t0 = time.perf_counter()
    oracle.force_rows(oracle.GRAV2D, q0, rows, EPS)
    dt = time.perf_counter() - t0
    return {
        "value": nrows * N / dt / 1e9, "unit": "Gpair-interactions/s", "cores": used, "kind": "oracle",
        "sample": f"one FP64 force evaluation on {nrows} sampled rows x {N} particles "
                  f"({nrows * N:.3e} pairs, {dt:.1f} s, {used} threads)",
    }


HMF_N = 10_000_000
HMF_DT = 0.1
HMF_BYTES = {"fp64": 96, "f32state": 48}   # per particle-step: 3 passes x (read + write of theta, p)
RING_N = 2048
RING_EPS = 0.01
RING_DT = 0.05
RING_FLOPS_PER_PAIR = 11          # eq. 9 in FP64, plus one rsqrt
RING_FP64_CYCLES_PER_PAIR = 12 * 4.6 + 16.0
LAUNCH_FLOOR_US = 1.55
kWAVE = 64
PEAK_HBM_GBS = 8000.0


def ring_workload(md, torch, args):
    """Ring model, N = 2048, eps = 0.01, dt = 0.05, waterbag (theta in [-pi/2, pi/2],
    p in [-0.5, 0.5], seed 1), FP64 and mixed."""
    import numpy as np

    from paper_1212_0262_amd import inputs
    q0, p0 = inputs.ring_waterbag(RING_N, seed=1)
    res = {}
    for name, prec in (("fp64", md.FP64), ("mixed", md.MIXED)):
        ctx = md.md_init(md.RING, prec, RING_N, RING_EPS)
        q = torch.from_numpy(q0).cuda()
        p = torch.from_numpy(p0).cuda()
        f = torch.empty_like(q)
        e0 = md.md_energy(ctx, q, p).cpu().numpy()
        md.md_force(ctx, q, f)
        qw, pw, fw = q.clone(), p.clone(), f.clone()
        md.md_step(ctx, qw, pw, fw, RING_DT, max(1, args.warmup))
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        md.md_step(ctx, q, p, f, RING_DT, args.steps)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        e1 = md.md_energy(ctx, q, p).cpu().numpy()
        # the pair (fused) kernel's own launches, timed by the library over the same
        # steps run again from the warm-up state: its events add a few us to each
        # launch of a ~10 us kernel, so this run is not the one the throughput is from
        qk, pk, fk = qw.clone(), pw.clone(), fw.clone()
        torch.cuda.synchronize()
        md.md_timing_begin(ctx, 3 * args.steps + 4)
        ev0.record()
        md.md_step(ctx, qk, pk, fk, RING_DT, args.steps)
        ev1.record()
        torch.cuda.synchronize()
        ms_timed = ev0.elapsed_time(ev1)
        k_ms, k_n, k_name = md.md_timing_end(ctx)
        # the same steps captured as one HIP graph (launch-bound at this N)
        qg, pg, fg = qw.clone(), pw.clone(), fw.clone()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        md.md_set_stream(ctx, s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            md.md_step(ctx, qg, pg, fg, RING_DT, args.steps)
        md.md_set_stream(ctx, torch.cuda.current_stream())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ev0.record()
        g.replay()
        ev1.record()
        torch.cuda.synchronize()
        graph_ms = ev0.elapsed_time(ev1)
        res_graph = {"graph_us_per_step": 1e3 * graph_ms / args.steps,
                     "graph_gpairs_per_s": 3.0 * RING_N ** 2 * args.steps / (graph_ms * 1e-3) / 1e9}
        form = "fused" if md.md_get_launch(ctx) == md.LAUNCH_FUSED else "staged"
        # the other launch form on the same tiles (pair kernel + update kernel per force)
        md.md_set_launch(ctx, md.LAUNCH_STAGED)
        qs, ps, fs = qw.clone(), pw.clone(), fw.clone()
        md.md_step(ctx, qs, ps, fs, RING_DT, 2)
        torch.cuda.synchronize()
        ev0.record()
        md.md_step(ctx, qs, ps, fs, RING_DT, args.steps)
        ev1.record()
        torch.cuda.synchronize()
        staged_ms = ev0.elapsed_time(ev1)
        res[name] = {"ms": ms, "us_per_step": 1e3 * ms / args.steps, **res_graph, "launch": form,
                     "us_per_step_with_kernel_events": 1e3 * ms_timed / args.steps,
                     "kernel_timed_as": k_name, "kernel_us_avg": 1e3 * k_ms / max(k_n, 1), "kernel_launches": k_n,
                     "staged_us_per_step": 1e3 * staged_ms / args.steps,
                     "gpairs_per_s": 3.0 * RING_N ** 2 * args.steps / (ms * 1e-3) / 1e9,
                     "dE_E": float(abs(e1[2] - e0[2]) / abs(e0[2])), "tiles": list(md.md_get_tiles(ctx))}
        ctx.close()
    cpu = None
    if not args.no_cpu:
        import oracle
        oracle.set_threads(1)
        t0 = time.perf_counter()
        nst = 2
        f = oracle.force(oracle.RING, q0, RING_EPS)
        oracle.step(oracle.RING, q0, p0, f, RING_DT, nst, RING_EPS)
        dt = time.perf_counter() - t0
        cpu = {"value": (3 * nst + 1) * RING_N ** 2 / dt / 1e9, "unit": "Gpair-interactions/s", "cores": 1,
               "kind": "oracle", "sample": f"{nst} FP64 Yoshida steps of the full N={RING_N} system, 1 thread"}
    fp = res["fp64"]
    # roofline of the FP64 pair (fused) kernel: 11 flops + 1 rsqrt per ordered pair (eq. 9:
    # 3 for the numerator, 4 for 1 + eps - cos d, 2 for the cube, 2 to accumulate); at
    # this N it is bound by latency, so the kernel time is set beside two floors: the
    # VALU floor of its instruction mix (12 FP64 VALU of 4.6 cycles + v_rsq_f64 of 16
    # cycles per pair and wavefront, measured costs) and the gap between back-to-back
    # launches (1.55 us measured for empty kernels)
    k_s = fp["kernel_us_avg"] * 1e-6
    tf = RING_FLOPS_PER_PAIR * RING_N ** 2 / k_s / 1e12
    valu_floor_us = RING_N ** 2 * RING_FP64_CYCLES_PER_PAIR / kWAVE / SIMD_CYCLES_PER_S * 1e6
    roof = {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": None,
            "kernel": fp["kernel_timed_as"], "kernel_us_avg": round(fp["kernel_us_avg"], 3),
            "kernel_launches": fp["kernel_launches"], "flops_per_pair": RING_FLOPS_PER_PAIR,
            "pairs_per_launch": RING_N ** 2,
            "latency": {"evaluation_us": round(fp["kernel_us_avg"], 3), "valu_floor_us": round(valu_floor_us, 3),
                        "launch_floor_us": LAUNCH_FLOOR_US,
                        "step_us_eager": round(fp["us_per_step"], 3),
                        "step_us_graph": round(fp["graph_us_per_step"], 3),
                        "evaluations_per_step": 3}}
    return {
        "metric": "Gpair-interactions/s (Ring N=2048, FP64)", "value": round(fp["gpairs_per_s"], 3),
        "unit": "Gpair-interactions/s", "ms_per_step": round(fp["us_per_step"] / 1e3, 5), "dtype": "f64",
        "config": {"workload": "ring waterbag N=2048 eps=0.01 dt=0.05 seed=1", "model": "ring", "n": RING_N,
                   "eps": RING_EPS, "dt": RING_DT, "precision": "fp64", "tiles": fp["tiles"]},
        "roofline": roof, "cpu_baseline": cpu, "ring": res,
    }


def hmf_workload(md, torch, args):
    """HMF, N = 10^7, waterbag theta in [-1, 1], p in [-1.2, 1.2] (seed 2), dt = 0.1:
    FP64 and FP32 state with FP64 magnetization; HBM-bound."""
    from paper_1212_0262_amd import inputs
    q0, p0 = inputs.hmf_waterbag(HMF_N, seed=2)
    res = {}
    for name, prec in (("fp64", md.FP64), ("f32state", md.MIXED_F32STATE)):
        ctx = md.md_init(md.HMF, prec, HMF_N, 0.0)
        q = torch.from_numpy(q0).cuda()
        p = torch.from_numpy(p0).cuda()
        f = torch.empty_like(q)
        e0 = md.md_energy(ctx, q, p).cpu().numpy()
        md.md_force(ctx, q, f)
        qw, pw, fw = q.clone(), p.clone(), f.clone()
        md.md_step(ctx, qw, pw, fw, HMF_DT, max(1, args.warmup))
        del qw, pw, fw
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        md.md_step(ctx, q, p, f, HMF_DT, args.steps)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        e1 = md.md_energy(ctx, q, p).cpu().numpy()
        # the stage passes, timed by the library over the same number of steps run
        # again (its events add to each ~60 us pass, so the throughput is not from
        # this run)
        qk, pk, fk = q.clone(), p.clone(), f.clone()
        torch.cuda.synchronize()
        md.md_timing_begin(ctx, 3 * args.steps + 4)
        ev0.record()
        md.md_step(ctx, qk, pk, fk, HMF_DT, args.steps)
        ev1.record()
        torch.cuda.synchronize()
        ms_timed = ev0.elapsed_time(ev1)
        pass_ms, passes, pass_name = md.md_timing_end(ctx)
        del qk, pk, fk
        ps = HMF_N * args.steps / (ms * 1e-3)
        pass_GBs = HMF_N * HMF_BYTES[name] / 3 / (pass_ms / passes * 1e-3) / 1e9
        res[name] = {"ms": ms, "ms_per_step": ms / args.steps, "particle_steps_per_s": ps,
                     "ms_per_step_with_pass_events": ms_timed / args.steps,
                     "algorithmic_GBs": ps * HMF_BYTES[name] / 1e9,
                     "pass_ms_avg": pass_ms / passes, "passes_timed": passes, "pass_timed_as": pass_name,
                     "pass_algorithmic_GBs": pass_GBs,
                     "dE_E": float(abs(e1[2] - e0[2]) / abs(e0[2]))}
        ctx.close()
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        oracle.set_threads(threads)
        nst = 3
        f = oracle.force(oracle.HMF, q0)
        t0 = time.perf_counter()
        oracle.step(oracle.HMF, q0, p0, f, HMF_DT, nst)
        dt = time.perf_counter() - t0
        cpu = {"value": HMF_N * nst / dt, "unit": "particle-steps/s", "cores": oracle.get_threads(),
               "kind": "oracle", "sample": f"{nst} FP64 Yoshida steps of the full N=1e7 system"}
    fp = res["fp64"]
    return {
        "metric": "particle-steps/s (HMF N=1e7, FP64)", "value": round(fp["particle_steps_per_s"], 1),
        "unit": "particle-steps/s", "ms_per_step": round(fp["ms_per_step"], 5), "dtype": "f64",
        "config": {"workload": "hmf waterbag N=1e7 dt=0.1 seed=2", "model": "hmf", "n": HMF_N, "dt": HMF_DT,
                   "precision": "fp64"},
        # the stage pass's own launches (timed by the library), 32 bytes per particle each
        "roofline": {"bound": "hbm", "achieved": round(fp["pass_algorithmic_GBs"], 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(fp["pass_algorithmic_GBs"] / PEAK_HBM_GBS, 4),
                     "traffic": hmf_traffic_from_profile(),
                     "kernel": "k_hmf_pass<double, 2, false>", "kernel_timed_as": fp["pass_timed_as"],
                     "kernel_ms_avg": round(fp["pass_ms_avg"], 5), "bytes_per_launch": HMF_N * HMF_BYTES["fp64"] // 3,
                     "step_GBs": round(fp["algorithmic_GBs"], 1),
                     "bytes_per_particle_step": HMF_BYTES["fp64"]},
        "cpu_baseline": cpu, "hmf": res,
    }


ENS_NB = 256
ENS_EPS = 0.01
ENS_DT = 0.05
ENS_SYM_KAHAN_FLOPS = 21      # half-angle Ring term 11 (+ rsqrt), two compensated adds of 5
ENS_STAGED_KAHAN_FLOPS = 16   # term 11 (+ rsqrt), one compensated add


def ensemble_workload(md, torch, args):
    """Ring ensemble: 256 realizations, N_b = round(exp(U(ln 1000, ln 16384))) (seed 4),
    waterbag ICs per realization (seeded [4, b]), eps = 0.01, dt = 0.05, FP32 pairs
    with Kahan-compensated accumulation, md_step's automatic launch form (symmetric
    here; the staged form with autotuned tiles timed beside it); the whole run
    replayed as one captured HIP graph."""
    import numpy as np

    from paper_1212_0262_amd import autotune, inputs
    sizes = inputs.ensemble_sizes(ENS_NB, seed=4)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    parts = [inputs.ensemble_member(b, int(n), seed=4) for b, n in enumerate(sizes)]
    q0 = np.concatenate([a for a, _ in parts], axis=1)
    p0 = np.concatenate([b for _, b in parts], axis=1)
    pairs_per_eval = float((sizes.astype(np.float64) ** 2).sum())
    prec = md.MIXED_KAHAN
    stream = torch.cuda.Stream()
    torch.cuda.current_stream().wait_stream(stream)
    ctx = md.md_batch_init(md.RING, prec, off, ENS_EPS, stream=stream)
    q = torch.from_numpy(q0).cuda()
    p = torch.from_numpy(p0).cuda()
    f = torch.empty_like(q)
    torch.cuda.synchronize()
    default_tiles = md.md_get_tiles(ctx)
    # the staged form's tiles, tuned (the symmetric form has no tile choice)
    md.md_set_launch(ctx, md.LAUNCH_STAGED)
    with torch.cuda.stream(stream):
        t_default = autotune.time_step(ctx, q)
        best, table = autotune.tune(ctx, q, cache=None)
    md.md_set_launch(ctx, md.LAUNCH_AUTO)
    launch = LAUNCH_NAMES[md.md_get_launch(ctx)]
    with torch.cuda.stream(stream):
        t_auto = autotune.time_step(ctx, q)
    log(f"bench: ensemble staged tiles default {default_tiles} {t_default:.3f} ms/step, tuned {best} "
        f"{table[0][1]:.3f} ms/step; automatic form {launch} {t_auto:.3f} ms/step")
    with torch.cuda.stream(stream):
        e0 = md.md_energy(ctx, q, p).cpu().numpy()
        md.md_force(ctx, q, f)
        # eager run on copies (also the warm-up)
        qe, pe, fe = q.clone(), p.clone(), f.clone()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        md.md_timing_begin(ctx, 3 * args.steps + 4)  # the dominant (tile-pair) kernel's launches
        ev0.record(stream)
        md.md_step(ctx, qe, pe, fe, ENS_DT, args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        eager_ms = ev0.elapsed_time(ev1)
        k_ms, k_n, k_name = md.md_timing_end(ctx)
        # capture the whole run as one graph on the real buffers, then replay it once (timed)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            md.md_step(ctx, q, p, f, ENS_DT, args.steps)
        torch.cuda.synchronize()
        ev0.record(stream)
        g.replay()
        ev1.record(stream)
        torch.cuda.synchronize()
        graph_ms = ev0.elapsed_time(ev1)
        e1 = md.md_energy(ctx, q, p).cpu().numpy()
        same = bool(torch.equal(q, qe) and torch.equal(p, pe))
    dE = np.abs(e1[:, 2] - e0[:, 2]) / np.abs(e0[:, 2])
    pairs = 3.0 * pairs_per_eval * args.steps
    # the same run in FP64 and in plain mixed (eager): the integrator's own energy
    # error, and what each FP32 form adds to it, per realization
    ref = {}
    for name, pr in (("fp64", md.FP64), ("mixed", md.MIXED)):
        c2 = md.md_batch_init(md.RING, pr, off, ENS_EPS, stream=stream)
        with torch.cuda.stream(stream):
            q2 = torch.from_numpy(q0).cuda()
            p2 = torch.from_numpy(p0).cuda()
            f2 = torch.empty_like(q2)
            md.md_force(c2, q2, f2)
            torch.cuda.synchronize()
            ev0.record(stream)
            md.md_step(c2, q2, p2, f2, ENS_DT, args.steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            ref[name] = {"ms": ev0.elapsed_time(ev1), "E1": md.md_energy(c2, q2, p2).cpu().numpy(),
                         "tiles": list(md.md_get_tiles(c2)), "launch": LAUNCH_NAMES[md.md_get_launch(c2)]}
        c2.close()
        del q2, p2, f2
    e64 = ref["fp64"]["E1"]
    prec_err = np.abs(e1[:, 2] - e64[:, 2]) / np.abs(e0[:, 2])
    prec_err_mixed = np.abs(ref["mixed"]["E1"][:, 2] - e64[:, 2]) / np.abs(e0[:, 2])
    dE64 = np.abs(e64[:, 2] - e0[:, 2]) / np.abs(e0[:, 2])
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        oracle.set_threads(threads)
        small = np.argsort(sizes)[:8]
        t0 = time.perf_counter()
        npairs = 0.0
        for b in small:
            qb, pb = q0[:, off[b]:off[b + 1]], p0[:, off[b]:off[b + 1]]
            fo = oracle.force(oracle.RING, qb, ENS_EPS)
            oracle.step(oracle.RING, qb, pb, fo, ENS_DT, 2, ENS_EPS)
            npairs += 7.0 * float(sizes[b]) ** 2
        dt = time.perf_counter() - t0
        cpu = {"value": npairs / dt / 1e9, "unit": "Gpair-interactions/s", "cores": oracle.get_threads(),
               "kind": "oracle", "sample": "force + 2 FP64 Yoshida steps of the 8 smallest realizations"}
    tile = md.md_get_sym_tile(ctx) or ENS_SYM_TILE
    ctx.close()
    # roofline of the symmetric kernel (Kahan; one launch per force evaluation): the pairs
    # of particles in different tiles of a realization, each evaluated once for both (11
    # flops + 1 rsqrt for the half-angle term, 5 for each of the two compensated adds),
    # and the ordered pairs within each tile, i side only (11 + 5)
    tile_pairs = diag_pairs = 0.0
    for nb_ in sizes.astype(np.int64):
        t = np.full(-(-int(nb_) // tile), tile, dtype=np.float64)
        t[-1] = nb_ - tile * (len(t) - 1)
        tile_pairs += (float(nb_) ** 2 - float((t * t).sum())) / 2
        diag_pairs += float((t * t).sum())
    k_s = k_ms / max(k_n, 1) * 1e-3
    sym = launch == "symmetric"
    flops = (ENS_SYM_KAHAN_FLOPS * tile_pairs + ENS_STAGED_KAHAN_FLOPS * diag_pairs) if sym \
        else (ENS_STAGED_KAHAN_FLOPS * pairs_per_eval)
    tf = flops / k_s / 1e12
    roof = {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / PEAK_FP32_TFLOPS, 4), "traffic": None, "kernel_timed_as": k_name,
            "kernel_ms_avg": round(k_ms / max(k_n, 1), 4), "kernel_launches": k_n,
            "flops_per_launch": flops,
            "evaluations_per_launch": (tile_pairs + diag_pairs) if sym else pairs_per_eval,
            "flops_per_evaluation": {"tile pairs (both particles)": ENS_SYM_KAHAN_FLOPS,
                                     "diagonal tiles (i side)": ENS_STAGED_KAHAN_FLOPS} if sym
            else ENS_STAGED_KAHAN_FLOPS}
    return {
        "metric": "Gpair-interactions/s (Ring ensemble, 256 realizations, graph-replayed)",
        "value": round(pairs / (graph_ms * 1e-3) / 1e9, 3), "unit": "Gpair-interactions/s",
        "ms_per_step": round(graph_ms / args.steps, 4), "dtype": "f32",
        "config": {"workload": "ring ensemble nb=256 N_b log-uniform [1000,16384] seed=4 eps=0.01 dt=0.05",
                   "model": "ring", "nb": ENS_NB, "n_total": int(off[-1]), "pairs_per_eval": pairs_per_eval,
                   "precision": "mixed_kahan", "launch": launch, "staged_tiles_tuned": list(best),
                   "staged_tiles_default": list(default_tiles)},
        "roofline": roof, "cpu_baseline": cpu,
        "ensemble": {"graph_ms": graph_ms, "eager_ms": eager_ms, "graph_equals_eager": same,
                     "step_ms": t_auto, "staged_step_ms_default_tiles": t_default,
                     "staged_step_ms_tuned": table[0][1], "speedup_vs_tuned_staged": table[0][1] / t_auto,
                     "staged_tune_table_top5": [[list(t), ms] for t, ms in table[:5]],
                     "dE_E_max": float(dE.max()), "dE_E_median": float(np.median(dE)),
                     "fp64_dE_E_max": float(dE64.max()), "fp64_dE_E_median": float(np.median(dE64)),
                     "kahan_vs_fp64_energy_diff_over_absE0_max": float(prec_err.max()),
                     "gate_kahan_vs_fp64_le_1e-5": bool(prec_err.max() <= 1e-5),
                     "mixed_vs_fp64_energy_diff_over_absE0_max": float(prec_err_mixed.max()),
                     "fp64_gpairs_per_s": pairs / (ref["fp64"]["ms"] * 1e-3) / 1e9,
                     "mixed_gpairs_per_s": pairs / (ref["mixed"]["ms"] * 1e-3) / 1e9,
                     "fp64_launch": ref["fp64"]["launch"], "mixed_launch": ref["mixed"]["launch"],
                     "fp64_tiles": ref["fp64"]["tiles"], "mixed_tiles": ref["mixed"]["tiles"]},
    }


ADJ_N = 32_768
ADJ_EPS = 1e-3
ADJ_DT = 0.01
ADJ_CKPT = 50
ADJ_HVP_FLOPS = 22          # per ordered pair (staged product; diagonal tiles of the symmetric one)
ADJ_HVP_SYM_FLOPS = 30      # per pair of a tile pair (symmetric product: the j side's four FMAs more)


def adjoint_workload(md, torch, args):
    """2D gravity adjoint: N = 32768, eps = 1e-3, uniform disk (seed 5), dt = 0.01,
    1000 steps with checkpoints every 50: gradient of the final kinetic energy with
    respect to (x, y, px, py) at t = 0 through md_step_vjp (FP64), checked against
    FP64 central differences of the forward map along 16 random unit directions
    (seeded [5, k])."""
    import numpy as np

    from paper_1212_0262_amd import autograd as mdgrad
    from paper_1212_0262_amd import inputs
    q0, p0 = inputs.grav2d_disk(ADJ_N, seed=5)
    ctx = md.md_init(md.GRAV2D, md.FP64, ADJ_N, ADJ_EPS)
    qd, pd = torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda()
    nst = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    K, gq, gp = mdgrad.kinetic_energy_gradient(ctx, qd, pd, ADJ_DT, nst, ADJ_CKPT)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0

    # the same gradient with every kick position recorded (no recomputation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Kr, gqr, gpr = mdgrad.kinetic_energy_gradient(ctx, qd, pd, ADJ_DT, nst, 0)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    rec_same = bool(torch.equal(gqr, gq) and torch.equal(gpr, gp) and float(Kr) == float(K))
    rec_bytes = md.md_record_stage_bytes(ctx, nst)
    del gqr, gpr
    log(f"bench: adjoint gradient {t_grad:.3f} s (checkpoints every {ADJ_CKPT}), {t_rec:.3f} s recorded "
        f"({rec_bytes / 2**30:.2f} GiB), identical: {rec_same}")

    def J(q, p):
        qq, pp = torch.from_numpy(q).cuda(), torch.from_numpy(p).cuda()
        f = torch.empty_like(qq)
        md.md_force(ctx, qq, f)
        md.md_step(ctx, qq, pp, f, ADJ_DT, nst)
        return 0.5 * float((pp * pp).sum())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J0 = J(q0, p0)
    t_fwd = time.perf_counter() - t0
    gq, gp = gq.cpu().numpy(), gp.cpu().numpy()
    dirs = []
    for k in range(16):
        rng = np.random.default_rng([5, k])
        v = rng.normal(size=(4, ADJ_N))
        v /= np.linalg.norm(v)
        dirs.append(v)
    # step size: sweep on the first direction
    sweep = {}
    v = dirs[0]
    ad0 = float(np.sum(gq * v[:2]) + np.sum(gp * v[2:]))
    for h in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
        fd = (J(q0 + h * v[:2], p0 + h * v[2:]) - J(q0 - h * v[:2], p0 - h * v[2:])) / (2 * h)
        sweep[h] = {"fd": fd, "rel_err": abs(ad0 - fd) / max(abs(fd), 1e-300)}
        log(f"bench: adjoint h={h:g} fd={fd:.10e} ad={ad0:.10e}")
    hbest = min(sweep, key=lambda k: sweep[k]["rel_err"])
    rel = []
    for v in dirs:
        ad = float(np.sum(gq * v[:2]) + np.sum(gp * v[2:]))
        fd = (J(q0 + hbest * v[:2], p0 + hbest * v[2:]) - J(q0 - hbest * v[:2], p0 - hbest * v[2:])) / (2 * hbest)
        rel.append(abs(ad - fd) / max(abs(fd), 1e-300))
    # roofline of the Hessian-vector product's pair kernel (FP64; 22 flops + 1 reciprocal
    # per ordered pair: r, |r|^2 + eps, w_i - w_j, r.(w_i - w_j)/s, 2 t/s, four accumulating FMAs;
    # the symmetric form, automatic at this N, evaluates each pair of a tile pair once with
    # the j side's four FMAs more, and every ordered pair of the diagonal tiles)
    wv = torch.from_numpy(np.random.default_rng(7).normal(size=(2, ADJ_N))).cuda()
    hv = torch.empty_like(qd)
    md.md_hvp(ctx, qd, wv, hv)
    torch.cuda.synchronize()
    md.md_timing_begin(ctx, 20)
    for _ in range(20):
        md.md_hvp(ctx, qd, wv, hv)
    torch.cuda.synchronize()
    k_ms, k_n, k_name = md.md_timing_end(ctx)
    k_s = k_ms / max(k_n, 1) * 1e-3
    if k_name == "k_hvp_sym":
        tile_pair_evals, diag_evals = sym_counts(ADJ_N, md.md_get_sym_tile(ctx))
        flops = ADJ_HVP_SYM_FLOPS * tile_pair_evals + ADJ_HVP_FLOPS * diag_evals
        per = {"tile_pair_evaluations_per_launch": tile_pair_evals, "diagonal_evaluations_per_launch": diag_evals,
               "flops_per_tile_pair_evaluation": ADJ_HVP_SYM_FLOPS, "flops_per_diagonal_evaluation": ADJ_HVP_FLOPS}
    else:
        flops = ADJ_HVP_FLOPS * ADJ_N ** 2
        per = {"flops_per_pair": ADJ_HVP_FLOPS, "pairs_per_launch": ADJ_N ** 2}
    tf = flops / k_s / 1e12
    roof = {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": None, "kernel_timed_as": k_name,
            "kernel_ms_avg": round(k_ms / max(k_n, 1), 4), "kernel_launches": k_n,
            "executed_flops_per_launch": flops, **per,
            "interaction_equivalent_tflops": round(ADJ_HVP_FLOPS * ADJ_N ** 2 / k_s / 1e12, 3)}
    ctx.close()
    cpu = None
    if not args.no_cpu:
        # the oracle's gradient at reduced N beside the GPU's (same map, FP64)
        import oracle
        oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
        n_s, st_s = 1024, 20
        qs, ps = inputs.grav2d_disk(n_s, seed=5)
        cs = md.md_init(md.GRAV2D, md.FP64, n_s, ADJ_EPS)
        _, gqs, gps = mdgrad.kinetic_energy_gradient(cs, torch.from_numpy(qs).cuda(), torch.from_numpy(ps).cuda(),
                                                     ADJ_DT, st_s, 5)
        cs.close()
        t0 = time.perf_counter()
        f = oracle.force(oracle.GRAV2D, qs, ADJ_EPS)
        _, pT, _ = oracle.step(oracle.GRAV2D, qs, ps, f, ADJ_DT, st_s, ADJ_EPS)
        oq, op = oracle.step_vjp(oracle.GRAV2D, qs, ps, ADJ_DT, st_s, np.zeros_like(qs), pT.copy(), ADJ_EPS)
        t_cpu = time.perf_counter() - t0
        g_gpu = np.concatenate([gqs.cpu().numpy().ravel(), gps.cpu().numpy().ravel()])
        g_cpu = np.concatenate([oq.ravel(), op.ravel()])
        cpu = {"value": round(t_cpu, 4), "unit": "s", "cores": oracle.get_threads(), "kind": "oracle",
               "sample": f"one FP64 gradient of K_T at N={n_s}, {st_s} steps (forward, then the reverse sweep)",
               "gpu_vs_oracle_gradient_rel_err": float(np.abs(g_gpu - g_cpu).max() / np.abs(g_cpu).max())}
        log(f"bench: adjoint oracle gradient N={n_s}: {t_cpu:.2f} s, GPU vs oracle "
            f"{cpu['gpu_vs_oracle_gradient_rel_err']:.2e}")
    pairs_fwd = 3.0 * ADJ_N ** 2 * nst
    return {
        "metric": "s per gradient of K_T w.r.t. (q0, p0) (2D adjoint N=32768, 1000 steps, FP64)",
        "value": round(t_grad, 4), "unit": "s", "ms_per_step": round(1e3 * t_grad / nst, 4), "dtype": "f64",
        "config": {"workload": "grav2d adjoint N=32768 eps=1e-3 dt=0.01 uniform disk seed=5, checkpoints every 50",
                   "model": "grav2d", "n": ADJ_N, "steps": nst, "checkpoint_every": ADJ_CKPT, "precision": "fp64"},
        "roofline": roof, "cpu_baseline": cpu,
        "adjoint": {"K_T": float(K), "forward_s": t_fwd, "gradient_s": t_grad,
                    "gradient_over_forward": t_grad / t_fwd,
                    "recorded_gradient_s": t_rec, "recorded_over_forward": t_rec / t_fwd,
                    "recorded_stage_bytes": rec_bytes, "recorded_equals_checkpointed": rec_same,
                    "forward_gpairs_per_s": pairs_fwd / t_fwd / 1e9,
                    "fd_step": hbest, "fd_sweep_dir0": {str(k): v for k, v in sweep.items()},
                    "rel_err_16_dirs_max": max(rel), "rel_err_16_dirs_median": float(np.median(rel)),
                    "grad_norm": float(np.sqrt(np.sum(gq * gq) + np.sum(gp * gp)))},
    }


def paper_errors_workload(md, torch, args):
    """The accuracy runs of Sec. 4: relative energy error eps(t) = |E(t) - E0|/|E0| of
    the CPU FP64 oracle, the GPU FP64 form and the GPU mixed form on the same
    initial state.  HMF and Ring spatially homogeneous at rest (theta ~ U(-pi, pi),
    p = 0), 2D uniform on the shell 1 <= r <= 1.5 at rest; dt = 0.1 (HMF) and
    0.005 (Ring, 2D), eps = 1e-3 (Ring, 2D).  The paper does not state N; the GPU
    runs use N = 10^6 (HMF) and 16384 (Ring, 2D); the oracle follows the same run
    for a bounded prefix (its cost grows as N^2)."""
    import numpy as np

    from paper_1212_0262_amd import inputs
    oracle = None
    if not args.no_cpu:
        import oracle
        oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    cpu_runs = {}
    runs = [("hmf", md.HMF, 1_000_000, 0.0, 0.1, 1000, 20, 200),
            ("ring", md.RING, 16384, 1e-3, 0.005, 2000, 20, 20),
            ("grav2d", md.GRAV2D, 16384, 1e-3, 0.005, 2000, 20, 40)]
    out = {}
    for name, model, n, eps, dt, nsteps, every, cpu_steps in runs:
        if model == md.GRAV2D:
            q0, p0 = inputs.shell_at_rest(n, seed=6)
        else:
            q0, p0 = inputs.homogeneous_at_rest(n, seed=6)
        curves = {}
        precs = [("gpu_fp64", md.FP64), ("gpu_mixed", md.MIXED_F32STATE if model == md.HMF else md.MIXED)]
        for label, prec in precs:
            ctx = md.md_init(model, prec, n, eps)
            q, p = torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda()
            f = torch.empty_like(q)
            md.md_force(ctx, q, f)
            es = [md.md_energy(ctx, q, p).cpu().numpy()]
            for _ in range(nsteps // every):
                md.md_step(ctx, q, p, f, dt, every)
                es.append(md.md_energy(ctx, q, p).cpu().numpy())
            curves[label] = np.array(es)
            ctx.close()
        E0 = float(curves["gpu_fp64"][0, 2])
        rel = {lab: np.abs(c[:, 2] - E0) / abs(E0) for lab, c in curves.items()}
        out[name] = {
            "n": n, "dt": dt, "eps": eps, "steps": nsteps, "report_every": every, "E0": E0,
            "K_end_gpu_fp64": float(curves["gpu_fp64"][-1, 0]),
            "max_rel_err": {lab: float(r.max()) for lab, r in rel.items()},
            "gpu_mixed_vs_gpu_fp64_max_dE_over_absE0": float(np.abs(curves["gpu_mixed"][:, 2]
                                                                    - curves["gpu_fp64"][:, 2]).max() / abs(E0)),
            "curve_t": [float(dt * every * i) for i in range(len(rel["gpu_fp64"]))][::5],
            "curve_gpu_fp64": [float(x) for x in rel["gpu_fp64"][::5]],
            "curve_gpu_mixed": [float(x) for x in rel["gpu_mixed"][::5]],
        }
        log(f"bench: paper errors {name}: max eps fp64 {out[name]['max_rel_err']['gpu_fp64']:.2e} "
            f"mixed {out[name]['max_rel_err']['gpu_mixed']:.2e}")
        if oracle is not None:
            # the CPU oracle on a bounded prefix of the same run, beside the GPU curves
            t0 = time.perf_counter()
            f = oracle.force(model, q0, eps)
            qo, po = q0, p0
            eo = [oracle.energy(model, qo, po, eps)]
            for _ in range(cpu_steps // every):
                qo, po, f = oracle.step(model, qo, po, f, dt, every, eps)
                eo.append(oracle.energy(model, qo, po, eps))
            cpu_s = time.perf_counter() - t0
            eo = np.array(eo)
            k = len(eo)
            cpu_runs[name] = {
                "steps": cpu_steps, "seconds": cpu_s,
                "max_rel_err_prefix": {"cpu_fp64": float((np.abs(eo[:, 2] - eo[0, 2]) / abs(eo[0, 2])).max()),
                                       **{lab: float(r[:k].max()) for lab, r in rel.items()}},
                "gpu_fp64_vs_cpu_max_dE_over_absE0": float(np.abs(curves["gpu_fp64"][:k, 2] - eo[:, 2]).max()
                                                           / abs(E0)),
                "gpu_mixed_vs_cpu_max_dE_over_absE0": float(np.abs(curves["gpu_mixed"][:k, 2] - eo[:, 2]).max()
                                                            / abs(E0)),
            }
    worst = max(v["gpu_mixed_vs_gpu_fp64_max_dE_over_absE0"] for v in out.values())
    return {
        "metric": "max |E_mixed - E_fp64| / |E0| over the paper's accuracy runs (HMF, Ring, 2D shell)",
        "value": worst, "unit": "relative", "ms_per_step": None, "dtype": "f64+f32",
        "config": {"workload": "accuracy runs of Sec. 4: homogeneous at rest (HMF, Ring), shell at rest (2D)"},
        "roofline": None,
        "cpu_baseline": None if oracle is None else {
            "value": round(sum(r["seconds"] for r in cpu_runs.values()), 3), "unit": "s",
            "cores": oracle.get_threads(), "kind": "oracle",
            "sample": "the same three runs on the CPU FP64 oracle for a bounded prefix (HMF 200, Ring 20, "
                      "2D 40 steps), energies at the same report times", "runs": cpu_runs},
        "paper_errors": out,
    }


def copy_calibration_workload(md, torch, args):
    """A plain device copy of known size, for the HBM-traffic counters: run it under
    rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE); the elementwise kernel reads and
    writes exactly 512 MiB per dispatch, so the counter per dispatch divided by
    that size is the factor that turns the counter into bytes for the library's
    kernels measured the same way."""
    mib, reps = 512, 3
    n = mib * (1 << 20) // 4
    src = torch.rand(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)  # one read and one write of n float32 values
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    gbs = 2 * mib * (1 << 20) / (ms * 1e-3) / 1e9
    return {"metric": "GB/s of a plain device copy (512 MiB read + 512 MiB written per dispatch)",
            "value": round(gbs, 1), "unit": "GB/s", "ms_per_step": round(ms, 4), "dtype": "f32",
            "config": {"workload": "copy calibration: torch.mul(src, 1.0, out=dst), 2^27 float32, 3 dispatches"},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None},
            "cpu_baseline": None}


def grav2d_workload(md, torch, args):
    import numpy as np

    from paper_1212_0262_amd import inputs
    q0, p0 = inputs.grav2d_disk(N, seed=SEED, sigma=SIGMA)

    log(f"bench: mixed N={N} steps={args.steps} warmup={args.warmup}")
    launch = {"auto": md.LAUNCH_AUTO, "staged": md.LAUNCH_STAGED, "symmetric": md.LAUNCH_SYMMETRIC}[args.launch]
    mixed = run_variant(md, torch, md.MIXED, q0, p0, args.steps, args.warmup, launch)
    log(f"bench: mixed {mixed['gpairs_per_s']:.1f} Gpairs/s, {mixed['ms_per_step']:.2f} ms/step, "
        f"dE/E={mixed['dE_E']:.2e}")
    K0, V0, E0 = mixed["E0"]
    if abs(E0) < 0.01 * (abs(K0) + abs(V0)):
        log(f"bench: warning: E0 = {E0:.6g} is {abs(E0) / (abs(K0) + abs(V0)):.2g} of K0 + |V0| "
            f"(K0 = {K0:.6g}, V0 = {V0:.6g}): |E - E0|/|E0| is ill-conditioned; see dE/(K0+|V0|)")
    fp64 = None
    if not args.no_fp64:
        log("bench: fp64")
        fp64 = run_variant(md, torch, md.FP64, q0, p0, args.steps, args.warmup)
        log(f"bench: fp64 {fp64['gpairs_per_s']:.1f} Gpairs/s, {fp64['ms_per_step']:.2f} ms/step, "
            f"dE/E={fp64['dE_E']:.2e}")
    variants = {}
    if fp64 is not None and not args.no_variants:
        # the other accumulations of the FP32 pair terms
        for name, prec in (("mixed_kahan", md.MIXED_KAHAN), ("mixed_pairf64", md.MIXED_PAIRF64)):
            log(f"bench: {name}")
            variants[name] = run_variant(md, torch, prec, q0, p0, args.steps, args.warmup)
            log(f"bench: {name} {variants[name]['gpairs_per_s']:.1f} Gpairs/s")
    staged = None
    if not args.no_variants and mixed["launch"] == "symmetric":
        # the staged form (each ordered pair evaluated) on the same steps, for comparison
        log("bench: mixed, staged launch")
        staged = run_variant(md, torch, md.MIXED, q0, p0, args.steps, args.warmup, md.LAUNCH_STAGED)
        log(f"bench: mixed staged {staged['gpairs_per_s']:.1f} Gpairs/s")
    golden = oracle_golden(N)
    gate = None
    if golden is not None:
        gate = oracle_gate(md, torch, q0, p0, golden,
                           [("mixed", md.MIXED)] + ([] if args.no_fp64 else [("fp64", md.FP64)]))
        if args.steps in golden["steps"]:  # the timed run itself, at its last step
            k = golden["steps"].index(args.steps)
            gate["timed_run_dE_vs_oracle_over_absE0"] = abs(mixed["E1"][2] - golden["E"][k]) / abs(golden["E"][0])
    cpu = None
    if not args.no_cpu:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(q0)
        log(f"bench: cpu {cpu['value']:.3f} Gpairs/s on {cpu['cores']} threads")

    # The dominant kernel's own launches, timed live by the library (HIP events on its stream).
    kernel_s = mixed["kernel_ms_avg"] * 1e-3
    if mixed["launch"] == "symmetric":
        # one launch per evaluation: each pair of two different tiles evaluated once for both
        # particles (14 flops), every ordered pair of a diagonal tile for its i side (10 flops,
        # the pads' included); it covers all N^2 interactions
        units = N * N
        evals_pairs, evals_diag = sym_counts(N, mixed["sym_tile"])
        evals = evals_pairs + evals_diag
        executed = SYM_FLOPS_PER_EVAL * evals_pairs + FLOPS_PER_PAIR * evals_diag
        kernel = f"k_sym<2, float, AccTile, {mixed['sym_tile'] // 256}> (tile pairs and diagonal tiles)"
        instr = {"valu_fp32": 8, "trans": 1, "per": "pair of a tile pair evaluated (both particles); "
                 "diagonal tiles 6 + 1 per ordered pair"}
    else:
        units = N * N
        evals = N * N
        executed = FLOPS_PER_PAIR * N * N
        kernel = "k_pair_2d<float, AccTile, ipl>"
        instr = {"valu_fp32": VALU_PER_PAIR, "trans": TRANS_PER_PAIR, "per": "pair"}
    interaction_tf = FLOPS_PER_PAIR * units / kernel_s / 1e12
    executed_tf = executed / kernel_s / 1e12
    evaluation_tf = FLOPS_PER_PAIR * N * N / (mixed["pair_ms_avg"] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(mixed["gpairs_per_s"], 3),
        "unit": "Gpair-interactions/s",
        "ms_per_step": round(mixed["ms_per_step"], 4),
        "dtype": "f32",
        "config": {
            "workload": "grav2d uniform disk N=262144 eps=1e-3 dt=0.01 sigma=0.5 seed=3 (mixed: FP32 pairs, "
                        "FP64 fold per j-tile)",
            "model": "grav2d", "n": N, "eps": EPS, "dt": DT, "precision": "mixed",
            "launch": mixed["launch"], "tiles_ipl_waves_jsplit_jtile": mixed["tiles"],
        },
        # achieved: the flops the kernel executes (the symmetric form evaluates each pair
        # once for both particles: 14 flops per evaluation), per launch / its live duration
        "roofline": {
            "bound": "alu", "achieved": round(executed_tf, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(executed_tf / PEAK_FP32_TFLOPS, 4),
            "traffic": traffic_from_profile(mixed["launch"], mixed["tiles"]),
            "kernel": kernel, "kernel_timed_as": mixed["kernel_name"],
            "kernel_ms_avg": round(mixed["kernel_ms_avg"], 4), "kernel_launches": mixed["kernel_launches"],
            "executed_flops_per_launch": executed, "pair_evaluations_per_launch": evals,
            "flops_per_evaluation": round(executed / max(evals, 1), 3),
            # the metric's convention: 10 flops per interaction (ordered pair) the launch covers
            "interaction_flops": FLOPS_PER_PAIR, "interactions_per_launch": units,
            "interaction_equivalent_tflops": round(interaction_tf, 3),
            "interaction_equivalent_frac": round(interaction_tf / PEAK_FP32_TFLOPS, 4),
            "instr_per_evaluation": instr,
            # SIMD cycles per interaction (pair of the N^2 count) and wavefront lane
            "cycles_per_pair_wave": round(SIMD_CYCLES_PER_S * 64 * kernel_s / units, 2),
            # one whole force evaluation (this kernel and the update) from the timed region
            "evaluation_ms": round(mixed["pair_ms_avg"], 4), "evaluation_tflops": round(evaluation_tf, 3),
            "evaluation_frac": round(evaluation_tf / PEAK_FP32_TFLOPS, 4),
        },
        "energy": {
            "mixed_dE_E": mixed["dE_E"], "mixed_dE_over_K0_plus_absV0": mixed["dE_KV"],
            "E0": mixed["E0"],
            # the accuracy gate: each form's energy against the FP64 oracle's at every report time
            "oracle_gate": gate if gate is not None else "no oracle golden for this N (tests/golden)",
            # E0 = K0 + V0 nearly cancels for this state (the log potential's mean over the disk
            # offsets the kinetic energy), which inflates |E - E0| / |E0|
            "E0_ill_conditioned": bool(abs(mixed["E0"][2]) < 0.01 * (abs(mixed["E0"][0]) + abs(mixed["E0"][1]))),
        },
        "cpu_baseline": cpu,
    }
    if staged is not None:
        out["mixed_staged"] = {
            "value": round(staged["gpairs_per_s"], 3), "ms_per_step": round(staged["ms_per_step"], 4),
            "tiles_ipl_waves_jsplit_jtile": staged["tiles"],
            "symmetric_speedup": round(mixed["gpairs_per_s"] / staged["gpairs_per_s"], 3),
            "energy_diff_vs_symmetric_over_absE0": abs(mixed["E1"][2] - staged["E1"][2]) / abs(staged["E0"][2]),
            "max_abs_dq_vs_symmetric": (mixed["final_q"] - staged["final_q"]).abs().max().item(),
        }
    if fp64 is not None:
        dq = (mixed["final_q"] - fp64["final_q"]).abs().max().item()
        dp = (mixed["final_p"] - fp64["final_p"]).abs().max().item()
        prec_err = abs(mixed["E1"][2] - fp64["E1"][2]) / abs(fp64["E0"][2])
        out["fp64"] = {
            "value": round(fp64["gpairs_per_s"], 3), "ms_per_step": round(fp64["ms_per_step"], 4),
            "dE_E": fp64["dE_E"], "dE_over_K0_plus_absV0": fp64["dE_KV"],
            "pair_tflops": round(FLOPS_PER_PAIR * N * N / (fp64["pair_ms_avg"] * 1e-3) / 1e12, 3),
            "frac_fp64_peak": round(FLOPS_PER_PAIR * N * N / (fp64["pair_ms_avg"] * 1e-3) / 1e12
                                    / PEAK_FP64_TFLOPS, 4),
            "kernel_timed_as": fp64["kernel_name"], "kernel_ms_avg": round(fp64["kernel_ms_avg"], 4),
        }
        out["mixed_vs_fp64"] = {
            "speedup": round(mixed["gpairs_per_s"] / fp64["gpairs_per_s"], 3),
            "energy_diff_over_absE0": prec_err,
            "energy_diff_over_K0_plus_absV0": abs(mixed["E1"][2] - fp64["E1"][2])
            / (abs(fp64["E0"][0]) + abs(fp64["E0"][1])),
            "max_abs_dq": dq, "max_abs_dp": dp,
        }
        # beside the oracle gate: the energy difference the mixed form makes to the GPU's FP64 run
        out["energy"]["mixed_vs_gpu_fp64_dE_over_E0_le_1e-5"] = bool(prec_err <= 1e-5)
        out["accumulation_variants"] = {
            "mixed_tile_fold": {"value": round(mixed["gpairs_per_s"], 3), "launch": mixed["launch"],
                                "energy_diff_over_absE0": prec_err, "gate_le_1e-5": bool(prec_err <= 1e-5)}}
        for name, v in variants.items():
            err = abs(v["E1"][2] - fp64["E1"][2]) / abs(fp64["E0"][2])
            out["accumulation_variants"][name] = {
                "value": round(v["gpairs_per_s"], 3), "ms_per_step": round(v["ms_per_step"], 4),
                "launch": v["launch"], "kernel_timed_as": v["kernel_name"],
                "kernel_ms_avg": round(v["kernel_ms_avg"], 4),
                "pair_tflops": round(FLOPS_PER_PAIR * N * N / (v["pair_ms_avg"] * 1e-3) / 1e12, 3),
                "dE_E": v["dE_E"], "energy_diff_over_absE0": err, "gate_le_1e-5": bool(err <= 1e-5),
                "max_abs_dq_vs_fp64": (v["final_q"] - fp64["final_q"]).abs().max().item()}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: 100 grav2d, 50 ring, 1000 hmf)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["grav2d", "ring", "hmf", "ensemble", "adjoint", "paper_errors",
                                           "copy_calibration"],
                    default="grav2d")
    ap.add_argument("--no-fp64", action="store_true", help="grav2d: skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true",
                    help="grav2d: skip the Kahan and per-pair FP64 accumulation runs and the staged-form timing")
    ap.add_argument("--launch", choices=["auto", "staged", "symmetric"], default="auto",
                    help="grav2d: launch form of the mixed run (auto: symmetric at this N)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; run it with --gpus 1",
              file=sys.stderr)
        return 2
    if args.steps is None:
        args.steps = {"grav2d": 100, "ring": 50, "hmf": 1000, "ensemble": 200, "adjoint": 1000,
                      "paper_errors": 0, "copy_calibration": 3}[args.workload]

    import torch

    from paper_1212_0262_amd import md

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    md.load()
    fn = {"grav2d": grav2d_workload, "ring": ring_workload, "hmf": hmf_workload,
          "ensemble": ensemble_workload, "adjoint": adjoint_workload,
          "paper_errors": paper_errors_workload, "copy_calibration": copy_calibration_workload}[args.workload]
    out = fn(md, torch, args)
    hib = out["unit"] not in ("s", "relative")
    line = {"metric": out.pop("metric"), "value": out.pop("value"), "unit": out.pop("unit"), "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": out.pop("ms_per_step"),
            "higher_is_better": hib, "scaling": "weak", "vs_baseline": None, "dtype": out.pop("dtype"),
            "data": "synthetic"}
    line.update(out)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
