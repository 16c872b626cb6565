"""Helpers for the GPU parity tests: move seeded host states to the device, run
libmd through its C ABI, and bring results back as numpy."""
from __future__ import annotations

import math

import numpy as np
import torch

from paper_1212_0262_amd import md

DEV = "cuda:0"


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def gpu_force(model, prec, q, eps, tiles=None):
    n = q.shape[-1]
    ctx = md.md_init(model, prec, n, eps)
    if tiles:
        md.md_set_tiles(ctx, *tiles)
    qd = dev(q)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    out = host(f)
    ctx.close()
    return out


def gpu_run(model, prec, q, p, eps, dt, nsteps, tiles=None, chunks=1):
    """md_force then nsteps Yoshida steps (in `chunks` calls); returns (q, p, f, energies-per-chunk)."""
    n = q.shape[-1]
    ctx = md.md_init(model, prec, n, eps)
    if tiles:
        md.md_set_tiles(ctx, *tiles)
    qd, pd = dev(q), dev(p)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    energies = [host(md.md_energy(ctx, qd, pd))]
    per = nsteps // chunks
    for c in range(chunks):
        k = per if c < chunks - 1 else nsteps - per * (chunks - 1)
        md.md_step(ctx, qd, pd, f, dt, k)
        energies.append(host(md.md_energy(ctx, qd, pd)))
    out = host(qd), host(pd), host(f), np.array(energies)
    ctx.close()
    return out


def gpu_energy(model, q, p, eps):
    ctx = md.md_init(model, md.FP64, q.shape[-1], eps)
    e = host(md.md_energy(ctx, dev(q), dev(p)))
    ctx.close()
    return e


def rel_inf(a, b):
    """max|a - b| / max|b| (max|b| floored at 1e-300)."""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def angle_diff(a, b):
    """a - b mapped to (-pi, pi]."""
    d = np.asarray(a) - np.asarray(b)
    return d - 2 * math.pi * np.round(d / (2 * math.pi))
