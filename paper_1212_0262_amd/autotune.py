"""Tile autotuner for the pair kernels of libmd.

Times one ``md_step`` with dt = 0 (every kernel of a step runs; the state does not
change) for a set of tile configurations (i_per_lane, waves, j_split, j_tile) of a
context on its actual input -- so each configuration is timed in the launch form
``md_step`` takes with it (staged or fused) -- keeps the fastest, and caches the
choice in a JSON file keyed by the device architecture, model, precision and the
problem's shape (N, or the realization sizes of a batch), so a later run can apply
it with :func:`apply_cached` without timing again.

All configurations compute the same sums in different orders, so the choice
changes results only at rounding level; it never changes what is computed.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
from typing import Iterable, Optional

import torch

from . import md

# The cache lives outside the package: $MD_TILES_CACHE, else ~/.cache/mdgpu/tiles_cache.json.
DEFAULT_CACHE = os.environ.get("MD_TILES_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "mdgpu",
                                                                  "tiles_cache.json")


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def shape_key(ctx: md.Context) -> str:
    """Cache key: arch / model / precision / problem shape."""
    if hasattr(ctx, "offsets"):
        sizes = (ctx.offsets[1:] - ctx.offsets[:-1]).astype("int64")
        shape = "batch-" + hashlib.sha256(sizes.tobytes()).hexdigest()[:16] + f"-nb{len(sizes)}"
    else:
        shape = f"n{ctx.n}"
    return f"{_arch()}/{md.MODEL_NAMES[ctx.model]}/{md.PREC_NAMES[ctx.prec]}/{shape}"


def candidates(ctx: md.Context) -> list:
    """Tile configurations worth timing for this context."""
    if hasattr(ctx, "offsets"):
        nmax = int((ctx.offsets[1:] - ctx.offsets[:-1]).max())
        smax = max(1, min(32, nmax // 64))
    else:
        smax = md.md_max_j_split(ctx.n)
        nmax = ctx.n
    splits = sorted({s for s in (1, 2, 4, 8, 16, 32, 64) if s <= smax and (s == 1 or s <= max(1, nmax // 64))})
    out = []
    for ipl, waves, s in itertools.product((1, 2, 4), (1, 2, 4), splits):
        out.append((ipl, waves, s, 128))
    return out


def time_step(ctx: md.Context, q: torch.Tensor, reps: int = 3) -> float:
    """Mean time in ms of one md_step with dt = 0 on the context's current tiles
    (on copies: q is not modified)."""
    qs = q.clone()
    p = torch.zeros_like(q)
    f = torch.empty_like(q)
    md.md_force(ctx, qs, f)
    md.md_step(ctx, qs, p, f, 0.0, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        md.md_step(ctx, qs, p, f, 0.0, 1)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_force(ctx: md.Context, q: torch.Tensor, reps: int = 3) -> float:
    """Mean md_force time in ms on the context's current tiles."""
    f = torch.empty_like(q)
    md.md_force(ctx, q, f)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        md.md_force(ctx, q, f)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(ctx: md.Context, q: torch.Tensor, configs: Optional[Iterable] = None, reps: int = 3,
         cache: Optional[str] = DEFAULT_CACHE, measure: str = "step") -> tuple:
    """Time every configuration (one md_step, or md_force with measure="force"),
    leave the fastest applied to ctx, record it in the cache (if given); returns
    (best_tiles, [(tiles, ms), ...] sorted by time).  A context in the symmetric
    launch form has no tile choice: it is timed once as it stands (set the staged
    form with md_set_launch first to tune that form's tiles)."""
    timer = time_step if measure == "step" else time_force
    if md.md_get_launch(ctx) == md.LAUNCH_SYMMETRIC:
        tiles = md.md_get_tiles(ctx)
        return tiles, [(tiles, timer(ctx, q, reps))]
    table = []
    for t in (configs if configs is not None else candidates(ctx)):
        try:
            md.md_set_tiles(ctx, *t)
        except md.MDError:
            continue
        table.append((md.md_get_tiles(ctx), timer(ctx, q, reps)))
    table.sort(key=lambda r: r[1])
    best = table[0][0]
    md.md_set_tiles(ctx, *best)
    if cache:
        data = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                data = json.load(fh)
        data[shape_key(ctx)] = {"tiles": list(best), "ms": table[0][1]}
        tmp = cache + ".tmp"
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best, table


def apply_cached(ctx: md.Context, cache: str = DEFAULT_CACHE) -> Optional[tuple]:
    """Apply the cached choice for this context, if any; returns it (or None)."""
    if not os.path.exists(cache):
        return None
    with open(cache) as fh:
        data = json.load(fh)
    rec = data.get(shape_key(ctx))
    if rec is None:
        return None
    md.md_set_tiles(ctx, *rec["tiles"])
    return tuple(rec["tiles"])
