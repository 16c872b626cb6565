"""Parity tolerances of the GPU tests, each about ten times the largest error
measured on MI355X for its kind of comparison, in a form that follows the
arithmetic (errors are max-norms of the difference relative to the largest
oracle value).

Forces
  * FP64 forms: 5e-14 * max(1, sqrt(n / 4096)).  Every FP64 pair term is formed
    to a few ulp (the FP64 reciprocal and reciprocal square root are refined to
    full precision; the Ring operands come from an FP64 sincos), so the GPU and
    the oracle differ by the rounding of two summation orders of n terms, which
    grows like u sqrt(n) times the cancellation of the sum.  Measured: 0.3e-15 to
    7.8e-15 for n <= 10,000, 3.2e-14 at n = 262,144.
  * FP32 forms (MD_MIXED, MD_MIXED_KAHAN, MD_MIXED_PAIRF64), 2D: 2e-6.  The
    positions are rounded to FP32 (relative 2^-24), which moves each pair term by
    its gradient times that shift; the FP32 terms are added in runs of `run`
    terms (the j-tile, 128 by default) before the FP64 fold, an error growing like
    2^-24 sqrt(run).  Measured on uniform-disk states: 2e-8 to 2.4e-7.  The factor
    sqrt(run / 128) covers longer FP32 runs (tiles of up to 4096 j).
  * FP32 forms, Ring: 5e-6.  The half-angle operands give 1 - cos(ti - tj) with an
    error proportional to the pair's own separation; it enters as the -3/2 power.
    Measured: 4e-8 to 5.4e-7.
  * eps below the workloads' (1e-3 for 2D, 1e-2 for Ring): the closest pairs'
    terms grow (the Ring term as u^{-3/2} with u >= eps), and with them the
    cancellation of the sum: the Ring FP64 tolerance scales as (eps_ref/eps)^1.5
    (measured 9.2e-14 at eps = 1e-3 against 6e-15 at 1e-2), every other one as
    (eps_ref/eps)^0.5 (measured 9.9e-7, Ring FP32 at eps = 1e-3; 4.6e-7, 2D FP32 at
    eps = 1e-4).
  * Clustered 2D states (two tight Gaussian clusters, the closest pairs near
    sqrt(eps)): 1e-5.  The FP32 rounding of the positions is relative to |r| ~ 0.5
    while the pair separations are ~0.02, so each term is 25 times less accurate;
    measured 1.06e-6.

Hessian-vector products (md_hvp)
  * FP64: 1e-13; measured up to 8.2e-15.
  * FP32 forms: 2e-5 (2D), 1e-5 (Ring).  The 1/s^2 term of the 2D Hessian doubles
    the sensitivity to the FP32 positions, and w is rounded to FP32 too; measured
    up to 2.3e-6 (2D) and 1.3e-6 (Ring).
"""
from __future__ import annotations

import math

from paper_1212_0262_amd import md

RING, GRAV2D = md.RING, md.GRAV2D


EPS_REF = {GRAV2D: 1e-3, RING: 1e-2}


def force_tol(model: int, prec: int, n: int, run: int = 128, clustered: bool = False, eps: float = None) -> float:
    """Tolerance of a force comparison at n particles (run: the FP32 j-tile; eps:
    the softening, where it is below the workloads')."""
    small = max(1.0, EPS_REF[model] / eps) if eps else 1.0
    if prec == md.FP64:
        return 5e-14 * max(1.0, math.sqrt(n / 4096)) * small ** (1.5 if model == RING else 0.5)
    if clustered:
        return 1e-5
    base = 2e-6 if model == GRAV2D else 5e-6
    return base * max(1.0, math.sqrt(run / 128)) * small ** 0.5


def hvp_tol(model: int, prec: int) -> float:
    if prec == md.FP64:
        return 1e-13
    return 2e-5 if model == GRAV2D else 1e-5


def check(label: str, err: float, tol: float) -> None:
    """Prints the measured error beside its tolerance, then asserts it."""
    print(f"{label}: err={err:.3e} tol={tol:.1e} ({tol / err if err > 0 else float('inf'):.0f}x)", flush=True)
    assert err < tol, (label, err, tol)
