"""Seeded synthetic initial conditions for the three long-range models.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no force, energy or integrator step), so both the GPU path
and the FP64 CPU oracle may take their inputs from it.

Layout of every state returned here: structure-of-arrays FP64, ``q`` and ``p``
of shape ``[d, n]`` (``d = 1`` for the angle models HMF and Ring, ``d = 2`` for
2D gravity with the x row first, then y), C-contiguous.

Generators (numpy PCG64 via ``default_rng``; draws happen in the order written):

* :func:`ring_waterbag` -- theta ~ U(-pi/2, pi/2), then p ~ U(-0.5, 0.5).
  The workload of the Ring timing and parity runs (N = 2048, eps = 0.01).
* :func:`hmf_waterbag` -- theta ~ U(-1, 1), then p ~ U(-1.2, 1.2).
  The waterbag state used for the HMF mean-field runs (N = 10^7).
* :func:`grav2d_disk` -- positions uniform in the unit disk (r = sqrt(U),
  phi = U(0, 2 pi)), then px, py ~ N(0, sigma) with their means subtracted so
  the total momentum is zero.  The 2D self-gravitating workload (N = 262,144).
* :func:`homogeneous_at_rest` and :func:`shell_at_rest` -- the states the paper
  uses for its energy-error runs (Section 4: HMF and Ring spatially homogeneous
  at rest; 2D gravity uniform on the shell 1.0 <= r <= 1.5 at rest).
* :func:`ensemble_sizes` -- realization sizes drawn log-uniform for batched
  ensembles of Ring systems.
"""
from __future__ import annotations

import numpy as np

HMF, RING, GRAV2D = 0, 1, 2


def dims(model: int) -> int:
    """Number of coordinate rows per particle: 2 for 2D gravity, else 1."""
    return 2 if model == GRAV2D else 1


def _state(q, p):
    return (np.ascontiguousarray(q, dtype=np.float64),
            np.ascontiguousarray(p, dtype=np.float64))


def ring_waterbag(n: int, seed: int = 1):
    """theta ~ U(-pi/2, pi/2), then p ~ U(-0.5, 0.5); shapes [1, n]."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi / 2, np.pi / 2, size=n)
    p = rng.uniform(-0.5, 0.5, size=n)
    return _state(th[None, :], p[None, :])


def hmf_waterbag(n: int, seed: int = 2, theta0: float = 1.0, p0: float = 1.2):
    """theta ~ U(-theta0, theta0), then p ~ U(-p0, p0); shapes [1, n]."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(-theta0, theta0, size=n)
    p = rng.uniform(-p0, p0, size=n)
    return _state(th[None, :], p[None, :])


def grav2d_disk(n: int, seed: int = 3, sigma: float = 0.5, radius: float = 1.0):
    """Uniform disk of the given radius, Gaussian momenta with zero mean; shapes [2, n]."""
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, size=n))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    q = np.stack([r * np.cos(phi), r * np.sin(phi)])
    p = rng.normal(0.0, sigma, size=(2, n))
    p -= p.mean(axis=1, keepdims=True)
    return _state(q, p)


def homogeneous_at_rest(n: int, seed: int = 0):
    """theta ~ U(-pi, pi), p = 0; shapes [1, n] (HMF / Ring energy-error runs)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi, np.pi, size=n)
    return _state(th[None, :], np.zeros((1, n)))


def shell_at_rest(n: int, seed: int = 0, r1: float = 1.0, r2: float = 1.5):
    """Uniform in the annulus r1 <= r <= r2, p = 0; shapes [2, n] (2D energy-error runs)."""
    rng = np.random.default_rng(seed)
    r = np.sqrt(rng.uniform(r1 * r1, r2 * r2, size=n))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    q = np.stack([r * np.cos(phi), r * np.sin(phi)])
    return _state(q, np.zeros((2, n)))


def uniform_state(model: int, n: int, seed: int, qscale: float = 1.0, pscale: float = 1.0):
    """Generic small random state for property and parity tests."""
    rng = np.random.default_rng(seed)
    d = dims(model)
    q = rng.uniform(-qscale, qscale, size=(d, n))
    p = rng.uniform(-pscale, pscale, size=(d, n))
    return _state(q, p)


def ensemble_sizes(nb: int = 256, seed: int = 4, nmin: int = 1000, nmax: int = 16384):
    """Realization sizes N_b = round(exp(U(ln nmin, ln nmax))), as int64."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=nb))).astype(np.int64)


def ensemble_member(b: int, n: int, seed: int = 4):
    """Waterbag Ring state of realization b (seeded by [seed, b]); shapes [1, n]."""
    rng = np.random.default_rng([seed, b])
    th = rng.uniform(-np.pi / 2, np.pi / 2, size=n)
    p = rng.uniform(-0.5, 0.5, size=n)
    return _state(th[None, :], p[None, :])
