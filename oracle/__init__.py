"""FP64 CPU oracle for the long-range MD hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never does, and this package imports
nothing from it: the two share no code.  See ``oracle.c`` for what is computed,
the passages of the paper each function follows, and the readings taken where
the paper is silent or garbled.

All arrays are host numpy FP64, structure-of-arrays ``[d, n]`` (``d = 2`` for
2D gravity, else 1).  Model ids: HMF = 0, RING = 1, GRAV2D = 2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HMF, RING, GRAV2D = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.c_double
_L = ctypes.c_long
_I = ctypes.c_int
_P = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        sig = {
            "or_set_threads": (None, [_I]),
            "or_get_threads": (_I, []),
            "or_yoshida": (None, [_P]),
            "or_magnetization": (None, [_L, _P, _P]),
            "or_force": (_I, [_I, _L, _D, _P, _P]),
            "or_force_rows": (_I, [_I, _L, _D, _P, _P, _L, _P]),
            "or_hmf_force_pairs": (_I, [_L, _P, _P]),
            "or_step": (_I, [_I, _L, _D, _P, _P, _P, _D, _L]),
            "or_kinetic": (_D, [_I, _L, _P]),
            "or_potential": (_D, [_I, _L, _D, _P]),
            "or_hmf_potential_pairs": (_D, [_L, _P]),
            "or_energy": (_I, [_I, _L, _D, _P, _P, _P]),
            "or_hvp": (_I, [_I, _L, _D, _P, _P, _P]),
            "or_step_vjp": (_I, [_I, _L, _D, _P, _P, _D, _L, _P, _P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def dims(model: int) -> int:
    return 2 if model == GRAV2D else 1


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


def yoshida() -> tuple:
    """(B0, B1, D0, D1) of eq. 4."""
    c = np.zeros(4)
    _load().or_yoshida(_ptr(c))
    return tuple(float(x) for x in c)


def magnetization(q) -> tuple:
    """(Mx, My) of eq. 7."""
    q = _f64(q).reshape(-1)
    m = np.zeros(2)
    _load().or_magnetization(q.size, _ptr(q), _ptr(m))
    return float(m[0]), float(m[1])


def force(model: int, q, eps: float = 0.0) -> np.ndarray:
    """f = -dV/dq at q, shape [d, n]."""
    q = _f64(q)
    n = q.shape[-1]
    f = np.zeros((dims(model), n))
    rc = _load().or_force(model, n, float(eps), _ptr(q), _ptr(f))
    if rc != 0:
        raise ValueError("oracle force: bad arguments")
    return f


def force_rows(model: int, q, rows, eps: float = 0.0) -> np.ndarray:
    """Force on particles `rows` only, shape [d, len(rows)]."""
    q = _f64(q)
    n = q.shape[-1]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    f = np.zeros((dims(model), rows.size))
    rc = _load().or_force_rows(model, n, float(eps), _ptr(q), _ptr(rows), rows.size, _ptr(f))
    if rc != 0:
        raise ValueError("oracle force_rows: bad arguments")
    return f


def hmf_force_pairs(q) -> np.ndarray:
    """HMF force as the O(N^2) pair sum of eq. 2's gradient, shape [1, n]."""
    q = _f64(q)
    n = q.shape[-1]
    f = np.zeros((1, n))
    _load().or_hmf_force_pairs(n, _ptr(q), _ptr(f))
    return f


def step(model: int, q, p, f, dt: float, nsteps: int, eps: float = 0.0):
    """nsteps Yoshida steps; returns new (q, p, f).  f must equal force(q) on entry."""
    q, p, f = _f64(q).copy(), _f64(p).copy(), _f64(f).copy()
    n = q.shape[-1]
    rc = _load().or_step(model, n, float(eps), _ptr(q), _ptr(p), _ptr(f), float(dt), int(nsteps))
    if rc != 0:
        raise ValueError("oracle step: bad arguments")
    return q, p, f


def kinetic(model: int, p) -> float:
    p = _f64(p)
    return float(_load().or_kinetic(model, p.shape[-1], _ptr(p)))


def potential(model: int, q, eps: float = 0.0) -> float:
    q = _f64(q)
    return float(_load().or_potential(model, q.shape[-1], float(eps), _ptr(q)))


def hmf_potential_pairs(q) -> float:
    q = _f64(q)
    return float(_load().or_hmf_potential_pairs(q.shape[-1], _ptr(q)))


def energy(model: int, q, p, eps: float = 0.0) -> np.ndarray:
    """[K, V, E] in FP64."""
    q, p = _f64(q), _f64(p)
    out = np.zeros(3)
    rc = _load().or_energy(model, q.shape[-1], float(eps), _ptr(q), _ptr(p), _ptr(out))
    if rc != 0:
        raise ValueError("oracle energy: bad arguments")
    return out


def hvp(model: int, q, w, eps: float = 0.0) -> np.ndarray:
    """H(q) w, H the Hessian of the potential (eqs. 1-3); shape [d, n]."""
    q, w = _f64(q), _f64(w)
    out = np.zeros_like(q)
    rc = _load().or_hvp(model, q.shape[-1], float(eps), _ptr(q), _ptr(w), _ptr(out))
    if rc != 0:
        raise ValueError("oracle hvp: bad arguments")
    return out


def step_vjp(model: int, q0, p0, dt: float, nsteps: int, lam_q, lam_p, eps: float = 0.0):
    """Adjoints at the start of nsteps Yoshida steps from (q0, p0), given the
    adjoints (lam_q, lam_p) at their end; returns (dJ/dq0, dJ/dp0)."""
    q0, p0 = _f64(q0), _f64(p0)
    lq, lp = _f64(lam_q).copy(), _f64(lam_p).copy()
    rc = _load().or_step_vjp(model, q0.shape[-1], float(eps), _ptr(q0), _ptr(p0), float(dt), int(nsteps),
                             _ptr(lq), _ptr(lp))
    if rc != 0:
        raise ValueError("oracle step_vjp: bad arguments")
    return lq, lp
