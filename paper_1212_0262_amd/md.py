"""Thin Python binding of libmd (include/md.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libmd.so``; this module checks
tensor shapes, dtypes and devices, passes raw device pointers and the current
HIP stream across the C ABI, and turns status codes into exceptions.  PyTorch
provides device memory and streams, nothing else.

The function names mirror the C entry points.  Arrays are FP64 CUDA(HIP)
tensors of shape ``[d, n]`` (``d = 2`` for 2D gravity, else 1), contiguous.

torch is imported before the library is loaded, so that libmd binds to the
HIP runtime torch already holds (both carry the SONAME ``libamdhip64.so.7``)
and the process has one runtime.  There is no fallback: if ``libmd.so`` has
not been built, :func:`load` raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch  # noqa: F401  (must precede loading libmd: shared HIP runtime)

HMF, RING, GRAV2D = 0, 1, 2
FP64, MIXED, MIXED_KAHAN, MIXED_PAIRF64, MIXED_F32STATE = 0, 1, 2, 3, 4
OK, EINVAL, EDEVICE, ENOMEM, ESTATE, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
LAUNCH_AUTO, LAUNCH_STAGED, LAUNCH_FUSED, LAUNCH_SYMMETRIC = 0, 1, 2, 3
SYMMETRIC_AUTO_N = 13312  # MD_SYMMETRIC_AUTO_N: LAUNCH_AUTO takes the symmetric 2D form from this n (MIXED, FP64)
SYMMETRIC_AUTO_N_COMP = 15360    # MD_SYMMETRIC_AUTO_N_COMP: the same for 2D with the compensated forms
SYMMETRIC_AUTO_N_RING = 13312    # MD_SYMMETRIC_AUTO_N_RING: the same for the Ring with the FP32 forms
SYMMETRIC_AUTO_N_RING64 = 10240  # MD_SYMMETRIC_AUTO_N_RING64: the same for the Ring with FP64
# MD_EPS_*: the softening each pair model and precision accepts (md_init)
EPS_MIN_2D_FP64, EPS_MAX_2D_FP64 = 1e-75, 1e75
EPS_MIN_2D_FP32 = 1e-30
EPS_MIN_RING_FP64 = 1e-12
EPS_MIN_RING_FP32 = 1e-25
EPS_MAX_FP32 = 1e30

MODEL_NAMES = {HMF: "hmf", RING: "ring", GRAV2D: "grav2d"}
PREC_NAMES = {FP64: "fp64", MIXED: "mixed", MIXED_KAHAN: "mixed_kahan",
              MIXED_PAIRF64: "mixed_pairf64", MIXED_F32STATE: "mixed_f32state"}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmd.so")

# name -> (restype, argtypes); every symbol declared in include/md.h
_V, _I, _I64, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "md_workspace_bytes": (_SZ, [_I, _I, _I64]),
    "md_init": (_I, [ctypes.POINTER(_V), _I, _I, _I64, _D, _V, _V, _SZ]),
    "md_batch_workspace_bytes": (_SZ, [_I, _I, _I, _V, _V]),
    "md_batch_init": (_I, [ctypes.POINTER(_V), _I, _I, _I, _V, _V, _V, _V, _SZ]),
    "md_batch_size": (_I, [_V]),
    "md_set_stream": (_I, [_V, _V]),
    "md_set_tiles": (_I, [_V, _I, _I, _I, _I]),
    "md_get_tiles": (_I, [_V, ctypes.POINTER(_I)]),
    "md_set_launch": (_I, [_V, _I]),
    "md_get_launch": (_I, [_V]),
    "md_get_sym_tile": (_I, [_V]),
    "md_max_j_split": (_I, [_I64]),
    "md_force": (_I, [_V, _V, _V]),
    "md_force_noalloc": (_I, [_I, _I, _I64, _D, _V, _V, _V]),
    "md_step": (_I, [_V, _V, _V, _V, _D, _I64]),
    "md_energy": (_I, [_V, _V, _V, _V]),
    "md_magnetization": (_I, [_V, _V, _V]),
    "md_check": (_I, [_V]),
    "md_hvp": (_I, [_V, _V, _V, _V]),
    "md_vjp_stage_bytes": (_SZ, [_V, _I64]),
    "md_step_vjp": (_I, [_V, _V, _V, _D, _I64, _V, _V, _V, _SZ]),
    "md_record_stage_bytes": (_SZ, [_V, _I64]),
    "md_step_record": (_I, [_V, _V, _V, _V, _D, _I64, _V, _SZ]),
    "md_step_vjp_recorded": (_I, [_V, _V, _D, _I64, _V, _V, _V, _SZ]),
    "md_timing_begin": (_I, [_V, _I]),
    "md_timing_end": (_I, [_V, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.c_char_p, _SZ]),
    "md_destroy": (_I, [_V]),
    "md_strerror": (ctypes.c_char_p, [_I]),
    "md_last_error": (ctypes.c_char_p, [_V]),
    "md_version": (ctypes.c_char_p, []),
}

_lib: Optional[ctypes.CDLL] = None


class MDError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {strerror(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


def load() -> ctypes.CDLL:
    """The loaded libmd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1212_0262_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(status: int) -> str:
    return load().md_strerror(int(status)).decode()


def md_version() -> str:
    return load().md_version().decode()


def dims(model: int) -> int:
    return 2 if model == GRAV2D else 1


def md_workspace_bytes(model: int, prec: int, n: int) -> int:
    return int(load().md_workspace_bytes(int(model), int(prec), int(n)))


def md_max_j_split(n: int) -> int:
    return int(load().md_max_j_split(int(n)))


def _stream_handle(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """A libmd context plus the workspace tensor it lives in."""

    def __init__(self, handle: int, model: int, prec: int, n: int, eps: float, workspace: torch.Tensor):
        self.handle = handle
        self.model, self.prec, self.n, self.eps = model, prec, n, eps
        self.d = dims(model)
        self.workspace = workspace

    def _check(self, status: int, where: str) -> None:
        if status != OK:
            detail = load().md_last_error(self.handle).decode() if self.handle else ""
            raise MDError(status, where, detail)

    def _arr(self, t: torch.Tensor, name: str) -> int:
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name}: expected a device tensor")
        if t.dtype != torch.float64:
            raise TypeError(f"{name}: expected float64, got {t.dtype}")
        if tuple(t.shape) != (self.d, self.n) or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous [{self.d}, {self.n}] tensor, got {tuple(t.shape)}")
        return t.data_ptr()

    def close(self) -> None:
        if self.handle:
            load().md_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def md_init(model: int, prec: int, n: int, eps: float = 0.0, stream=None,
            workspace: Optional[torch.Tensor] = None) -> Context:
    """Create a context on the current device; allocates the workspace with torch if not given."""
    need = md_workspace_bytes(model, prec, n)
    if workspace is None:
        if need == 0:
            raise MDError(EINVAL, "md_init", f"invalid model/prec/n ({model}, {prec}, {n})")
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = load().md_init(ctypes.byref(h), int(model), int(prec), int(n), float(eps), _stream_handle(stream),
                        workspace.data_ptr(), workspace.numel() * workspace.element_size())
    if st != OK:
        raise MDError(st, "md_init")
    return Context(h.value, int(model), int(prec), int(n), float(eps), workspace)


def _batch_arrays(offsets, eps):
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nb = off.size - 1
    e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (max(nb, 0),)))
    return off, e, nb


def md_batch_workspace_bytes(model: int, prec: int, offsets, eps) -> int:
    off, e, nb = _batch_arrays(offsets, eps)
    return int(load().md_batch_workspace_bytes(int(model), int(prec), nb, off.ctypes.data, e.ctypes.data))


def md_batch_init(model: int, prec: int, offsets, eps, stream=None,
                  workspace: Optional[torch.Tensor] = None) -> Context:
    """Context for an ensemble of realizations: offsets[nb + 1] (CSR, host), eps per
    realization (scalar or [nb]).  Arrays are the realizations concatenated."""
    off, e, nb = _batch_arrays(offsets, eps)
    need = md_batch_workspace_bytes(model, prec, off, e)
    if workspace is None:
        if need == 0:
            raise MDError(EINVAL, "md_batch_init", "invalid model/prec/offsets/eps")
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = load().md_batch_init(ctypes.byref(h), int(model), int(prec), nb, off.ctypes.data, e.ctypes.data,
                              _stream_handle(stream), workspace.data_ptr(),
                              workspace.numel() * workspace.element_size())
    if st != OK:
        raise MDError(st, "md_batch_init")
    ctx = Context(h.value, int(model), int(prec), int(off[-1]), float(e[0]), workspace)
    ctx.nb = nb
    ctx.offsets = off.copy()
    return ctx


def md_batch_size(ctx: Context) -> int:
    return int(load().md_batch_size(ctx.handle))


def md_set_stream(ctx: Context, stream=None) -> None:
    ctx._check(load().md_set_stream(ctx.handle, _stream_handle(stream)), "md_set_stream")


def md_set_tiles(ctx: Context, i_per_lane: int = 0, waves: int = 0, j_split: int = 0, j_tile: int = 0) -> None:
    ctx._check(load().md_set_tiles(ctx.handle, int(i_per_lane), int(waves), int(j_split), int(j_tile)),
               "md_set_tiles")


def md_get_tiles(ctx: Context) -> tuple:
    out = (ctypes.c_int * 4)()
    ctx._check(load().md_get_tiles(ctx.handle, out), "md_get_tiles")
    return tuple(int(v) for v in out)


def md_set_launch(ctx: Context, mode: int) -> None:
    """LAUNCH_AUTO, LAUNCH_STAGED, LAUNCH_FUSED or LAUNCH_SYMMETRIC (md_step's launch form)."""
    ctx._check(load().md_set_launch(ctx.handle, int(mode)), "md_set_launch")


def md_get_launch(ctx: Context) -> int:
    """The form md_step takes: LAUNCH_STAGED, LAUNCH_FUSED or LAUNCH_SYMMETRIC."""
    r = int(load().md_get_launch(ctx.handle))
    ctx._check(min(r, 0), "md_get_launch")
    return r


def md_get_sym_tile(ctx: Context) -> int:
    """Particles per tile of the symmetric form (1024 or 512) if md_step takes it, else 0."""
    r = int(load().md_get_sym_tile(ctx.handle))
    ctx._check(min(r, 0), "md_get_sym_tile")
    return r


def md_force(ctx: Context, q: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
    ctx._check(load().md_force(ctx.handle, ctx._arr(q, "q"), ctx._arr(f, "f")), "md_force")
    return f


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024  # MD_NOALLOC_SCRATCH_BYTES


def md_force_noalloc(model: int, prec: int, q: torch.Tensor, eps: float, f: torch.Tensor, stream=None) -> None:
    """f = force(q) with the library's static workspace: no context, and nothing
    allocated, here or in the library (f is the caller's).  Staged form, built-in
    tiles (j split halved until its partials fit the static array)."""
    d, n = dims(model), q.shape[-1]
    for name, t in (("q", q), ("f", f)):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
            raise TypeError(f"{name}: expected a device float64 tensor")
        if tuple(t.shape) != (d, n) or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous [{d}, {n}] tensor, got {tuple(t.shape)}")
    st = load().md_force_noalloc(int(model), int(prec), int(n), float(eps), _stream_handle(stream), q.data_ptr(),
                                 f.data_ptr())
    if st == ENOMEM:
        raise MDError(st, "md_force_noalloc",
                      f"n = {n} needs more than the {NOALLOC_SCRATCH_BYTES >> 20} MiB static workspace")
    if st != OK:
        raise MDError(st, "md_force_noalloc")


def md_step(ctx: Context, q: torch.Tensor, p: torch.Tensor, f: torch.Tensor, dt: float, nsteps: int) -> None:
    ctx._check(load().md_step(ctx.handle, ctx._arr(q, "q"), ctx._arr(p, "p"), ctx._arr(f, "f"),
                              float(dt), int(nsteps)), "md_step")


def md_check(ctx: Context) -> None:
    """Waits for the context's stream; raises MDError(ENONFINITE) if the energies or
    magnetization last written were not finite."""
    ctx._check(load().md_check(ctx.handle), "md_check")


def md_energy(ctx: Context, q: torch.Tensor, p: torch.Tensor, out: Optional[torch.Tensor] = None,
              check: bool = True) -> torch.Tensor:
    """{K, V, E} as a device float64 tensor of 3 ([nb, 3] for a batch context).
    With check (the default) it waits for the stream and raises MDError(ENONFINITE)
    if a value is not finite (md_check); pass check=False under graph capture."""
    nb = getattr(ctx, "nb", 1)
    if out is None:
        out = torch.empty((nb, 3) if nb > 1 or hasattr(ctx, "nb") else 3, dtype=torch.float64, device=q.device)
    if out.dtype != torch.float64 or out.numel() < 3 * nb or out.device.type != "cuda" or not out.is_contiguous():
        raise ValueError(f"out: expected a contiguous device float64 tensor of at least {3 * nb} elements")
    ctx._check(load().md_energy(ctx.handle, ctx._arr(q, "q"), ctx._arr(p, "p"), out.data_ptr()), "md_energy")
    if check:
        md_check(ctx)
    return out


def md_magnetization(ctx: Context, q: torch.Tensor, out: Optional[torch.Tensor] = None,
                     check: bool = True) -> torch.Tensor:
    """(Mx, My) as a device float64 tensor of 2; check as md_energy."""
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=q.device)
    ctx._check(load().md_magnetization(ctx.handle, ctx._arr(q, "q"), out.data_ptr()), "md_magnetization")
    if check:
        md_check(ctx)
    return out


def md_hvp(ctx: Context, q: torch.Tensor, w: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out = H(q) w, H the Hessian of the potential."""
    if out is None:
        out = torch.empty_like(q)
    ctx._check(load().md_hvp(ctx.handle, ctx._arr(q, "q"), ctx._arr(w, "w"), ctx._arr(out, "out")), "md_hvp")
    return out


def md_vjp_stage_bytes(ctx: Context, nsteps: int) -> int:
    return int(load().md_vjp_stage_bytes(ctx.handle, int(nsteps)))


def md_step_vjp(ctx: Context, q0: torch.Tensor, p0: torch.Tensor, dt: float, nsteps: int, lam_q: torch.Tensor,
                lam_p: torch.Tensor, stage: Optional[torch.Tensor] = None) -> None:
    """In place: (lam_q, lam_p) at the end of nsteps steps from (q0, p0) become the
    adjoints at (q0, p0).  stage: device scratch (allocated here if None)."""
    need = md_vjp_stage_bytes(ctx, nsteps)
    if stage is None:
        stage = torch.empty(max(need, 8), dtype=torch.uint8, device=q0.device)
    ctx._check(load().md_step_vjp(ctx.handle, ctx._arr(q0, "q0"), ctx._arr(p0, "p0"), float(dt), int(nsteps),
                                  ctx._arr(lam_q, "lam_q"), ctx._arr(lam_p, "lam_p"), stage.data_ptr(),
                                  stage.numel() * stage.element_size()), "md_step_vjp")


def md_record_stage_bytes(ctx: Context, nsteps: int) -> int:
    return int(load().md_record_stage_bytes(ctx.handle, int(nsteps)))


def md_step_record(ctx: Context, q: torch.Tensor, p: torch.Tensor, f: torch.Tensor, dt: float, nsteps: int,
                   stage: Optional[torch.Tensor] = None) -> torch.Tensor:
    """md_step that also records every kick position into stage (allocated here
    if None); returns stage for md_step_vjp_recorded."""
    need = md_record_stage_bytes(ctx, nsteps)
    if stage is None:
        stage = torch.empty(max(need, 8), dtype=torch.uint8, device=q.device)
    ctx._check(load().md_step_record(ctx.handle, ctx._arr(q, "q"), ctx._arr(p, "p"), ctx._arr(f, "f"), float(dt),
                                     int(nsteps), stage.data_ptr(), stage.numel() * stage.element_size()),
               "md_step_record")
    return stage


def md_step_vjp_recorded(ctx: Context, q0: torch.Tensor, dt: float, nsteps: int, lam_q: torch.Tensor,
                         lam_p: torch.Tensor, stage: torch.Tensor) -> None:
    """In place: the reverse sweep over a run recorded by md_step_record from q0."""
    ctx._check(load().md_step_vjp_recorded(ctx.handle, ctx._arr(q0, "q0"), float(dt), int(nsteps),
                                           ctx._arr(lam_q, "lam_q"), ctx._arr(lam_p, "lam_p"), stage.data_ptr(),
                                           stage.numel() * stage.element_size()), "md_step_vjp_recorded")


def md_timing_begin(ctx: Context, max_launches: int) -> None:
    """Time the first max_launches launches of the context's dominant kernel (HIP
    events on its stream); read the result with md_timing_end."""
    ctx._check(load().md_timing_begin(ctx.handle, int(max_launches)), "md_timing_begin")


def md_timing_end(ctx: Context) -> tuple:
    """(summed ms, launches timed, kernel name) since md_timing_begin; waits for the
    last timed launch and turns timing off."""
    ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
    name = ctypes.create_string_buffer(64)
    ctx._check(load().md_timing_end(ctx.handle, ctypes.byref(ms), ctypes.byref(n), name, 64), "md_timing_end")
    return ms.value, n.value, name.value.decode()


def md_destroy(ctx: Context) -> None:
    ctx.close()
