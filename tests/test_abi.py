"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
entry point include/md.h declares, and rejects bad arguments before it touches a
device.  No compute call runs here."""
import ctypes
import os
import re

import pytest

md = pytest.importorskip("paper_1212_0262_amd.md")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        return md.load()
    except ImportError as e:
        pytest.skip(str(e))


def _declared():
    txt = open(os.path.join(ROOT, "include", "md.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = _lib()
    names = _declared()
    assert len(names) >= 10, names
    for name in names:
        assert hasattr(lib, name), name
        assert name in md.SIGNATURES, f"binding lacks {name}"
    assert set(md.SIGNATURES) == set(names)


def test_strerror_and_version():
    _lib()
    for code in (md.OK, md.EINVAL, md.EDEVICE, md.ENOMEM, md.ESTATE, md.ENONFINITE, md.EUNSUPPORTED):
        assert md.strerror(code) and md.strerror(code) != "unknown status"
    assert md.strerror(12345) == "unknown status"
    assert "gfx950" in md.md_version()


def test_workspace_bytes():
    _lib()
    for model in (md.RING, md.GRAV2D):
        for prec in (md.FP64, md.MIXED, md.MIXED_KAHAN, md.MIXED_PAIRF64):
            b = md.md_workspace_bytes(model, prec, 1000)
            assert b > 0 and b % 256 == 0
        assert md.md_workspace_bytes(model, md.MIXED_F32STATE, 1000) == 0
    assert md.md_workspace_bytes(md.HMF, md.FP64, 10) > 0
    assert md.md_workspace_bytes(md.HMF, md.MIXED_F32STATE, 10) > md.md_workspace_bytes(md.HMF, md.FP64, 10)
    assert md.md_workspace_bytes(md.HMF, md.MIXED, 10) == 0
    assert md.md_workspace_bytes(7, md.FP64, 10) == 0
    assert md.md_workspace_bytes(md.RING, md.FP64, 0) == 0
    assert md.md_workspace_bytes(md.GRAV2D, md.FP64, (1 << 23) + 1) == 0
    # the pair partials grow with the largest j split
    n = 262144
    s = md.md_max_j_split(n)
    assert md.md_workspace_bytes(md.GRAV2D, md.FP64, n) >= s * 2 * n * 8


def test_max_j_split():
    _lib()
    assert md.md_max_j_split(1) == 64
    assert md.md_max_j_split(2048) == 64
    assert md.md_max_j_split(262144) == 16
    assert md.md_max_j_split(1 << 23) == 1
    assert md.md_max_j_split(0) == 1


def _init(lib, model, prec, n, eps, ws=256, wsb=1 << 40):
    h = ctypes.c_void_p()
    st = lib.md_init(ctypes.byref(h), model, prec, n, eps, None, ws, wsb)
    return st, h.value


@pytest.mark.parametrize("args,expect", [
    ((md.GRAV2D, md.FP64, 100, 0.0), md.EINVAL),       # eps must be > 0 (eq. 3)
    ((md.RING, md.MIXED, 100, -1e-3), md.EINVAL),
    ((md.RING, md.FP64, 100, float("nan")), md.EINVAL),
    ((md.GRAV2D, md.FP64, 0, 1e-3), md.EINVAL),        # n >= 1
    ((md.GRAV2D, md.FP64, -5, 1e-3), md.EINVAL),
    ((9, md.FP64, 100, 1e-3), md.EINVAL),              # unknown model
    ((md.HMF, md.MIXED, 100, 0.0), md.EUNSUPPORTED),   # HMF: FP64 or FP32 state only
    ((md.GRAV2D, md.MIXED_F32STATE, 100, 1e-3), md.EUNSUPPORTED),
    ((md.GRAV2D, 17, 100, 1e-3), md.EUNSUPPORTED),
])
def test_init_rejects_bad_arguments(args, expect):
    lib = _lib()
    st, h = _init(lib, *args)
    assert st == expect and h is None


def test_eps_ranges_match_the_header():
    txt = open(os.path.join(ROOT, "include", "md.h")).read()
    macros = dict(re.findall(r"#define MD_(EPS_[A-Z0-9_]+)\s+(\S+)", txt))
    assert len(macros) == 6, macros
    for name, value in macros.items():
        assert getattr(md, name) == float(value), name


# (model, prec, eps): each side of every bound of the accepted softening
EPS_CASES = [
    (md.GRAV2D, md.FP64, md.EPS_MIN_2D_FP64, md.EPS_MAX_2D_FP64),
    (md.GRAV2D, md.MIXED, md.EPS_MIN_2D_FP32, md.EPS_MAX_FP32),
    (md.GRAV2D, md.MIXED_KAHAN, md.EPS_MIN_2D_FP32, md.EPS_MAX_FP32),
    (md.GRAV2D, md.MIXED_PAIRF64, md.EPS_MIN_2D_FP32, md.EPS_MAX_FP32),
    (md.RING, md.FP64, md.EPS_MIN_RING_FP64, None),
    (md.RING, md.MIXED, md.EPS_MIN_RING_FP32, md.EPS_MAX_FP32),
    (md.RING, md.MIXED_KAHAN, md.EPS_MIN_RING_FP32, md.EPS_MAX_FP32),
]


@pytest.mark.parametrize("model,prec,lo,hi", EPS_CASES)
def test_eps_range_is_enforced(model, prec, lo, hi):
    """Softening below (or above) the range of a pair form is MD_EINVAL from md_init,
    md_batch_init and md_force_noalloc, before any device work; the bounds
    themselves pass validation (on a machine without a GPU the call then stops at
    the device, not at the argument)."""
    import numpy as np
    lib = _lib()
    bad = [lo * 0.5] + ([hi * 2.0] if hi else [])
    good = [lo] + ([hi] if hi else [1e200])
    off = np.array([0, 10, 20], dtype=np.int64)
    h = ctypes.c_void_p()
    for eps in bad:
        assert _init(lib, model, prec, 100, eps)[0] == md.EINVAL, eps
        e2 = np.array([0.01 if model == md.RING else 1e-3, eps])
        assert lib.md_batch_init(ctypes.byref(h), model, prec, 2, off.ctypes.data, e2.ctypes.data, None, 256,
                                 1 << 40) == md.EINVAL, eps
        assert lib.md_force_noalloc(model, prec, 100, eps, None, 256, 256) == md.EINVAL, eps
    for eps in good:
        st, hh = _init(lib, model, prec, 100, eps)
        assert st != md.EINVAL, eps
        if st == md.OK:
            lib.md_destroy(hh)


def test_init_rejects_bad_workspace():
    lib = _lib()
    need = md.md_workspace_bytes(md.GRAV2D, md.MIXED, 1000)
    assert _init(lib, md.GRAV2D, md.MIXED, 1000, 1e-3, ws=None)[0] == md.EINVAL
    assert _init(lib, md.GRAV2D, md.MIXED, 1000, 1e-3, ws=256 + 8)[0] == md.EINVAL   # not 256-aligned
    assert _init(lib, md.GRAV2D, md.MIXED, 1000, 1e-3, wsb=need - 1)[0] == md.ENOMEM
    assert lib.md_init(None, md.GRAV2D, md.MIXED, 1000, 1e-3, None, 256, need) == md.EINVAL


def test_null_context_calls():
    lib = _lib()
    assert lib.md_force(None, 256, 256) == md.EINVAL
    assert lib.md_step(None, 256, 256, 256, 0.1, 1) == md.EINVAL
    assert lib.md_energy(None, 256, 256, 256) == md.EINVAL
    assert lib.md_magnetization(None, 256, 256) == md.EINVAL
    assert lib.md_set_tiles(None, 1, 1, 1, 16) == md.EINVAL
    assert lib.md_get_tiles(None, None) == md.EINVAL
    assert lib.md_set_launch(None, md.LAUNCH_FUSED) == md.EINVAL
    assert lib.md_get_launch(None) == md.EINVAL
    assert lib.md_get_sym_tile(None) == md.EINVAL
    assert lib.md_set_stream(None, None) == md.EINVAL
    assert lib.md_destroy(None) == md.OK
    assert lib.md_last_error(None) == b""


def test_product_path_has_no_oracle_dependency():
    """The library and its binding never reach the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1212_0262_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), fn
                assert "liboracle" not in txt and "oracle.c" not in txt, fn
    so = md.LIB_PATH
    if os.path.exists(so):
        assert b"or_force" not in open(so, "rb").read()


def test_batch_validation_on_host():
    """Batched ensembles: bad CSR offsets or eps are rejected before any device work."""
    import numpy as np
    lib = _lib()
    h = ctypes.c_void_p()
    e2 = np.array([0.01, 0.01])

    def init(model, prec, off, eps, nb=None):
        off = np.ascontiguousarray(off, dtype=np.int64)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        nb = off.size - 1 if nb is None else nb
        return lib.md_batch_init(ctypes.byref(h), model, prec, nb, off.ctypes.data, eps.ctypes.data, None, 256,
                                 1 << 40)
    assert init(md.RING, md.FP64, [0, 10, 5], e2) == md.EINVAL        # decreasing offsets
    assert init(md.RING, md.FP64, [0, 10, 10], e2) == md.EINVAL       # empty realization
    assert init(md.RING, md.FP64, [3, 10, 20], e2) == md.EINVAL       # offsets[0] != 0
    assert init(md.RING, md.FP64, [0, 10, 20], [0.01, 0.0]) == md.EINVAL
    assert init(md.GRAV2D, md.MIXED, [0, 10, 20], [0.01, float("inf")]) == md.EINVAL
    assert init(md.RING, md.FP64, [0, 10], [0.01], nb=0) == md.EINVAL
    assert init(md.HMF, md.FP64, [0, 10, 20], e2) == md.EUNSUPPORTED
    assert init(md.RING, md.MIXED_F32STATE, [0, 10, 20], e2) == md.EUNSUPPORTED
    assert init(md.RING, md.FP64, [0, 1 << 23, (1 << 24) + 1], e2) == md.EINVAL  # too many particles in total
    assert md.md_batch_workspace_bytes(md.RING, md.FP64, [0, 10, 20], 0.01) > 0
    assert md.md_batch_workspace_bytes(md.RING, md.FP64, [0, 10, 5], 0.01) == 0
    assert lib.md_batch_size(None) == 0


def test_no_kernel_has_a_private_segment():
    """Every kernel of the built library runs from registers and LDS alone: the
    build records the compiler's resource-usage figures and refuses scratch.
    A private segment costs time on every dispatch (about 1.2 us measured on a
    one-block HMF reduction kernel, 10% of the HMF step at N = 1e5)."""
    import json
    from paper_1212_0262_amd import build
    if not os.path.exists(build.RESOURCES):
        pytest.skip("library not built")
    kernels = json.load(open(build.RESOURCES))
    assert len(kernels) >= 100
    srcs = {k["source"] for k in kernels}
    assert srcs == set(build.SOURCES) - {"api.hip"}, srcs
    for k in kernels:
        assert k["scratch"] == 0 and not k["dynamic_stack"], k
        assert k["vgpr_spill"] == 0, k  # (SGPR spills go to VGPR lanes, not memory)
        assert k["vgprs"] + k["agprs"] <= 512, k
    names = " ".join(k["kernel"] for k in kernels)
    for kern in ("k_hmf_pass", "k_hmf_limbs_to_m", "k_update", "k_sym", "k_fused", "k_batch_sym"):
        assert kern in names, kern


def test_timing_entry_points_reject_null_context():
    lib = _lib()
    ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
    assert lib.md_timing_begin(None, 4) == md.EINVAL
    assert lib.md_timing_end(None, ctypes.byref(ms), ctypes.byref(n), None, 0) == md.EINVAL
