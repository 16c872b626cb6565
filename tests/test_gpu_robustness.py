"""GPU robustness: code paths the workload tests do not reach -- HMF with
unaligned arrays (scalar accesses) and ragged N (vector tails), the tile
autotuner, and randomized small systems over every model, precision and tile
configuration (hypothesis), each against the FP64 oracle with the tolerances of
test_gpu_parity.py."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1212_0262_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
md = pytest.importorskip("paper_1212_0262_amd.md")
hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

from gpu_helpers import dev, host, rel_inf  # noqa: E402
from tolerances import check, force_tol  # noqa: E402

HMF, RING, GRAV2D = md.HMF, md.RING, md.GRAV2D


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield


def _offset_view(a: np.ndarray) -> torch.Tensor:
    """A contiguous device view of `a` whose data pointer is 8-byte but not
    16-byte aligned."""
    d, n = a.shape
    big = torch.zeros((d, n + 1), dtype=torch.float64, device="cuda")
    flat = big.reshape(-1)[1:1 + d * n].view(d, n)
    flat.copy_(torch.from_numpy(a))
    assert flat.data_ptr() % 16 == 8 and flat.is_contiguous()
    return flat


@pytest.mark.parametrize("n", [1, 3, 1001, 20_003])
def test_hmf_unaligned_arrays_take_the_scalar_path(n):
    q, p = inputs.hmf_waterbag(n, seed=90)
    f0 = oracle.force(HMF, q)
    qo, po, fo = oracle.step(HMF, q, p, f0, 0.1, 5, 0.0)
    ctx = md.md_init(HMF, md.FP64, n, 0.0)
    qd, pd = _offset_view(q), _offset_view(p)
    f = _offset_view(np.zeros_like(q))
    md.md_force(ctx, qd, f)
    assert np.abs(host(f) - f0).max() < 1e-13
    md.md_step(ctx, qd, pd, f, 0.1, 5)
    assert np.abs(host(qd) - qo).max() < 1e-12 and np.abs(host(pd) - po).max() < 1e-12
    assert np.abs(host(f) - fo).max() < 1e-12


@pytest.mark.parametrize("n,unaligned", [(20_003, False), (1001, True)])
def test_hmf_angles_beyond_the_reduction_range(n, unaligned):
    """The FP64 pass reduces every angle of a thread by pi/2 in two FMA steps, exact
    for |theta| < 2^30; any angle beyond (the dynamics never reach one) is redone by
    the device library's sincos afterwards.  Such angles in vector lanes, at the
    range's edge and in the scalar tail, against the oracle's sin and cos: the
    force and the magnetization, and the force md_step leaves equal to md_force at
    the positions it leaves, bit for bit."""
    q, p = inputs.hmf_waterbag(n, seed=92)
    idx = [0, 1, 2, 3, 500, n - 2, n - 1]
    vals = [3.0e9, -2.0 ** 30, 2.0 ** 30 - 0.5, -1.1e12, 4.5e15, 2.0 ** 30, -6.0e9]
    q[0, idx] = vals
    fo = oracle.force(HMF, q)
    mo = np.array([np.cos(q[0]).sum(), np.sin(q[0]).sum()]) / n
    ctx = md.md_init(HMF, md.FP64, n, 0.0)
    put = _offset_view if unaligned else dev
    qd, pd = put(q), put(p)
    f = put(np.zeros_like(q))
    md.md_force(ctx, qd, f)
    assert np.abs(host(f) - fo).max() < 1e-13
    assert np.abs(host(md.md_magnetization(ctx, qd)) - mo).max() < 1e-13
    md.md_step(ctx, qd, pd, f, 0.1, 3)
    assert np.isfinite(host(qd)).all() and np.isfinite(host(pd)).all()
    f2 = put(np.zeros_like(q))
    md.md_force(ctx, qd, f2)
    np.testing.assert_array_equal(host(f2), host(f))
    ctx.close()


@pytest.mark.parametrize("n", [1, 2, 5, 4097, 20_003])
def test_hmf_f32state_ragged_tails(n):
    """FP32 state moves 4 particles per vector access; the n mod 4 others take the
    scalar tail path.  Energies match the oracle to the FP32-state bar."""
    q, p = inputs.hmf_waterbag(n, seed=91)
    f = oracle.force(HMF, q)
    qo, po, _ = oracle.step(HMF, q, p, f, 0.1, 10, 0.0)
    e0 = oracle.energy(HMF, q, p)
    eo = oracle.energy(HMF, qo, po)
    ctx = md.md_init(HMF, md.MIXED_F32STATE, n, 0.0)
    qd, pd = dev(q), dev(p)
    fd = torch.empty_like(qd)
    md.md_force(ctx, qd, fd)
    md.md_step(ctx, qd, pd, fd, 0.1, 10)
    eg = host(md.md_energy(ctx, qd, pd))
    scale = abs(e0[0]) + abs(e0[1]) + n / 2
    assert abs(eg[2] - eo[2]) < 1e-5 * scale
    d = host(qd) - qo
    assert np.abs(d - 2 * np.pi * np.round(d / (2 * np.pi))).max() < 1e-3


def test_autotuner_picks_and_caches(tmp_path):
    from paper_1212_0262_amd import autotune
    n = 5000
    q, _ = inputs.grav2d_disk(n, seed=92)
    ctx = md.md_init(GRAV2D, md.MIXED, n, 1e-3)
    qd = dev(q)
    cache = str(tmp_path / "tiles.json")
    configs = [(1, 4, 8, 128), (2, 2, 4, 128), (1, 1, 16, 64)]
    best, table = autotune.tune(ctx, qd, configs=configs, reps=2, cache=cache)
    assert len(table) == 3 and tuple(best) == tuple(table[0][0])
    assert md.md_get_tiles(ctx) == tuple(best)
    data = json.load(open(cache))
    assert list(data.values())[0]["tiles"] == list(best)
    other = md.md_init(GRAV2D, md.MIXED, n, 1e-3)
    assert autotune.apply_cached(other, cache) == tuple(best)
    assert md.md_get_tiles(other) == tuple(best)
    # the tuned context computes the same forces (to rounding)
    f1, f2 = torch.empty_like(qd), torch.empty_like(qd)
    md.md_force(ctx, qd, f1)
    md.md_set_tiles(other, 1, 4, 1, 128)
    md.md_force(other, qd, f2)
    assert rel_inf(host(f1), host(f2)) < 1e-5


@settings(max_examples=40, deadline=None, derandomize=True)
@given(model=st.sampled_from([RING, GRAV2D]),
       prec=st.sampled_from([md.FP64, md.MIXED, md.MIXED_KAHAN, md.MIXED_PAIRF64]),
       n=st.integers(min_value=1, max_value=700),
       ipl=st.sampled_from([1, 2, 4]), waves=st.sampled_from([1, 2, 4]),
       split=st.integers(min_value=1, max_value=64), jtile=st.sampled_from([16, 48, 128, 4096]),
       seed=st.integers(min_value=0, max_value=10_000))
def test_random_small_systems_match_oracle(model, prec, n, ipl, waves, split, jtile, seed):
    eps = 1e-3 if model == GRAV2D else 0.01
    q, _ = inputs.grav2d_disk(n, seed=seed) if model == GRAV2D else inputs.ring_waterbag(n, seed=seed)
    ctx = md.md_init(model, prec, n, eps)
    md.md_set_tiles(ctx, ipl, waves, min(split, md.md_max_j_split(n)), jtile)
    qd = dev(q)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    fo = oracle.force(model, q, eps)
    fg = host(f)
    if n == 1:
        assert np.all(fg == 0.0)
    else:
        check(f"random system model={model} prec={prec} n={n} tiles=({ipl}, {waves}, {split}, {jtile})",
              rel_inf(fg, fo), force_tol(model, prec, n, run=min(jtile, n)))


@settings(max_examples=30, deadline=None, derandomize=True)
@given(model=st.sampled_from([RING, GRAV2D]),
       prec=st.sampled_from([md.FP64, md.MIXED, md.MIXED_KAHAN, md.MIXED_PAIRF64]),
       n=st.integers(min_value=1, max_value=3000),
       ipl=st.sampled_from([1, 2, 4]),
       split=st.integers(min_value=1, max_value=64), jtile=st.sampled_from([16, 32, 80, 128, 4096]),
       seed=st.integers(min_value=0, max_value=10_000))
def test_random_fused_equals_staged(model, prec, n, ipl, split, jtile, seed):
    """Any tiles the fused launch accepts: md_step bit for bit equal to the staged
    launch (two steps, so the alternating operand buffers are both used)."""
    eps, dt = (1e-3, 0.01) if model == GRAV2D else (0.01, 0.05)
    q0, p0 = inputs.grav2d_disk(n, seed=seed) if model == GRAV2D else inputs.ring_waterbag(n, seed=seed)
    ctx = md.md_init(model, prec, n, eps)
    md.md_set_tiles(ctx, ipl, 4, min(split, md.md_max_j_split(n)), jtile)
    try:
        md.md_set_launch(ctx, md.LAUNCH_FUSED)
    except md.MDError:
        return  # tiles the fused block cannot hold: covered by the validation test
    outs = []
    for launch in (md.LAUNCH_FUSED, md.LAUNCH_STAGED):
        md.md_set_launch(ctx, launch)
        q, p = dev(q0), dev(p0)
        f = torch.empty_like(q)
        md.md_force(ctx, q, f)
        md.md_step(ctx, q, p, f, dt, 2)
        outs.append((host(q), host(p), host(f)))
    for x, y in zip(*outs):
        np.testing.assert_array_equal(x, y)
