"""md_timing_begin / md_timing_end: the measurement hook that brackets each launch
of a context's dominant kernel with HIP events on its stream.

  * one timed launch per force evaluation in every launch form (symmetric tile
    pairs, staged, fused, the HMF stage pass, ensembles), named after its kernel;
  * the count stops at max_launches;
  * results are bit-identical with timing on and off;
  * launches enqueued under graph capture are not timed, and the graph's replays
    equal the eager run;
  * the timed durations fit inside the elapsed time of the region;
  * md_timing_end without md_timing_begin is MD_ESTATE.
"""
import numpy as np
import pytest

from paper_1212_0262_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
md = pytest.importorskip("paper_1212_0262_amd.md")
from gpu_helpers import dev, host  # noqa: E402

# model, precision, n, eps, launch form (None: HMF), timed kernel, timed launches of md_step(2)
CASES = [
    (md.GRAV2D, md.MIXED, 65536, 1e-3, md.LAUNCH_SYMMETRIC, "k_sym (2D)", 6),
    (md.RING, md.FP64, 4096, 0.01, md.LAUNCH_SYMMETRIC, "k_sym (Ring)", 6),
    (md.GRAV2D, md.MIXED, 5000, 1e-3, md.LAUNCH_STAGED, "k_pair_2d", 6),
    (md.RING, md.MIXED, 5000, 0.01, md.LAUNCH_STAGED, "k_pair_win", 6),
    (md.RING, md.FP64, 5000, 0.01, md.LAUNCH_STAGED, "k_pair_ring", 6),
    (md.GRAV2D, md.FP64, 2048, 1e-3, md.LAUNCH_FUSED, "k_fused", 6),
    (md.HMF, md.FP64, 100_000, 0.0, None, "k_hmf_pass", 7),  # the first pass, then three per step
]


def _state(model, n, seed=5):
    if model == md.GRAV2D:
        return inputs.grav2d_disk(n, seed=seed)
    if model == md.RING:
        return inputs.ring_waterbag(n, seed=seed)
    return inputs.hmf_waterbag(n, seed=seed)


def _run(ctx, q0, p0, nsteps, timed, max_launches=64):
    q, p = dev(q0), dev(p0)
    f = torch.empty_like(q)
    md.md_force(ctx, q, f)
    torch.cuda.synchronize()
    if timed:
        md.md_timing_begin(ctx, max_launches)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    md.md_step(ctx, q, p, f, 0.01, nsteps)
    e1.record()
    torch.cuda.synchronize()
    res = md.md_timing_end(ctx) if timed else None
    return host(q), host(p), host(f), res, e0.elapsed_time(e1)


@pytest.mark.parametrize("model,prec,n,eps,launch,name,launches", CASES)
def test_timed_launches_named_counted_and_bit_identical(model, prec, n, eps, launch, name, launches):
    q0, p0 = _state(model, n)
    ctx = md.md_init(model, prec, n, eps)
    if launch is not None:
        md.md_set_launch(ctx, launch)
        assert md.md_get_launch(ctx) == launch
    qa, pa, fa, _, _ = _run(ctx, q0, p0, 2, timed=False)
    qb, pb, fb, (ms, count, kname), elapsed = _run(ctx, q0, p0, 2, timed=True)
    ctx.close()
    assert kname == name
    assert count == launches
    assert 0.0 < ms <= elapsed * 1.05 + 0.05
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(pa, pb)
    np.testing.assert_array_equal(fa, fb)


def test_count_stops_at_max_launches_and_end_turns_timing_off():
    q0, p0 = _state(md.GRAV2D, 5000)
    ctx = md.md_init(md.GRAV2D, md.MIXED, 5000, 1e-3)
    md.md_set_launch(ctx, md.LAUNCH_STAGED)
    _, _, _, (ms, count, kname), _ = _run(ctx, q0, p0, 3, timed=True, max_launches=4)
    assert count == 4 and ms > 0.0 and kname == "k_pair_2d"
    with pytest.raises(md.MDError) as ei:
        md.md_timing_end(ctx)
    assert ei.value.status == md.ESTATE
    # begun twice: the second call starts over
    md.md_timing_begin(ctx, 8)
    md.md_timing_begin(ctx, 2)
    q, p = dev(q0), dev(p0)
    f = torch.empty_like(q)
    md.md_force(ctx, q, f)
    md.md_force(ctx, q, f)
    md.md_force(ctx, q, f)
    _, count, _ = md.md_timing_end(ctx)
    assert count == 2
    ctx.close()


def test_timing_rejects_bad_counts():
    ctx = md.md_init(md.RING, md.MIXED, 1000, 0.01)
    for bad in (0, -1, 65537):
        with pytest.raises(md.MDError) as ei:
            md.md_timing_begin(ctx, bad)
        assert ei.value.status == md.EINVAL
    ctx.close()


def test_ensemble_tile_pair_kernel_timed():
    sizes = [3000, 5000, 2048]
    qs, ps = zip(*(inputs.ensemble_member(b, n, seed=7) for b, n in enumerate(sizes)))
    q0, p0 = np.concatenate(qs, axis=1), np.concatenate(ps, axis=1)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ctx = md.md_batch_init(md.RING, md.MIXED, off, [0.01] * len(sizes))
    md.md_set_launch(ctx, md.LAUNCH_SYMMETRIC)
    qa, pa, fa, _, _ = _run(ctx, q0, p0, 2, timed=False)
    qb, pb, fb, (ms, count, kname), _ = _run(ctx, q0, p0, 2, timed=True)
    assert kname == "k_batch_sym" and count == 6 and ms > 0.0
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(fa, fb)
    md.md_set_launch(ctx, md.LAUNCH_STAGED)
    _, _, _, (_, count, kname), _ = _run(ctx, q0, p0, 1, timed=True)
    assert kname == "k_batch_pair_ring_win" and count == 3
    ctx.close()


def test_capture_is_not_timed_and_replays_match_eager():
    n = 65536
    q0, p0 = _state(md.GRAV2D, n)
    s = torch.cuda.Stream()
    ctx = md.md_init(md.GRAV2D, md.MIXED, n, 1e-3, stream=s)
    q, p = dev(q0), dev(p0)
    f = torch.empty_like(q)
    with torch.cuda.stream(s):
        md.md_force(ctx, q, f)
    s.synchronize()
    qe, pe, fe = q.clone(), p.clone(), f.clone()
    with torch.cuda.stream(s):
        md.md_step(ctx, qe, pe, fe, 0.01, 2)
    s.synchronize()
    md.md_timing_begin(ctx, 16)
    g = torch.cuda.CUDAGraph()
    qg, pg, fg = q.clone(), p.clone(), f.clone()
    with torch.cuda.graph(g, stream=s):
        md.md_step(ctx, qg, pg, fg, 0.01, 2)
    _, count, _ = md.md_timing_end(ctx)
    assert count == 0
    for _ in range(3):
        qg.copy_(q)
        pg.copy_(p)
        fg.copy_(f)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(qg), host(qe))
        np.testing.assert_array_equal(host(pg), host(pe))
        np.testing.assert_array_equal(host(fg), host(fe))
    ctx.close()
