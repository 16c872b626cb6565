"""The fused small-N launch (one launch per force evaluation) against the staged
launch (pair kernel + update kernel): for the same tiles both add the same pair
terms in the same order, so md_step's results agree bit for bit.  Also the form
md_get_launch reports, the validation of md_set_launch, and a fused run against
the FP64 oracle."""
import os

import numpy as np
import pytest

import oracle
from paper_1212_0262_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
md = pytest.importorskip("paper_1212_0262_amd.md")
from gpu_helpers import dev, host, rel_inf  # noqa: E402

RING, GRAV2D = md.RING, md.GRAV2D
PRECS = [md.FP64, md.MIXED, md.MIXED_KAHAN, md.MIXED_PAIRF64]


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield


def _state(model, n, seed):
    return inputs.grav2d_disk(n, seed=seed) if model == GRAV2D else inputs.ring_waterbag(n, seed=seed)


def _groups(split):
    g = 1
    while g < 8 and split % (2 * g) == 0:
        g *= 2
    return g


def _fused_fits(model, ipl, split):
    """The library's rule: split / lane groups <= 16 wavefronts, and each
    wavefront's LDS slice (48 KiB / wavefronts) holds its partials."""
    S = split // _groups(split)
    return S <= 16 and ipl * (2 if model == GRAV2D else 1) * 64 * 8 <= 49152 // S


def _run(model, prec, n, eps, dt, nsteps, tiles, launch, seed):
    q0, p0 = _state(model, n, seed)
    ctx = md.md_init(model, prec, n, eps)
    md.md_set_tiles(ctx, *tiles)
    md.md_set_launch(ctx, launch)
    assert md.md_get_launch(ctx) == launch
    q, p = dev(q0), dev(p0)
    f = torch.empty_like(q)
    md.md_force(ctx, q, f)
    md.md_step(ctx, q, p, f, dt, nsteps)
    return host(q), host(p), host(f)


@pytest.mark.parametrize("n", [1, 2, 63, 100, 1000, 2048, 5001])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("model,eps,dt", [(RING, 0.01, 0.05), (GRAV2D, 1e-3, 0.01)])
def test_fused_equals_staged_bitwise(model, eps, dt, prec, n):
    """Default tiles, and the most j ranges (8 lane groups of 8 wavefronts)."""
    for split in (0, min(64, md.md_max_j_split(n))):
        tiles = (1, 4, split, 128)
        a = _run(model, prec, n, eps, dt, 3, tiles, md.LAUNCH_STAGED, seed=80 + n)
        b = _run(model, prec, n, eps, dt, 3, tiles, md.LAUNCH_FUSED, seed=80 + n)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("ipl,split,jtile", [(1, 1, 16), (2, 3, 48), (4, 8, 4096), (2, 16, 128), (1, 5, 64),
                                             (1, 2, 32), (2, 6, 16), (1, 12, 48), (4, 24, 128), (2, 40, 64),
                                             (1, 64, 16), (4, 13, 128)])
@pytest.mark.parametrize("model,eps,dt", [(RING, 0.01, 0.05), (GRAV2D, 1e-3, 0.01)])
def test_fused_tile_shapes(model, eps, dt, ipl, split, jtile):
    """Tile shapes over 1, 2, 4 and 8 lane groups, ragged n: still bit for bit the
    staged result."""
    n = 3001
    tiles = (ipl, 4, split, jtile)
    if not _fused_fits(model, ipl, split):  # the library refuses the fused form for these tiles
        ctx = md.md_init(model, md.FP64, n, eps)
        md.md_set_tiles(ctx, *tiles)
        with pytest.raises(md.MDError) as ei:
            md.md_set_launch(ctx, md.LAUNCH_FUSED)
        assert ei.value.status == md.EUNSUPPORTED
        assert md.md_get_launch(ctx) == md.LAUNCH_STAGED
        ctx.close()
        return
    for prec in (md.FP64, md.MIXED):
        a = _run(model, prec, n, eps, dt, 2, tiles, md.LAUNCH_STAGED, seed=81)
        b = _run(model, prec, n, eps, dt, 2, tiles, md.LAUNCH_FUSED, seed=81)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_auto_launch_form_and_validation():
    small = md.md_init(RING, md.FP64, 2048, 0.01)
    assert md.md_get_launch(small) == md.LAUNCH_FUSED          # n <= 4096 and the built-in tiles fit
    assert md.md_get_tiles(small) == (1, 4, 64, 128)
    for model, n_fused in ((RING, 4096), (GRAV2D, 6144)):     # the automatic sizes, per model
        for n, form in ((n_fused, md.LAUNCH_FUSED), (n_fused + 1, md.LAUNCH_STAGED)):
            ctx = md.md_init(model, md.MIXED, n, 1e-3)
            assert md.md_get_launch(ctx) == form, (model, n)
            md.md_destroy(ctx)
    big = md.md_init(GRAV2D, md.FP64, 12288, 1e-3)
    assert md.md_get_launch(big) == md.LAUNCH_STAGED           # above the fused form's automatic size
    md.md_set_launch(big, md.LAUNCH_FUSED)
    assert md.md_get_launch(big) == md.LAUNCH_FUSED
    with pytest.raises(md.MDError):                             # 17 wavefronts (odd split: one lane group)
        md.md_set_tiles(big, 1, 4, 17, 128)
    with pytest.raises(md.MDError):                             # 13 wavefronts x 4 KiB of partials > 48 KiB
        md.md_set_tiles(big, 4, 4, 13, 128)
    assert md.md_get_tiles(big)[2] == 64                        # unchanged by the refused calls
    md.md_set_launch(big, md.LAUNCH_STAGED)
    md.md_set_tiles(big, 1, 4, 17, 128)
    assert md.md_get_launch(big) == md.LAUNCH_STAGED
    with pytest.raises(md.MDError):
        md.md_set_launch(big, md.LAUNCH_FUSED)
    md.md_set_launch(big, md.LAUNCH_AUTO)
    assert md.md_get_launch(big) == md.LAUNCH_STAGED
    huge = md.md_init(GRAV2D, md.FP64, 70000, 1e-3)              # no fused operand buffers
    with pytest.raises(md.MDError):
        md.md_set_launch(huge, md.LAUNCH_FUSED)
    hmf = md.md_init(md.HMF, md.FP64, 1000, 0.0)
    assert md.md_get_launch(hmf) == md.LAUNCH_STAGED
    with pytest.raises(md.MDError):
        md.md_set_launch(hmf, md.LAUNCH_FUSED)
    batch = md.md_batch_init(RING, md.FP64, [0, 500, 1200], 0.01)
    assert md.md_get_launch(batch) == md.LAUNCH_STAGED
    with pytest.raises(md.MDError):
        md.md_set_launch(small, 7)


@pytest.mark.parametrize("model,eps,dt,prec,tol", [(RING, 0.01, 0.05, md.FP64, 1e-10), (GRAV2D, 1e-3, 0.01, md.FP64, 1e-10),
                                                   (RING, 0.01, 0.05, md.MIXED, 1e-5), (GRAV2D, 1e-3, 0.01, md.MIXED, 1e-4)])
def test_fused_trajectory_matches_oracle(model, eps, dt, prec, tol):
    n, nst = 2048, 5
    q0, p0 = _state(model, n, seed=82)
    f0 = oracle.force(model, q0, eps)
    qo, po, fo = oracle.step(model, q0, p0, f0, dt, nst, eps)
    ctx = md.md_init(model, prec, n, eps)
    assert md.md_get_launch(ctx) == md.LAUNCH_FUSED
    q, p = dev(q0), dev(p0)
    f = torch.empty_like(q)
    md.md_force(ctx, q, f)
    md.md_step(ctx, q, p, f, dt, nst)
    assert rel_inf(host(q), qo) < tol and rel_inf(host(p), po) < tol and rel_inf(host(f), fo) < 10 * tol


def test_fused_step_is_graph_capturable():
    n, eps, dt = 2048, 0.01, 0.05
    q0, p0 = _state(RING, n, seed=83)
    ctx = md.md_init(RING, md.FP64, n, eps)
    s = torch.cuda.Stream()
    md.md_set_stream(ctx, s)
    q, p = dev(q0), dev(p0)
    f = torch.empty_like(q)
    with torch.cuda.stream(s):
        md.md_force(ctx, q, f)
    s.synchronize()
    qe, pe, fe = q.clone(), p.clone(), f.clone()
    with torch.cuda.stream(s):
        md.md_step(ctx, qe, pe, fe, dt, 4)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    qg, pg, fg = q.clone(), p.clone(), f.clone()
    with torch.cuda.graph(g, stream=s):
        md.md_step(ctx, qg, pg, fg, dt, 2)
    for rep in range(2):
        qg.copy_(q); pg.copy_(p); fg.copy_(f)
        torch.cuda.synchronize()
        g.replay(); g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(qg), host(qe))
        np.testing.assert_array_equal(host(pg), host(pe))
        np.testing.assert_array_equal(host(fg), host(fe))
