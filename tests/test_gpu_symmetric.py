"""The symmetric launch form (MD_LAUNCH_SYMMETRIC) of the 2D and Ring models: each
pair evaluated once and added to both particles, the per-tile FP64 slots added
in a fixed order.

  * forces against the oracle at sizes that cover one and several tile pairs,
    ragged last tiles (pad particles) and both sides of the form's size range,
    in both precisions, with the staged form's tolerances (the pair terms are the
    same terms, grouped differently);
  * agreement with the staged form to FP32 rounding, and bit-identical repeated
    evaluations (no atomics);
  * the total force vanishes to rounding: the i-side and j-side terms of a pair
    are the same product with opposite signs;
  * a short trajectory against the oracle's;
  * the launch form md_get_launch reports, and the refusals of md_set_launch;
  * a graph-captured step equal to the eager step on every replay.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1212_0262_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
md = pytest.importorskip("paper_1212_0262_amd.md")
from gpu_helpers import dev, host, rel_inf  # noqa: E402
from tolerances import check, force_tol  # noqa: E402

GRAV2D, RING = md.GRAV2D, md.RING
EPS = 1e-3
PRECS = [md.MIXED, md.MIXED_KAHAN, md.MIXED_PAIRF64, md.FP64]
MODELS = [(GRAV2D, 1e-3), (RING, 0.01)]


def _state(model, n, seed):
    return inputs.grav2d_disk(n, seed=seed) if model == GRAV2D else inputs.ring_waterbag(n, seed=seed)


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield


def _force(q, launch, prec=md.MIXED, model=GRAV2D, eps=EPS):
    n = q.shape[-1]
    ctx = md.md_init(model, prec, n, eps)
    md.md_set_launch(ctx, launch)
    assert md.md_get_launch(ctx) == launch
    qd = dev(q)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    out = host(f)
    ctx.close()
    return out


@pytest.mark.parametrize("model,eps", MODELS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [2048, 2049, 3000, 4096, 5120, 9999])
def test_symmetric_force_matches_oracle(n, prec, model, eps):
    q, _ = _state(model, n, seed=300 + n)
    fo = oracle.force(model, q, eps)
    fg = _force(q, md.LAUNCH_SYMMETRIC, prec, model, eps)
    check(f"symmetric model={model} prec={prec} n={n}", rel_inf(fg, fo), force_tol(model, prec, n))


@pytest.mark.parametrize("prec", PRECS)
def test_symmetric_force_clustered_state(prec):
    """Two tight clusters far apart (large |F| from close pairs, and pairs that
    cross tiles between the clusters)."""
    n = 6000
    rng = np.random.default_rng(17)
    q = np.concatenate([rng.normal(-0.5, 0.02, size=(2, n // 2)), rng.normal(0.5, 0.02, size=(2, n - n // 2))], axis=1)
    q = q[:, rng.permutation(n)]
    fo = oracle.force(GRAV2D, q, EPS)
    fg = _force(q, md.LAUNCH_SYMMETRIC, prec)
    check(f"symmetric clustered prec={prec} n={n}", rel_inf(fg, fo), force_tol(GRAV2D, prec, n, clustered=True))


@pytest.mark.parametrize("model,eps", MODELS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [40_000, 65_537, 100_000, 131_073])
def test_symmetric_against_staged(n, prec, model, eps):
    """Both forms sum the same pair terms in different groupings.  The sizes take each
    tile size: 256 up to 65,536, then 1024 (2D) or 512 (Ring, up to 131,072)."""
    q, _ = _state(model, n, seed=7)
    fs = _force(q, md.LAUNCH_SYMMETRIC, prec, model, eps)
    ft = _force(q, md.LAUNCH_STAGED, prec, model, eps)
    tol = force_tol(model, prec, n)
    check(f"symmetric vs staged model={model} prec={prec} n={n}", rel_inf(fs, ft), tol)
    rows = np.concatenate([np.random.default_rng(n).choice(n, size=16, replace=False), [0, n - 1]])
    fo = oracle.force_rows(model, q, rows, eps)
    check(f"symmetric rows model={model} prec={prec} n={n}", rel_inf(fs[..., rows], fo), tol)


@pytest.mark.parametrize("model,eps", MODELS)
@pytest.mark.parametrize("prec", PRECS)
def test_symmetric_repeatable_and_momentum_free(prec, model, eps):
    n = 70_001
    q, _ = _state(model, n, seed=11)
    ctx = md.md_init(model, prec, n, eps)
    assert md.md_get_launch(ctx) == md.LAUNCH_SYMMETRIC
    qd = dev(q)
    f1, f2 = torch.empty_like(qd), torch.empty_like(qd)
    md.md_force(ctx, qd, f1)
    md.md_force(ctx, qd, f2)
    assert torch.equal(f1, f2)
    fh = host(f1).reshape(-1, n)
    total = np.abs(fh.sum(axis=1)).max()
    scale = np.abs(fh).sum(axis=1).max()
    print(f"symmetric model={model} prec={prec} |sum f| = {total:.3e} of sum |f| = {scale:.3e}")
    assert total < (1e-13 if prec == md.FP64 else 1e-6) * scale
    ctx.close()


@pytest.mark.parametrize("model,eps,dt", [(GRAV2D, 1e-3, 0.01), (RING, 0.01, 0.05)])
@pytest.mark.parametrize("prec", PRECS)
def test_symmetric_trajectory_matches_oracle(prec, model, eps, dt):
    n, nst = 4096, 10
    q0, p0 = _state(model, n, seed=21)
    f0 = oracle.force(model, q0, eps)
    qo, po, _ = oracle.step(model, q0, p0, f0, dt, nst, eps)
    ctx = md.md_init(model, prec, n, eps)
    md.md_set_launch(ctx, md.LAUNCH_SYMMETRIC)
    qd, pd = dev(q0), dev(p0)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    md.md_step(ctx, qd, pd, f, dt, nst)
    eq = np.abs(host(qd) - qo).max()
    ep = np.abs(host(pd) - po).max()
    e0 = oracle.energy(model, q0, p0, eps)
    eg = host(md.md_energy(ctx, qd, pd))
    eo = oracle.energy(model, qo, po, eps)
    de = abs(eg[2] - eo[2]) / (abs(e0[0]) + abs(e0[1]))
    print(f"symmetric trajectory model={model} prec={prec}: max|dq|={eq:.3e} max|dp|={ep:.3e} energy diff={de:.3e}")
    if prec != md.FP64:
        assert eq < 1e-5 and ep < 1e-4 and de < 1e-5
    else:  # the FP64 trajectory tolerance of the staged form
        assert eq < 1e-11 and ep < 1e-9 and de < 1e-12
    ctx.close()


@pytest.mark.parametrize("model,eps", MODELS)
def test_symmetric_at_the_maximum_size(model, eps):
    """n = 2^20, the largest n the form accepts (1024 tiles; the slots take 8 GB
    for Ring, 16 GB for 2D): sampled rows of the automatic (symmetric) mixed form
    against the oracle."""
    n = 1 << 20
    q, _ = _state(model, n, seed=41)
    ctx = md.md_init(model, md.MIXED, n, eps)
    assert md.md_get_launch(ctx) == md.LAUNCH_SYMMETRIC
    qd = dev(q)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    rows = np.concatenate([np.random.default_rng(41).choice(n, size=16, replace=False), [0, 1023, 1024, n - 1]])
    fo = oracle.force_rows(model, q, rows, eps)
    check(f"symmetric model={model} n={n} sampled rows", rel_inf(host(f)[..., rows], fo),
          force_tol(model, md.MIXED, n))
    ctx.close()


@pytest.mark.parametrize("model,prec,n", [
    (GRAV2D, md.MIXED, 267_044),        # 261 tiles: FP32 slots, 4 particles a thread, 5 slots past the trees
    (GRAV2D, md.FP64, 134_127),         # 131 tiles: FP64 slots, 2 particles a thread, 3 past the trees
    (RING, md.MIXED_KAHAN, 135_000),    # 132 tiles: 4 past the trees
])
def test_symmetric_vector_update_ragged_slot_count(model, prec, n):
    """Sizes where the update reads the slots with 16-byte loads (several particles a
    thread) and the slot count is not a multiple of the 8-slot trees, so the last
    slots take the one-by-one path: sampled rows (first and last tile, the last
    particles before the pads) against the oracle."""
    eps = EPS if model == GRAV2D else 0.01
    q, _ = _state(model, n, seed=43)
    ctx = md.md_init(model, prec, n, eps)
    assert md.md_get_launch(ctx) == md.LAUNCH_SYMMETRIC
    qd = dev(q)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    rng = np.random.default_rng(43)
    rows = np.concatenate([rng.choice(n, size=12, replace=False), [0, 1023, n - 1025, n - 2, n - 1]])
    fo = oracle.force_rows(model, q, rows, eps)
    check(f"symmetric vector update model={model} prec={prec} n={n} sampled rows", rel_inf(host(f)[..., rows], fo),
          force_tol(model, prec, n))
    ctx.close()


def test_sym_tile_sizes():
    """The tile of the symmetric form (md_get_sym_tile): 256 up to 65,536 particles, then
    512 for the Ring up to 131,072 and 1024 otherwise; 0 when another form runs."""
    for model, n, tile in [(GRAV2D, 20_000, 256), (GRAV2D, 65_536, 256), (GRAV2D, 65_537, 1024),
                           (RING, 65_536, 256), (RING, 65_537, 512), (RING, 131_072, 512), (RING, 131_073, 1024)]:
        ctx = md.md_init(model, md.MIXED, n, EPS)
        assert md.md_get_launch(ctx) == md.LAUNCH_SYMMETRIC
        assert md.md_get_sym_tile(ctx) == tile, (model, n)
        md.md_set_launch(ctx, md.LAUNCH_STAGED)
        assert md.md_get_sym_tile(ctx) == 0
        ctx.close()
    b = md.md_batch_init(RING, md.MIXED_KAHAN, [0, 8000, 16000], [0.01] * 2)
    md.md_set_launch(b, md.LAUNCH_SYMMETRIC)
    assert md.md_get_sym_tile(b) == 512                        # ensembles: tiles of 512
    b.close()


def test_launch_form_and_refusals():
    big = md.md_init(GRAV2D, md.MIXED, md.SYMMETRIC_AUTO_N, EPS)
    assert md.md_get_launch(big) == md.LAUNCH_SYMMETRIC
    big64 = md.md_init(GRAV2D, md.FP64, md.SYMMETRIC_AUTO_N, EPS)
    assert md.md_get_launch(big64) == md.LAUNCH_SYMMETRIC
    # the Ring's own thresholds (its symmetric form gains more per pair than 2D's)
    for prec, n0 in ((md.MIXED, md.SYMMETRIC_AUTO_N_RING), (md.FP64, md.SYMMETRIC_AUTO_N_RING64)):
        ring = md.md_init(RING, prec, n0, 0.01)
        assert md.md_get_launch(ring) == md.LAUNCH_SYMMETRIC
        ring_below = md.md_init(RING, prec, n0 - 1, 0.01)
        assert md.md_get_launch(ring_below) == md.LAUNCH_STAGED
        ring.close()
        ring_below.close()
    below = md.md_init(GRAV2D, md.MIXED, md.SYMMETRIC_AUTO_N - 1, EPS)
    assert md.md_get_launch(below) != md.LAUNCH_SYMMETRIC
    md.md_set_launch(below, md.LAUNCH_SYMMETRIC)
    assert md.md_get_launch(below) == md.LAUNCH_SYMMETRIC
    md.md_set_launch(big, md.LAUNCH_STAGED)
    assert md.md_get_launch(big) == md.LAUNCH_STAGED
    md.md_set_launch(big, md.LAUNCH_AUTO)
    assert md.md_get_launch(big) == md.LAUNCH_SYMMETRIC
    # every FP32 accumulation takes the form (the 2D compensated forms share one threshold, the Ring FP32
    # forms another)
    for model, prec, n0 in [(GRAV2D, md.MIXED_KAHAN, md.SYMMETRIC_AUTO_N_COMP),
                            (GRAV2D, md.MIXED_PAIRF64, md.SYMMETRIC_AUTO_N_COMP),
                            (RING, md.MIXED_KAHAN, md.SYMMETRIC_AUTO_N_RING),
                            (RING, md.MIXED_PAIRF64, md.SYMMETRIC_AUTO_N_RING)]:
        for n, form in ((n0, md.LAUNCH_SYMMETRIC), (n0 - 1, md.LAUNCH_STAGED)):
            ctx = md.md_init(model, prec, n, EPS)
            assert md.md_get_launch(ctx) == form, (model, prec, n)
            ctx.close()
    for model, prec, n in [(GRAV2D, md.MIXED, 2047), (GRAV2D, md.FP64, 2047), (RING, md.FP64, 2047),
                           (RING, md.MIXED_KAHAN, 2047), (GRAV2D, md.MIXED_PAIRF64, 2047),
                           (GRAV2D, md.MIXED, (1 << 20) + 1), (RING, md.MIXED, (1 << 20) + 1)]:
        ctx = md.md_init(model, prec, n, EPS)
        assert md.md_get_launch(ctx) != md.LAUNCH_SYMMETRIC
        with pytest.raises(md.MDError):
            md.md_set_launch(ctx, md.LAUNCH_SYMMETRIC)
        ctx.close()
    batch = md.md_batch_init(GRAV2D, md.FP64, [0, 3000, 6000], EPS)  # no symmetric FP64 2D ensembles
    with pytest.raises(md.MDError):
        md.md_set_launch(batch, md.LAUNCH_SYMMETRIC)
    for c in (big, big64, below, batch):
        c.close()


def test_symmetric_step_graph_replays():
    n, dt = 5000, 0.01
    q0, p0 = inputs.grav2d_disk(n, seed=31)
    ctx = md.md_init(GRAV2D, md.MIXED, n, EPS)
    md.md_set_launch(ctx, md.LAUNCH_SYMMETRIC)
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
    for rep in range(3):
        qg.copy_(q); pg.copy_(p); fg.copy_(f)
        torch.cuda.synchronize()
        g.replay(); g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(qg), host(qe))
        np.testing.assert_array_equal(host(pg), host(pe))
        np.testing.assert_array_equal(host(fg), host(fe))
    ctx.close()


# ------------------------------------------------------------------ ensembles --

BATCH_SIZES = [1, 700, 1024, 1025, 2048, 3000, 5000]


def _ensemble(model, sizes, seed):
    qs, ps = [], []
    for b, n in enumerate(sizes):
        q, p = inputs.grav2d_disk(n, seed=seed + b) if model == GRAV2D else inputs.ensemble_member(b, n, seed=seed)
        qs.append(q)
        ps.append(p)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return np.concatenate(qs, axis=1), np.concatenate(ps, axis=1), off


def _batch_force(model, prec, q, off, eps_b, launch):
    ctx = md.md_batch_init(model, prec, off, eps_b)
    md.md_set_launch(ctx, launch)
    assert md.md_get_launch(ctx) == launch
    qd = dev(q)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    out = host(f)
    ctx.close()
    return out


@pytest.mark.parametrize("model,prec,eps", [(RING, md.MIXED, 0.01), (RING, md.MIXED_KAHAN, 0.01), (RING, md.FP64, 0.01),
                                            (GRAV2D, md.MIXED, 1e-3), (GRAV2D, md.MIXED_KAHAN, 1e-3)])
def test_symmetric_ensemble_matches_oracle(model, prec, eps):
    """Every realization (ragged last tiles, single-tile and one-particle ones,
    uneven eps) against the oracle on that realization alone."""
    q, _, off = _ensemble(model, BATCH_SIZES, seed=50)
    eps_b = np.full(len(BATCH_SIZES), eps)
    eps_b[-2] = 2 * eps
    f = _batch_force(model, prec, q, off, eps_b, md.LAUNCH_SYMMETRIC)
    for b, n in enumerate(BATCH_SIZES):
        qb, fb = q[:, off[b]:off[b + 1]], f[:, off[b]:off[b + 1]]
        if n == 1:
            assert np.all(fb == 0.0)
            continue
        check(f"symmetric ensemble model={model} prec={prec} N_b={n}", rel_inf(fb, oracle.force(model, qb, eps_b[b])),
              force_tol(model, prec, n))


def test_symmetric_ensemble_against_staged_and_repeatable():
    sizes = [3000, 9000, 16384, 12000, 1500]
    q, _, off = _ensemble(RING, sizes, seed=60)
    eps_b = np.full(len(sizes), 0.01)
    fs = _batch_force(RING, md.MIXED_KAHAN, q, off, eps_b, md.LAUNCH_SYMMETRIC)
    ft = _batch_force(RING, md.MIXED_KAHAN, q, off, eps_b, md.LAUNCH_STAGED)
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        check(f"symmetric vs staged ensemble N_b={sizes[b]}", rel_inf(fs[:, sl], ft[:, sl]),
              force_tol(RING, md.MIXED_KAHAN, sizes[b]))
    assert np.array_equal(fs, _batch_force(RING, md.MIXED_KAHAN, q, off, eps_b, md.LAUNCH_SYMMETRIC))


def test_symmetric_ensemble_step_and_graph():
    """A few steps of a Ring ensemble in the symmetric form against the oracle per
    realization, and the same steps graph-captured, equal on every replay."""
    sizes = [2048, 5000, 1024, 3500]
    q0, p0, off = _ensemble(RING, sizes, seed=70)
    eps_b = np.full(len(sizes), 0.01)
    ctx = md.md_batch_init(RING, md.MIXED_KAHAN, off, eps_b)
    md.md_set_launch(ctx, md.LAUNCH_SYMMETRIC)
    s = torch.cuda.Stream()
    md.md_set_stream(ctx, s)
    q, p = dev(q0), dev(p0)
    f = torch.empty_like(q)
    with torch.cuda.stream(s):
        md.md_force(ctx, q, f)
    s.synchronize()
    qe, pe, fe = q.clone(), p.clone(), f.clone()
    with torch.cuda.stream(s):
        md.md_step(ctx, qe, pe, fe, 0.05, 4)
    s.synchronize()
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        fo = oracle.force(RING, q0[:, sl], 0.01)
        qo, po, _ = oracle.step(RING, q0[:, sl], p0[:, sl], fo, 0.05, 4, 0.01)
        assert np.abs(host(qe)[:, sl] - qo).max() < 1e-5
        assert np.abs(host(pe)[:, sl] - po).max() < 1e-4
    g = torch.cuda.CUDAGraph()
    qg, pg, fg = q.clone(), p.clone(), f.clone()
    with torch.cuda.graph(g, stream=s):
        md.md_step(ctx, qg, pg, fg, 0.05, 2)
    for rep in range(3):
        qg.copy_(q); pg.copy_(p); fg.copy_(f)
        torch.cuda.synchronize()
        g.replay(); g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(qg), host(qe))
        np.testing.assert_array_equal(host(pg), host(pe))
    ctx.close()


def test_symmetric_ensemble_launch_form_and_refusals():
    small = md.md_batch_init(RING, md.MIXED_KAHAN, [0, 500, 1500, 2000], [0.01] * 3)
    assert md.md_get_launch(small) == md.LAUNCH_STAGED          # more diagonal tiles than tile pairs
    big = md.md_batch_init(RING, md.MIXED_KAHAN, [0, 8000, 16000], [0.01] * 2)
    assert md.md_get_launch(big) == md.LAUNCH_SYMMETRIC
    md.md_set_launch(big, md.LAUNCH_STAGED)
    assert md.md_get_launch(big) == md.LAUNCH_STAGED
    with pytest.raises(md.MDError):
        md.md_set_launch(big, md.LAUNCH_FUSED)
    for model, prec in [(GRAV2D, md.FP64), (RING, md.MIXED_PAIRF64), (GRAV2D, md.MIXED_PAIRF64)]:
        c = md.md_batch_init(model, prec, [0, 3000, 9000], [0.01] * 2)
        assert md.md_get_launch(c) == md.LAUNCH_STAGED
        with pytest.raises(md.MDError):
            md.md_set_launch(c, md.LAUNCH_SYMMETRIC)
        c.close()
    for c in (small, big):
        c.close()


def test_autotuner_times_the_symmetric_form_once():
    """The symmetric form has no tile choice: tune() times it once and leaves the tiles."""
    from paper_1212_0262_amd import autotune
    n = md.SYMMETRIC_AUTO_N
    q, _ = inputs.grav2d_disk(n, seed=81)
    ctx = md.md_init(GRAV2D, md.MIXED, n, EPS)
    assert md.md_get_launch(ctx) == md.LAUNCH_SYMMETRIC
    tiles = md.md_get_tiles(ctx)
    best, table = autotune.tune(ctx, dev(q), configs=[(1, 4, 8, 128), (2, 2, 4, 128)], reps=1, cache=None)
    assert len(table) == 1 and tuple(best) == tuple(tiles) and md.md_get_tiles(ctx) == tuple(tiles)
    ctx.close()


# ------------------------------------------------------------ random cases --

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402


@settings(max_examples=25, deadline=None, derandomize=True)
@given(model=st.sampled_from([RING, GRAV2D]), prec=st.sampled_from([md.MIXED, md.FP64]),
       n=st.integers(min_value=2048, max_value=7000), eps_scale=st.sampled_from([0.1, 1.0, 10.0]),
       seed=st.integers(min_value=0, max_value=10_000))
def test_random_symmetric_systems_match_oracle(model, prec, n, eps_scale, seed):
    """Random sizes (one to seven tiles, ragged or not), eps and seeds: the
    symmetric form against the oracle with the staged form's tolerances."""
    eps = (1e-3 if model == GRAV2D else 0.01) * eps_scale
    q, _ = _state(model, n, seed=seed)
    fg = _force(q, md.LAUNCH_SYMMETRIC, prec, model, eps)
    check(f"random symmetric model={model} prec={prec} n={n} eps={eps}", rel_inf(fg, oracle.force(model, q, eps)),
          force_tol(model, prec, n, eps=eps))


@settings(max_examples=15, deadline=None, derandomize=True)
@given(prec=st.sampled_from([md.MIXED, md.MIXED_KAHAN, md.FP64]),
       sizes=st.lists(st.integers(min_value=1, max_value=4500), min_size=1, max_size=6),
       seed=st.integers(min_value=0, max_value=10_000))
def test_random_symmetric_ensembles_match_oracle(prec, sizes, seed):
    """Random Ring ensembles (any mix of single-particle, single-tile and
    multi-tile realizations) in the symmetric form, per realization against the
    oracle."""
    q, _, off = _ensemble(RING, sizes, seed=seed)
    eps_b = np.full(len(sizes), 0.01)
    f = _batch_force(RING, prec, q, off, eps_b, md.LAUNCH_SYMMETRIC)
    for b, n in enumerate(sizes):
        sl = slice(off[b], off[b + 1])
        if n == 1:
            assert np.all(f[:, sl] == 0.0)
        else:
            check(f"random symmetric ensemble prec={prec} N_b={n}", rel_inf(f[:, sl], oracle.force(RING, q[:, sl], 0.01)),
                  force_tol(RING, prec, n))


# ------------------------------------------------------- coincident angles --

def test_ring_fp64_symmetric_coincident_angles():
    """Ring FP64, symmetric launch: a tile pair forms eq. 9's numerator
    sin ti cos tj - cos ti sin tj as one product and one FMA, so for two particles
    at exactly the same angle in different tiles it is the rounding error of
    cos t sin t, at most 2^-53 |cos t sin t|, instead of 0; u = 1 + eps - cos 0 is
    eps to within a few ulp of 1.  Each such pair adds + on the lower tile's
    particle and - on the higher one's, with the prefactor 1/(2 sqrt2 N), so in an
    all-equal state (whose forces vanish) no force exceeds
    (N - 1)/(2 sqrt2 N) 2^-53 |cos t sin t| eps^{-3/2}.  The staged form gives
    exactly 0."""
    n, eps, th = 12_288, 0.01, 0.7
    bound = (n - 1) / (2 * np.sqrt(2) * n) * 2.0 ** -53 * abs(np.cos(th) * np.sin(th)) * (eps * (1 - 1e-12)) ** -1.5
    q = np.full((1, n), th)
    fs = _force(q, md.LAUNCH_SYMMETRIC, md.FP64, RING, eps)
    ft = _force(q, md.LAUNCH_STAGED, md.FP64, RING, eps)
    print(f"all-equal state FP64: max |f| symmetric {np.abs(fs).max():.3e} (bound {bound:.3e}), "
          f"staged {np.abs(ft).max():.1e}")
    assert np.all(ft == 0.0)
    assert np.abs(fs).max() <= 1.01 * bound


def test_ring_fp32_symmetric_coincident_angles():
    """Ring FP32 forms, symmetric launch: a tile pair forms the half-angle
    numerator a = 2 sin(d/2) as one product and one FMA (one rounding fewer than
    the staged form's two rounded products, which make it exactly antisymmetric).
    For two particles at exactly the same angle in different tiles a is then the
    rounding error of the product A B, |a| <= 2^-24 |A B|, instead of 0.  The term
    a b r'^3, with b = A^2 + B^2 = 2 and r' = (a^2 + 2 eps)^{-1/2}, is then at most
    2^-24 |A B| b (2 eps)^{-3/2}; it is the same for every such pair, added with
    + on the lower tile's particle and - on the higher one's, so the force
    (prefactor 1/(2N)) on a particle of an all-equal state, which should vanish,
    is at most (N - 1)/(2N) times that.  The staged form gives exactly 0 there.  A waterbag state with angles duplicated across tiles still
    meets the parity tolerance."""
    n, eps = 40_960, 0.01
    th = 0.7
    A = np.float32(np.sqrt(2.0) * np.sin(th / 2))
    B = np.float32(np.sqrt(2.0) * np.cos(th / 2))
    b = float(A) ** 2 + float(B) ** 2
    bound = (n - 1) / (2 * n) * 2.0 ** -24 * abs(float(A) * float(B)) * b * (2 * eps) ** -1.5
    q = np.full((1, n), th)
    for prec in (md.MIXED, md.MIXED_KAHAN, md.MIXED_PAIRF64):
        fs = _force(q, md.LAUNCH_SYMMETRIC, prec, RING, eps)
        ft = _force(q, md.LAUNCH_STAGED, prec, RING, eps)
        print(f"all-equal state prec={prec}: max |f| symmetric {np.abs(fs).max():.3e} (bound {bound:.3e}), "
              f"staged {np.abs(ft).max():.1e}")
        assert np.all(ft == 0.0)
        assert np.abs(fs).max() <= 1.01 * bound
    # a waterbag state where every particle of tile 0 reappears in tiles 5, 17 and 39
    q, _ = inputs.ring_waterbag(n, seed=19)
    for t in (5, 17, 39):
        q[0, t * 1024:(t + 1) * 1024] = q[0, :1024]
    rows = np.concatenate([np.arange(0, 1024, 97), np.arange(5 * 1024, 6 * 1024, 101), [n - 1]])
    fo = oracle.force_rows(RING, q, rows, eps)
    for prec in (md.MIXED, md.MIXED_KAHAN):
        fs = _force(q, md.LAUNCH_SYMMETRIC, prec, RING, eps)
        check(f"duplicated angles prec={prec}", rel_inf(fs[:, rows], fo), force_tol(RING, prec, n))
