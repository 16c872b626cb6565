"""GPU parity of the derivatives: Hessian-vector products (md_hvp) and the reverse
sweep of the integrator (md_step_vjp) against the FP64 oracle, and the gradient of
the final kinetic energy (autograd.kinetic_energy_gradient) against central finite
differences of the GPU's own FP64 forward map.

Tolerances (max-norm relative to the largest oracle value):
  * Hessian-vector products: tests/tolerances.py (FP64 1e-13; FP32 forms 2e-5
    for 2D, whose 1/s^2 term doubles the sensitivity to the FP32 positions and
    whose vector w is rounded to FP32 as well, and 1e-5 for Ring, whose
    half-angle u = 1 - cos d + eps enters as u^{-5/2}).
  * FP64 reverse sweeps: 1e-9 (10 steps of products and axpys).
  * HMF products: 1e-11 -- the mean-field form (eqs. 6, 7) reorders an O(N) sum of
    O(1) terms against the oracle's pair sum; both are FP64.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1212_0262_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
md = pytest.importorskip("paper_1212_0262_amd.md")
from paper_1212_0262_amd import autograd as mdgrad  # noqa: E402
from gpu_helpers import dev, host, rel_inf  # noqa: E402
from tolerances import check, hvp_tol  # noqa: E402

HMF, RING, GRAV2D = md.HMF, md.RING, md.GRAV2D


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield


def _state(model, n, seed):
    if model == HMF:
        return inputs.hmf_waterbag(n, seed=seed)
    return inputs.grav2d_disk(n, seed=seed) if model == GRAV2D else inputs.ring_waterbag(n, seed=seed)


@pytest.mark.parametrize("n", [1, 2, 65, 257, 1000, 3001])
@pytest.mark.parametrize("prec", [md.FP64, md.MIXED, md.MIXED_KAHAN])
@pytest.mark.parametrize("model,eps", [(GRAV2D, 1e-3), (RING, 0.01)])
def test_hvp_matches_oracle(model, eps, prec, n):
    q, _ = _state(model, n, seed=60 + n)
    w = np.random.default_rng(n).normal(size=q.shape)
    ho = oracle.hvp(model, q, w, eps)
    ctx = md.md_init(model, prec, n, eps)
    hg = host(md.md_hvp(ctx, dev(q), dev(w)))
    if n == 1:
        assert np.all(hg == 0.0)
        return
    check(f"hvp model={model} prec={prec} n={n}", rel_inf(hg, ho), hvp_tol(model, prec))


@pytest.mark.parametrize("n,launch", [(2048, md.LAUNCH_SYMMETRIC), (3001, md.LAUNCH_SYMMETRIC),
                                      (5003, md.LAUNCH_SYMMETRIC), (32768, md.LAUNCH_AUTO), (70_001, md.LAUNCH_AUTO)])
def test_hvp_symmetric_matches_oracle(n, launch):
    """2D FP64 with the force in the symmetric form: the product takes it too (each
    pair evaluated once for both particles, tile-pair slots added in a fixed order),
    against the oracle and against the staged product; ragged sizes put pad particles
    in the last tile.  N = 32768 is the adjoint workload's size, where the automatic
    form is the symmetric one (tiles of 256, as below it); 70,001 takes tiles of 1024."""
    q, _ = _state(GRAV2D, n, seed=90 + n)
    w = np.random.default_rng(n + 3).normal(size=q.shape)
    ho = oracle.hvp(GRAV2D, q, w, 1e-3)
    ctx = md.md_init(GRAV2D, md.FP64, n, 1e-3)
    md.md_set_launch(ctx, launch)
    assert md.md_get_launch(ctx) == md.LAUNCH_SYMMETRIC
    hs = host(md.md_hvp(ctx, dev(q), dev(w)))
    hs2 = host(md.md_hvp(ctx, dev(q), dev(w)))
    np.testing.assert_array_equal(hs, hs2)                     # fixed order: repeatable bit for bit
    md.md_set_launch(ctx, md.LAUNCH_STAGED)
    hst = host(md.md_hvp(ctx, dev(q), dev(w)))
    tol = hvp_tol(GRAV2D, md.FP64) * max(1.0, np.sqrt(n / 4096))
    check(f"symmetric hvp n={n} vs oracle", rel_inf(hs, ho), tol)
    check(f"symmetric hvp n={n} vs staged", rel_inf(hs, hst), tol)


def test_step_vjp_symmetric_matches_oracle():
    """The reverse sweep with the symmetric product (2D FP64, forced symmetric form,
    a ragged size) against the oracle's."""
    n, nst, eps, dt = 2500, 6, 1e-3, 0.01
    q0, p0 = _state(GRAV2D, n, seed=64)
    rng = np.random.default_rng(10)
    lq0, lp0 = rng.normal(size=q0.shape), rng.normal(size=p0.shape)
    oq, op = oracle.step_vjp(GRAV2D, q0, p0, dt, nst, lq0, lp0, eps)
    ctx = md.md_init(GRAV2D, md.FP64, n, eps)
    md.md_set_launch(ctx, md.LAUNCH_SYMMETRIC)
    lq, lp = dev(lq0), dev(lp0)
    md.md_step_vjp(ctx, dev(q0), dev(p0), dt, nst, lq, lp)
    eq, ep = rel_inf(host(lq), oq), rel_inf(host(lp), op)
    print(f"symmetric vjp rel_err q={eq:.3e} p={ep:.3e}")
    assert eq < 1e-9 and ep < 1e-9


@pytest.mark.parametrize("n", [1, 2, 65, 1001, 5003])
@pytest.mark.parametrize("prec", [md.FP64, md.MIXED_F32STATE])
def test_hmf_hvp_matches_oracle(prec, n):
    """The O(N) mean-field product against the oracle's O(N^2) pair sum; it runs in
    FP64 whatever the context's state precision."""
    q, _ = _state(HMF, n, seed=70 + n)
    w = np.random.default_rng(n + 1).normal(size=q.shape)
    ho = oracle.hvp(HMF, q, w, 0.0)
    ctx = md.md_init(HMF, prec, n, 0.0)
    hg = host(md.md_hvp(ctx, dev(q), dev(w)))
    if n == 1:
        assert np.abs(hg).max() < 1e-15  # w (c^2 + s^2) - (c^2 + s^2) w
        return
    err = rel_inf(hg, ho)
    print(f"hvp model=HMF prec={prec} n={n} rel_err={err:.3e}")
    assert err < 1e-11, err


@pytest.mark.parametrize("model,eps,dt", [(GRAV2D, 1e-3, 0.01), (RING, 0.01, 0.05), (HMF, 0.0, 0.1)])
def test_step_vjp_matches_oracle(model, eps, dt):
    n, nst = 300, 10
    q0, p0 = _state(model, n, seed=61)
    rng = np.random.default_rng(7)
    lq0, lp0 = rng.normal(size=q0.shape), rng.normal(size=p0.shape)
    oq, op = oracle.step_vjp(model, q0, p0, dt, nst, lq0, lp0, eps)
    ctx = md.md_init(model, md.FP64, n, eps)
    lq, lp = dev(lq0), dev(lp0)
    md.md_step_vjp(ctx, dev(q0), dev(p0), dt, nst, lq, lp)
    eq, ep = rel_inf(host(lq), oq), rel_inf(host(lp), op)
    print(f"vjp model={model} rel_err q={eq:.3e} p={ep:.3e}")
    assert eq < 1e-9 and ep < 1e-9


def test_step_vjp_mixed_close_to_oracle():
    """Mixed 2D: the adjoint of the FP32-pair map is within 1e-3 (relative) of the
    FP64 oracle's after 10 steps."""
    n, nst, eps, dt = 300, 10, 1e-3, 0.01
    q0, p0 = _state(GRAV2D, n, seed=62)
    rng = np.random.default_rng(8)
    lq0, lp0 = rng.normal(size=q0.shape), rng.normal(size=p0.shape)
    oq, op = oracle.step_vjp(GRAV2D, q0, p0, dt, nst, lq0, lp0, eps)
    ctx = md.md_init(GRAV2D, md.MIXED, n, eps)
    lq, lp = dev(lq0), dev(lp0)
    md.md_step_vjp(ctx, dev(q0), dev(p0), dt, nst, lq, lp)
    assert rel_inf(host(lq), oq) < 1e-3 and rel_inf(host(lp), op) < 1e-3


@pytest.mark.parametrize("model,prec,eps,dt,n", [(GRAV2D, md.MIXED, 1e-3, 0.01, 500), (GRAV2D, md.FP64, 1e-3, 0.01, 501),
                                                 (HMF, md.FP64, 0.0, 0.1, 500), (HMF, md.FP64, 0.0, 0.1, 20_001)])
def test_step_vjp_composes_over_segments(model, prec, eps, dt, n):
    """Checkpointed segments: 9 steps at once == 5 then 4, bit for bit (odd n: the
    padded stage slots keep the recomputed trajectory identical to md_step's)."""
    q0, p0 = _state(model, n, seed=63)
    ctx = md.md_init(model, prec, n, eps)
    qd, pd = dev(q0), dev(p0)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    q4, p4, f4 = qd.clone(), pd.clone(), f.clone()
    md.md_step(ctx, q4, p4, f4, dt, 4)
    rng = np.random.default_rng(9)
    l0q, l0p = rng.normal(size=q0.shape), rng.normal(size=p0.shape)
    aq, ap = dev(l0q), dev(l0p)
    md.md_step_vjp(ctx, qd, pd, dt, 9, aq, ap)
    bq, bp = dev(l0q), dev(l0p)
    md.md_step_vjp(ctx, q4, p4, dt, 5, bq, bp)
    md.md_step_vjp(ctx, qd, pd, dt, 4, bq, bp)
    np.testing.assert_array_equal(host(aq), host(bq))
    np.testing.assert_array_equal(host(ap), host(bp))


def test_step_vjp_rejects_small_stage_buffer():
    ctx = md.md_init(GRAV2D, md.FP64, 100, 1e-3)
    q = torch.zeros((2, 100), dtype=torch.float64, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(md.MDError):
        md.md_step_vjp(ctx, q, q.clone(), 0.01, 3, q.clone(), q.clone(), small)
    hmf = md.md_init(HMF, md.MIXED_F32STATE, 100, 0.0)
    h = q[:1].contiguous()
    with pytest.raises(md.MDError):  # the FP32-state trajectory has no FP64 snapshots
        md.md_step_vjp(hmf, h, h.clone(), 0.01, 3, h.clone(), h.clone())
    batch = md.md_batch_init(RING, md.FP64, [0, 50, 100], 0.01)
    with pytest.raises(md.MDError):
        md.md_hvp(batch, h, h.clone())


@pytest.mark.parametrize("model,eps,dt", [(GRAV2D, 1e-2, 0.01), (RING, 0.02, 0.02), (HMF, 0.0, 0.1)])
def test_kinetic_energy_gradient_matches_finite_differences(model, eps, dt):
    """d K_T / d(q0, p0) through the autograd Function (checkpoints every 7 steps)
    against central differences of the FP64 forward map along 4 random directions."""
    n, nst = 256, 30
    q0, p0 = _state(model, n, seed=64)
    ctx = md.md_init(model, md.FP64, n, eps)
    K, gq, gp = mdgrad.kinetic_energy_gradient(ctx, dev(q0), dev(p0), dt, nst, checkpoint_every=7)

    def J(q, p):
        qd, pd = dev(q), dev(p)
        f = torch.empty_like(qd)
        md.md_force(ctx, qd, f)
        md.md_step(ctx, qd, pd, f, dt, nst)
        return 0.5 * float((pd * pd).sum())
    assert abs(J(q0, p0) - float(K)) <= 1e-14 * abs(float(K))
    rng = np.random.default_rng(10)
    gq, gp = host(gq), host(gp)
    for _ in range(4):
        vq, vp = rng.normal(size=q0.shape), rng.normal(size=p0.shape)
        h = 1e-6
        fd = (J(q0 + h * vq, p0 + h * vp) - J(q0 - h * vq, p0 - h * vp)) / (2 * h)
        ad = float(np.sum(gq * vq) + np.sum(gp * vp))
        print(f"grad model={model} ad={ad:.12e} fd={fd:.12e}")
        assert abs(ad - fd) < 1e-6 * max(1.0, abs(fd)), (ad, fd)


@pytest.mark.parametrize("model,eps,dt", [(HMF, 0.0, 0.1), (RING, 0.02, 0.02)])
def test_magnetization_gradient_matches_oracle_and_finite_differences(model, eps, dt):
    """d M_T / d(q0, p0), M_T = |(mean cos q_T, mean sin q_T)|, through the autograd
    Function: against the oracle's reverse sweep seeded with the observable's
    derivative at the oracle's final state, and against central differences of the
    GPU FP64 forward map along 4 random directions."""
    n, nst = 256, 30
    q0, p0 = _state(model, n, seed=65)
    ctx = md.md_init(model, md.FP64, n, eps)
    M, gq, gp = mdgrad.magnetization_gradient(ctx, dev(q0), dev(p0), dt, nst, checkpoint_every=7)
    gq, gp = host(gq), host(gp)
    # oracle gradient
    f0 = oracle.force(model, q0, eps)
    qT, _, _ = oracle.step(model, q0, p0, f0, dt, nst, eps)
    mx, my = np.cos(qT).mean(), np.sin(qT).mean()
    Mo = np.hypot(mx, my)
    assert abs(float(M) - Mo) < 1e-12
    lq = (-mx * np.sin(qT) + my * np.cos(qT)) / (n * Mo)
    oq, op = oracle.step_vjp(model, q0, p0, dt, nst, lq, np.zeros_like(p0), eps)
    assert rel_inf(gq, oq) < 1e-9 and rel_inf(gp, op) < 1e-9

    def J(q, p):
        qd, pd = dev(q), dev(p)
        f = torch.empty_like(qd)
        md.md_force(ctx, qd, f)
        md.md_step(ctx, qd, pd, f, dt, nst)
        return float(torch.sqrt(torch.cos(qd).mean() ** 2 + torch.sin(qd).mean() ** 2))
    rng = np.random.default_rng(11)
    for _ in range(4):
        vq, vp = rng.normal(size=q0.shape), rng.normal(size=p0.shape)
        h = 1e-6
        fd = (J(q0 + h * vq, p0 + h * vp) - J(q0 - h * vq, p0 - h * vp)) / (2 * h)
        ad = float(np.sum(gq * vq) + np.sum(gp * vp))
        print(f"magnetization grad model={model} ad={ad:.12e} fd={fd:.12e}")
        assert abs(ad - fd) < 1e-7 * max(1.0, abs(fd)), (ad, fd)


@pytest.mark.parametrize("model,prec,eps,dt,n,launch", [
    (GRAV2D, md.FP64, 1e-3, 0.01, 501, md.LAUNCH_FUSED), (GRAV2D, md.MIXED, 1e-3, 0.01, 501, md.LAUNCH_STAGED),
    (RING, md.FP64, 0.01, 0.05, 2048, md.LAUNCH_FUSED), (RING, md.MIXED_KAHAN, 0.01, 0.05, 300, md.LAUNCH_STAGED),
    (HMF, md.FP64, 0.0, 0.1, 20_001, md.LAUNCH_AUTO)])
def test_recorded_run_matches_md_step_and_vjp(model, prec, eps, dt, n, launch):
    """md_step_record = md_step bit for bit; the sweep over the recording =
    md_step_vjp (which recomputes the same steps) bit for bit."""
    nst = 7
    q0, p0 = _state(model, n, seed=66)
    ctx = md.md_init(model, prec, n, eps)
    md.md_set_launch(ctx, launch)
    qd, pd = dev(q0), dev(p0)
    f0 = torch.empty_like(qd)
    md.md_force(ctx, qd, f0)
    qa, pa, fa = qd.clone(), pd.clone(), f0.clone()
    md.md_step(ctx, qa, pa, fa, dt, nst)
    qb, pb, fb = qd.clone(), pd.clone(), f0.clone()
    stage = md.md_step_record(ctx, qb, pb, fb, dt, nst)
    for x, y in ((qa, qb), (pa, pb), (fa, fb)):
        np.testing.assert_array_equal(host(x), host(y))
    rng = np.random.default_rng(12)
    l0q, l0p = rng.normal(size=q0.shape), rng.normal(size=p0.shape)
    aq, ap = dev(l0q), dev(l0p)
    md.md_step_vjp(ctx, qd, pd, dt, nst, aq, ap)
    bq, bp = dev(l0q), dev(l0p)
    md.md_step_vjp_recorded(ctx, qd, dt, nst, bq, bp, stage)
    np.testing.assert_array_equal(host(aq), host(bq))
    np.testing.assert_array_equal(host(ap), host(bp))


def test_recorded_gradient_equals_checkpointed():
    n, nst, eps, dt = 1000, 40, 1e-2, 0.01
    q0, p0 = _state(GRAV2D, n, seed=67)
    ctx = md.md_init(GRAV2D, md.FP64, n, eps)
    Ka, gqa, gpa = mdgrad.kinetic_energy_gradient(ctx, dev(q0), dev(p0), dt, nst, checkpoint_every=7)
    Kb, gqb, gpb = mdgrad.kinetic_energy_gradient(ctx, dev(q0), dev(p0), dt, nst, checkpoint_every=0)
    assert float(Ka) == float(Kb)
    np.testing.assert_array_equal(host(gqa), host(gqb))
    np.testing.assert_array_equal(host(gpa), host(gpb))


def test_record_rejections():
    hmf = md.md_init(HMF, md.MIXED_F32STATE, 100, 0.0)
    h = torch.zeros((1, 100), dtype=torch.float64, device="cuda")
    with pytest.raises(md.MDError):
        md.md_step_record(hmf, h, h.clone(), h.clone(), 0.1, 2)
    ctx = md.md_init(GRAV2D, md.FP64, 100, 1e-3)
    q = torch.zeros((2, 100), dtype=torch.float64, device="cuda")
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(md.MDError):
        md.md_step_record(ctx, q, q.clone(), q.clone(), 0.01, 2, small)
    with pytest.raises(md.MDError):
        md.md_step_vjp_recorded(ctx, q, 0.01, 2, q.clone(), q.clone(), small)
    assert md.md_record_stage_bytes(ctx, 5) == 15 * 200 * 8


def test_adjoint_config_full_size_reduced_steps():
    """The adjoint workload's system at its full size (2D, N = 32768, eps = 1e-3,
    uniform disk, seed 5, dt = 0.01) over 50 steps with checkpoints every 10: the
    gradient of K_T against FP64 central differences along 2 random unit
    directions, and the recorded gradient equal to the checkpointed one."""
    n, nst, eps, dt = 32768, 50, 1e-3, 0.01
    q0, p0 = inputs.grav2d_disk(n, seed=5)
    ctx = md.md_init(GRAV2D, md.FP64, n, eps)
    K, gq, gp = mdgrad.kinetic_energy_gradient(ctx, dev(q0), dev(p0), dt, nst, checkpoint_every=10)
    Kr, gqr, gpr = mdgrad.kinetic_energy_gradient(ctx, dev(q0), dev(p0), dt, nst, checkpoint_every=0)
    assert float(K) == float(Kr) and torch.equal(gq, gqr) and torch.equal(gp, gpr)

    def J(q, p):
        qd, pd = dev(q), dev(p)
        f = torch.empty_like(qd)
        md.md_force(ctx, qd, f)
        md.md_step(ctx, qd, pd, f, dt, nst)
        return 0.5 * float((pd * pd).sum())
    gq, gp = host(gq), host(gp)
    for k in range(2):
        v = np.random.default_rng([5, k]).normal(size=(4, n))
        v /= np.linalg.norm(v)
        h = 1e-4
        fd = (J(q0 + h * v[:2], p0 + h * v[2:]) - J(q0 - h * v[:2], p0 - h * v[2:])) / (2 * h)
        ad = float(np.sum(gq * v[:2]) + np.sum(gp * v[2:]))
        print(f"adjoint full size dir {k}: ad={ad:.12e} fd={fd:.12e}")
        assert abs(ad - fd) < 1e-6 * max(1.0, abs(fd)), (ad, fd)


def test_adjoint_config_full_run():
    """The adjoint workload as configured: 2D, N = 32768, eps = 1e-3, uniform disk
    (seed 5), dt = 0.01, 1000 steps with checkpoints every 50.  The gradient of K_T
    against FP64 central differences (h = 1e-4, the best step of the benchmark's
    sweep from 1e-4 to 1e-8) along 2 of the benchmark's 16 random unit directions.
    Over 1000 steps the difference quotient carries its own truncation error,
    amplified by the chaotic dynamics: measured 3e-8 to 2e-7 relative over the 16
    directions; the bar is 2e-6."""
    n, nst, eps, dt, every, h = 32768, 1000, 1e-3, 0.01, 50, 1e-4
    q0, p0 = inputs.grav2d_disk(n, seed=5)
    ctx = md.md_init(GRAV2D, md.FP64, n, eps)
    K, gq, gp = mdgrad.kinetic_energy_gradient(ctx, dev(q0), dev(p0), dt, nst, checkpoint_every=every)
    gq, gp = host(gq), host(gp)

    def J(q, p):
        qd, pd = dev(q), dev(p)
        f = torch.empty_like(qd)
        md.md_force(ctx, qd, f)
        md.md_step(ctx, qd, pd, f, dt, nst)
        return 0.5 * float((pd * pd).sum())
    assert J(q0, p0) == float(K)  # the forward map the gradient is of
    for k in range(2):
        v = np.random.default_rng([5, k]).normal(size=(4, n))
        v /= np.linalg.norm(v)
        fd = (J(q0 + h * v[:2], p0 + h * v[2:]) - J(q0 - h * v[:2], p0 - h * v[2:])) / (2 * h)
        ad = float(np.sum(gq * v[:2]) + np.sum(gp * v[2:]))
        rel = abs(ad - fd) / max(1.0, abs(fd))
        print(f"adjoint config run dir {k}: ad={ad:.12e} fd={fd:.12e} rel={rel:.3e}")
        assert rel < 2e-6, (ad, fd)
    ctx.close()
