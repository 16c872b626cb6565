"""md_force_noalloc (the force without a workspace, for callers that cannot
allocate) against md_force through the C ABI.

Both run the same kernels in the staged form with the same tiles wherever the
built-in j split's partials fit the 64 MiB static array, so the forces must be
bit-identical there; at N = 262,144 (2D) the built-in 16 j ranges need 64 MiB of
partials alone and the entry point halves them to 8, so the reference context
takes 8 j ranges too.  Each case makes two calls in a row, the second with a
smaller input, since every call shares the one array and finds the previous
call's contents in it.
"""
import numpy as np
import pytest

import oracle
from paper_1212_0262_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
md = pytest.importorskip("paper_1212_0262_amd.md")
from gpu_helpers import dev, host, rel_inf  # noqa: E402
from tolerances import check, force_tol  # noqa: E402

HMF, RING, GRAV2D = md.HMF, md.RING, md.GRAV2D


def _state(model, n, seed):
    if model == GRAV2D:
        return inputs.grav2d_disk(n, seed=seed)[0]
    if model == RING:
        return inputs.ring_waterbag(n, seed=seed)[0]
    return inputs.hmf_waterbag(n, seed=seed)[0]


def _reference(model, prec, q, eps, jsplit=None):
    """md_force on a context in the staged form (built-in tiles unless jsplit)."""
    n = q.shape[-1]
    ctx = md.md_init(model, prec, n, eps)
    if model != HMF:
        md.md_set_launch(ctx, md.LAUNCH_STAGED)
        if jsplit:
            md.md_set_tiles(ctx, 0, 0, jsplit, 0)
    qd = dev(q)
    f = torch.empty_like(qd)
    md.md_force(ctx, qd, f)
    out = host(f)
    ctx.close()
    return out


def _noalloc(model, prec, q, eps):
    qd = dev(q)
    f = torch.full_like(qd, float("nan"))
    md.md_force_noalloc(model, prec, qd, eps, f)
    torch.cuda.synchronize()
    return host(f)


@pytest.mark.parametrize("model,prec,eps,n1,n2,js1", [
    (GRAV2D, md.MIXED, 1e-3, 50_001, 3001, None),
    (GRAV2D, md.FP64, 1e-3, 20_000, 777, None),
    (RING, md.MIXED_KAHAN, 0.01, 30_001, 2048, None),
    (RING, md.FP64, 0.01, 20_000, 1000, None),
    (HMF, md.FP64, 0.0, 1_000_000, 10_001, None),
    (GRAV2D, md.MIXED, 1e-3, 262_144, 65_536, 8),
])
def test_noalloc_matches_md_force_two_calls(model, prec, eps, n1, n2, js1):
    for k, (n, js) in enumerate(((n1, js1), (n2, None))):
        q = _state(model, n, seed=40 + k)
        print(f"noalloc model={model} prec={prec} n={n} call {k + 1}", flush=True)
        got = _noalloc(model, prec, q, eps)
        ref = _reference(model, prec, q, eps, js)
        np.testing.assert_array_equal(got, ref)
        if n <= 10_001:  # the oracle in seconds
            tol = 1e-13 if model == HMF else force_tol(model, prec, n)
            check(f"noalloc model={model} prec={prec} n={n} against the oracle", rel_inf(got, oracle.force(model, q, eps)),
                  tol)


def test_noalloc_refuses_what_does_not_fit():
    n = 1 << 22  # 2D mixed: 2 x 4 MiB x 4 B operands + 2 x 4 MiB x 8 B partials > 64 MiB
    q = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    f = torch.zeros_like(q)
    with pytest.raises(md.MDError) as ei:
        md.md_force_noalloc(GRAV2D, md.MIXED, q, 1e-3, f)
    assert ei.value.status == md.ENOMEM
    assert "static workspace" in str(ei.value)
    with pytest.raises(md.MDError) as ei:
        md.md_force_noalloc(GRAV2D, md.MIXED, q[:, :1000].contiguous(), 0.0, f[:, :1000].contiguous())
    assert ei.value.status == md.EINVAL
    torch.cuda.synchronize()
    assert torch.count_nonzero(f).item() == 0  # refused before anything ran
