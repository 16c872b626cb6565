"""The 2D self-gravitating benchmark run against the FP64 oracle at every report
time (Sec. 4 judges a run by its relative energy error |E(t) - E0| / |E0|).

The golden files tests/golden/grav2d_disk_seed3_n{N}.json are written by
tests/golden/make_grav2d_golden.py, which calls only the oracle and the seeded
input generator: K, V, E of the oracle's FP64 Yoshida run (Sec. 3, eq. 4) every
10 steps up to 100, from the benchmark's state (positions uniform in the unit
disk, momenta Gaussian with sigma = 0.5 and zero mean, seed 3; eps = 1e-3,
dt = 0.01), with the positions and momenta of 32 sampled particles at those
times.

Bars, at every report time:
  * the energy: within 1e-6 of |E0| (FP64) or 1e-5 of |E0| (the FP32 forms) of
    the oracle's energy at the same time.  E0 nearly cancels for this state
    (K0 + V0 is 0.6-0.7% of K0 + |V0|), so the same bars are also tighter
    figures against K0 + |V0|;
  * the sampled positions and momenta: the trajectories separate only through
    rounding over t = 1, so FP64 stays within 1e-9 and the FP32 forms within
    1e-5 of the oracle's.

N = 65,536 is past the symmetric form's threshold: the automatic form there is
the one the benchmark times at N = 262,144, in every precision.  The full-size
case needs the golden file of N = 262,144 (about 1.5 h of oracle time on 8
cores) and is skipped without it.
"""
import json
import os

import numpy as np
import pytest

from paper_1212_0262_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
md = pytest.importorskip("paper_1212_0262_amd.md")
from gpu_helpers import dev, host  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
ENERGY_BAR = {md.FP64: 1e-6, md.MIXED: 1e-5, md.MIXED_KAHAN: 1e-5, md.MIXED_PAIRF64: 1e-5}
STATE_BAR = {md.FP64: 1e-9, md.MIXED: 1e-5, md.MIXED_KAHAN: 1e-5, md.MIXED_PAIRF64: 1e-5}


def _golden(n):
    path = os.path.join(GOLDEN, f"grav2d_disk_seed3_n{n}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_grav2d_golden.py --n {n})")
    with open(path) as fh:
        g = json.load(fh)
    assert g["n"] == n and g["seed"] == 3 and g["eps"] == 1e-3 and g["dt"] == 0.01
    return g


def _run(g, prec, launch=md.LAUNCH_AUTO):
    """md_force, then md_step in chunks of the golden's report interval; energies
    and the sampled particles at every report time."""
    n, every = g["n"], g["every"]
    q0, p0 = inputs.grav2d_disk(n, seed=g["seed"], sigma=g["sigma"])
    ctx = md.md_init(md.GRAV2D, prec, n, g["eps"])
    md.md_set_launch(ctx, launch)
    form = md.md_get_launch(ctx)
    q, p = dev(q0), dev(p0)
    f = torch.empty_like(q)
    md.md_force(ctx, q, f)
    rows = g["sample_rows"]
    E, qs, ps = [host(md.md_energy(ctx, q, p))], [host(q)[:, rows]], [host(p)[:, rows]]
    for s0, s1 in zip(g["steps"][:-1], g["steps"][1:]):
        assert s1 - s0 == every
        md.md_step(ctx, q, p, f, g["dt"], every)
        E.append(host(md.md_energy(ctx, q, p)))
        qs.append(host(q)[:, rows])
        ps.append(host(p)[:, rows])
    ctx.close()
    return np.array(E), np.array(qs), np.array(ps), form


def _check(g, prec, E, qs, ps, label):
    Eo = np.array([g["K"], g["V"], g["E"]]).T
    E0 = abs(Eo[0, 2])
    KV0 = abs(Eo[0, 0]) + abs(Eo[0, 1])
    dE = np.abs(E[:, 2] - Eo[:, 2])
    dq = np.abs(qs - np.array(g["q_sample"])).max()
    dp = np.abs(ps - np.array(g["p_sample"])).max()
    drift_or = np.abs(Eo[:, 2] - Eo[0, 2]).max() / E0
    print(f"{label} prec={md.PREC_NAMES[prec]}: max |E - E_oracle| / |E0| = {dE.max() / E0:.3e} "
          f"(/ (K0+|V0|) = {dE.max() / KV0:.3e}); oracle's own max |E(t) - E0| / |E0| = {drift_or:.3e}; "
          f"sampled max|dq| = {dq:.2e}, max|dp| = {dp:.2e}")
    assert dE.max() <= ENERGY_BAR[prec] * E0, (dE / E0).tolist()
    assert dq <= STATE_BAR[prec] and dp <= STATE_BAR[prec], (dq, dp)
    return dE.max() / E0


@pytest.mark.parametrize("prec", [md.MIXED, md.MIXED_KAHAN, md.MIXED_PAIRF64, md.FP64])
def test_grav2d_n65536_every_report_time(prec):
    g = _golden(65536)
    E, qs, ps, form = _run(g, prec)
    assert form == md.LAUNCH_SYMMETRIC
    # the energy at t = 0 is the same FP64 sum over pairs, in another order
    Eo0 = np.array([g["K"][0], g["V"][0], g["E"][0]])
    assert np.abs(E[0] - Eo0).max() <= 1e-12 * (abs(Eo0[0]) + abs(Eo0[1]))
    _check(g, prec, E, qs, ps, "N=65536 symmetric")


def test_grav2d_n65536_staged_form():
    """The staged form (every ordered pair evaluated) on the same run."""
    g = _golden(65536)
    E, qs, ps, form = _run(g, md.MIXED, md.LAUNCH_STAGED)
    assert form == md.LAUNCH_STAGED
    _check(g, md.MIXED, E, qs, ps, "N=65536 staged")


@pytest.mark.parametrize("prec", [md.MIXED, md.FP64])
def test_grav2d_full_size_every_report_time(prec):
    """N = 262,144, the benchmark's configuration and launch form."""
    g = _golden(262144)
    E, qs, ps, form = _run(g, prec)
    assert form == md.LAUNCH_SYMMETRIC
    Eo0 = np.array([g["K"][0], g["V"][0], g["E"][0]])
    assert np.abs(E[0] - Eo0).max() <= 1e-12 * (abs(Eo0[0]) + abs(Eo0[1]))
    k = len(g["steps"])
    _check(g, prec, E[:k], qs[:k], ps[:k], "N=262144 symmetric")
