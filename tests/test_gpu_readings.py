"""The alternative readings (cgks_scheme_desc.reading_flags) on the HIP path
against the oracle under the same reading: gamma_1 taking the gamma_Lo share
of Eq. 3.12, smoothness indicators of the unscaled members (Eq. 3.13, 3.19),
zero strengths before the first step (Eq. 3.2).  FP64, relative L1 <= 1e-10,
and the cascade's branch counts equal to the oracle's."""
import numpy as np
import pytest

import oracle
from paper_2508_13705_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
BRANCHES = ("ao", "linear5", "linear7", "linear9")


def _say(msg):
    print(f"\n[readings] {msg}", flush=True)


def _with_flags(pb, flags):
    return dict(pb, scheme=dict(pb["scheme"], reading_flags=flags))


def _compare(pb, nsteps, dim):
    from paper_2508_13705_amd import cgks
    s = cgks.Solver(pb)
    s.step(nsteps)
    got, h = s.read(), s.health()
    ref = oracle.run(pb, nsteps=nsteps, t_end=0.0)
    assert got["status"] == ref["status"] == 0
    assert got["steps"] == nsteps and abs(got["t"] - ref["t"]) <= 1e-13 * ref["t"]
    ax = (1, 2) if dim == 2 else (1,)
    norm = np.abs(ref["avg"]).sum(axis=ax)
    e = float((np.abs(got["avg"] - ref["avg"]).sum(axis=ax) / norm).max())
    _say(f"  rel-L1 {e:.2e}; gpu {[h[k] for k in BRANCHES]} oracle {[ref['stats'][k] for k in BRANCHES]}")
    assert e <= TOL64
    for k in BRANCHES:
        assert h[k] == ref["stats"][k], k
    assert h["fallbacks"] == ref["stats"]["fallback"]
    return got, ref


@pytest.mark.parametrize("flags", [1, 2, 4, 7])
@pytest.mark.parametrize("order", [5, 9])
def test_quadrant_2d_under_each_reading(order, flags):
    pb = _with_flags(W.quadrant_2d(W.random_quadrants(3), 24, order, nsteps=6), flags)
    _say(f"quadrant 24^2 order {order} reading flags {flags}")
    _, ref = _compare(pb, 6, 2)
    if flags & 1:
        # the reading changes the result (it has AO cells to act on)
        base = oracle.run(_with_flags(pb, flags & ~1), nsteps=6, t_end=0.0)
        assert np.abs(base["avg"] - ref["avg"]).max() > 0


@pytest.mark.parametrize("flags", [3, 4])
def test_shock_tube_1d_under_each_reading(flags):
    pb = _with_flags(W.shock_tube("lax", 300, 7), flags)
    _say(f"lax 300 order 7 reading flags {flags}")
    _compare(pb, 40, 1)


def test_first_step_takes_the_full_order_with_zero_strengths():
    from paper_2508_13705_amd import cgks
    pb = _with_flags(W.quadrant_2d(W.random_quadrants(3), 24, 9, nsteps=1), 4)
    s = cgks.Solver(pb)
    s.step(1)
    h = s.health()
    assert h["ao"] == h["linear5"] == h["linear7"] == 0
    assert h["linear9"] == h["recon_total"]


def test_unknown_reading_flag_is_rejected():
    from paper_2508_13705_amd import cgks
    pb = _with_flags(W.shock_tube("sod", 50, 5), 8)
    with pytest.raises(cgks.CgksError):
        cgks.Solver(pb)
