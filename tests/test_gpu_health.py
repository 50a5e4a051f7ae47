"""Device diagnostics through the C ABI: the reconstruction counts by cascade
branch (Algorithm 1) against the oracle's own counts, the near-tie counter,
the cell-averaged gradient readback (Sec. 3.3) and the device conservation
totals (fixed-order compensated sums)."""
import math

import numpy as np
import pytest

import oracle
from paper_2508_13705_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[health] {msg}", flush=True)


BRANCHES = ("ao", "linear5", "linear7", "linear9")


def _counts(pb, precision, nsteps):
    from paper_2508_13705_amd import cgks
    s = cgks.Solver(pb, precision=precision)
    s.step(nsteps)
    h = s.health()
    ref = oracle.run(pb, nsteps=nsteps, t_end=0.0)
    return h, ref


CASES_2D = [(o, seed) for o in (5, 7, 9) for seed in (3, 8)]


@pytest.mark.parametrize("order,seed", CASES_2D)
def test_branch_counts_equal_oracle_2d(order, seed):
    """Four-quadrant problems of every order: the GPU takes every cascade
    decision the oracle takes, so the numbers of reconstructions by AO(5,3)
    and by each linear stencil are equal exactly (FP64; no near ties)."""
    pb = W.quadrant_2d(W.random_quadrants(seed), 24, order, nsteps=6)
    _say(f"quadrant seed {seed} order {order}")
    h, ref = _counts(pb, "fp64", 6)
    _say(f"  gpu {[h[k] for k in BRANCHES]} ties {h['near_ties']}; oracle {[ref['stats'][k] for k in BRANCHES]}")
    assert h["status"] == 0 and ref["status"] == 0
    assert h["near_ties"] == 0
    assert h["recon_total"] == sum(ref["stats"][k] for k in BRANCHES)
    for k in BRANCHES:
        assert h[k] == ref["stats"][k], k
    assert h["ao"] > 0
    assert h["dff_lt1"] == h["recon_total"] - h[f"linear{order}"]
    assert h["fallbacks"] == ref["stats"]["fallback"]


@pytest.mark.parametrize("order", [5, 7, 9])
@pytest.mark.parametrize("name", ["sod", "lax"])
def test_branch_counts_equal_oracle_1d(name, order):
    pb = W.shock_tube(name, 300, order)   # two 254-cell segments and a ragged third
    h, ref = _counts(pb, "fp64", 40)
    _say(f"{name} order {order}: gpu {[h[k] for k in BRANCHES]}, oracle {[ref['stats'][k] for k in BRANCHES]}")
    assert h["near_ties"] == 0
    assert h["recon_total"] == 40 * 2 * 302
    for k in BRANCHES:
        assert h[k] == ref["stats"][k], k
    assert h["fallbacks"] == ref["stats"]["fallback"]


def test_branch_counts_fp32_flux_within_ties():
    """FP32-flux: strengths carry FP32 rounding, so a decision can differ from
    the FP64 oracle's only where the stencil sum lies near the threshold;
    the counts are reported and differ by no more than the flagged ties."""
    pb = W.quadrant_2d(W.random_quadrants(3), 24, 9, nsteps=6)
    h, ref = _counts(pb, "fp32_flux", 6)
    diff = sum(abs(h[k] - ref["stats"][k]) for k in BRANCHES)
    _say(f"fp32-flux branch-count differences {diff}, near ties {h['near_ties']}")
    assert h["recon_total"] == sum(ref["stats"][k] for k in BRANCHES)
    assert diff <= 0.01 * h["recon_total"]


def test_smooth_data_takes_the_full_order():
    """Smooth advection (no strengths above threshold): every reconstruction
    takes the scheme's own linear stencil and no tile issues a tally."""
    from paper_2508_13705_amd import cgks
    pb = W.fourier_2d(5, 40, 9, nsteps=3)
    s = cgks.Solver(pb)
    s.step(3)
    h = s.health()
    assert h["linear9"] == h["recon_total"] == 3 * 2 * 2 * 40 * 40 * 5
    assert h["ao"] == h["linear5"] == h["linear7"] == h["dff_lt1"] == h["near_ties"] == 0


@pytest.mark.parametrize("dim", [1, 2])
def test_gradient_readback(dim):
    """Cell-averaged gradients: the Gauss-weighted means of the line slopes
    (2-D), the stored slope (1-D)."""
    from paper_2508_13705_amd import cgks
    if dim == 2:
        pb = W.quadrant_2d(W.random_quadrants(4), 20, 7, nsteps=3)
    else:
        pb = W.shock_tube("sod", 80, 9)
    s = cgks.Solver(pb)
    s.step(3)
    r = s.read()
    if dim == 1:
        assert np.array_equal(r["gx"], r["sx"])
        return
    _, wq = W.gauss_legendre(3)
    for key, sl in (("gx", "sx"), ("gy", "sy")):
        want = np.einsum("l,vlji->vji", wq, r[sl])
        assert np.abs(r[key] - want).max() <= 1e-14 * max(1.0, np.abs(want).max())
    assert np.abs(r["gx"]).max() > 0


def _fsum_rel(got, avg, axes):
    nv = avg.shape[0]
    for v in range(nv):
        exact = math.fsum(avg[v].ravel().tolist())
        scale = np.abs(avg[v]).sum()
        assert abs(got[v] - exact) <= 1e-15 * scale, (v, got[v], exact)


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_conservation_sums_device(precision):
    """Device totals equal the exactly rounded host sums to 1e-15 of the sum
    of magnitudes, are bitwise the same on every call, and on a periodic
    grid stay constant over the steps (the update telescopes; FP64
    accumulation in both precisions)."""
    import torch
    from paper_2508_13705_amd import cgks
    pb = W.turbulence_2d(seed=4, n=300, order=9, nsteps=4)   # 90000 cells: 6 blocks, ragged last
    s = cgks.Solver(pb, precision=precision)
    t0 = s.conservation_sums().cpu().numpy()
    _fsum_rel(t0, s.read()["avg"], (1, 2))
    s.step(4)
    a = s.conservation_sums().cpu().numpy()
    b = s.conservation_sums().cpu().numpy()
    assert np.array_equal(a, b)
    r = s.read()
    _fsum_rel(a, r["avg"], (1, 2))
    scale = np.abs(r["avg"]).sum(axis=(1, 2))
    drift = np.abs(a - t0) / scale
    _say(f"{precision}: totals drift over 4 steps {drift.max():.2e} of the sum of magnitudes")
    assert drift.max() <= 1e-15


def test_conservation_sums_1d():
    import torch
    from paper_2508_13705_amd import cgks
    pb = W.fourier_1d(n=1000)
    s = cgks.Solver(pb)
    s.step(10)
    got = s.conservation_sums().cpu().numpy()
    _fsum_rel(got, s.read()["avg"], (1,))
