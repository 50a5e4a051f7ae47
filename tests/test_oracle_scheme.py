"""Whole-scheme pins of the oracle: the paper's accuracy tables, exact
Riemann solutions, conservation, free-stream preservation, 2-D/1-D
consistency, x<->y symmetry and the first-order limit of the DFF."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from exact_riemann import cell_averages
from paper_2508_13705_amd import workloads as W

TABLES = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _errors_1d(order, n):
    pb = W.advection_1d(order, n)
    r = oracle.run(pb)
    assert r["status"] == 0 and r["stats"]["ao"] == 0
    ex, _, _ = W._fourier_rho_1d([(0.2, 1.0, -math.pi * r["t"])], 0.0, 2.0, n)
    e = np.abs(r["avg"][0] - ex)
    return np.array([e.mean(), math.sqrt((e * e).mean()), e.max()])


def _errors_2d(order, n):
    pb = W.advection_2d(order, n)
    r = oracle.run(pb)
    assert r["status"] == 0 and r["stats"]["ao"] == 0
    # (U, V) = (1, 1): the wave sin(pi (x + y)) moves by 2t in phase
    ex = W.smooth_2d([(0.2, 1.0, 1.0, -2.0 * math.pi * r["t"])], n, order)["state"]["avg"][0]
    e = np.abs(r["avg"][0] - ex)
    return np.array([e.mean(), math.sqrt((e * e).mean()), e.max()])


# (dim, order, meshes, relative tolerance on the printed errors)
TABLE_CASES = [(1, 5, [5, 10, 20, 40], 0.025), (1, 7, [5, 10, 20], 0.005), (1, 9, [5, 10], 0.06),
               (2, 5, [5, 10], 0.002), (2, 7, [5], 0.01), (2, 9, [5], 0.03)]


@pytest.mark.parametrize("dim,order,meshes,tol", TABLE_CASES)
def test_accuracy_tables(dim, order, meshes, tol):
    rows = TABLES[f"{dim}d"][str(order)]["rows"]
    prev = None
    for n in meshes:
        got = (_errors_1d if dim == 1 else _errors_2d)(order, n)
        want = np.array(rows[str(n)])
        assert np.all(np.abs(got - want) <= tol * want), (n, got, want)
        if prev is not None:
            o_got = np.log2(prev[0] / got[0])
            o_want = math.log2(rows[str(n // 2)][0] / rows[str(n)][0])
            assert abs(o_got - o_want) < 0.1
        prev = got


@pytest.mark.slow
@pytest.mark.parametrize("dim,order,n,tol", [(1, 9, 20, 0.06), (2, 7, 10, 0.002)])
def test_accuracy_tables_finer(dim, order, n, tol):
    got = (_errors_1d if dim == 1 else _errors_2d)(order, n)
    want = np.array(TABLES[f"{dim}d"][str(order)]["rows"][str(n)])
    assert np.all(np.abs(got - want) <= tol * want)


def test_dff_drives_first_order():
    """A vanishing threshold makes every DFF ~ 0 and the scheme first order."""
    errs = []
    for n in (20, 40):
        pb = W.advection_1d(5, n)
        pb["scheme"]["sigma_thres"] = 1e-200
        r = oracle.run(pb)
        ex, _, _ = W._fourier_rho_1d([(0.2, 1.0, -math.pi * r["t"])], 0.0, 2.0, n)
        errs.append(np.abs(r["avg"][0] - ex).mean())
    order = math.log2(errs[0] / errs[1])
    assert 0.7 < order < 1.3


@pytest.mark.parametrize("bc", ["periodic", "transmissive", "reflective"])
def test_free_stream_2d(bc):
    n, order = 12, 9
    st = [(0.8, 0.3, -0.5, 1.2)] * 4
    if bc == "reflective":
        st = [(0.8, 0.0, 0.0, 1.2)] * 4
    pb = W.quadrant_2d(st, n, order, nsteps=4, bc=bc)
    r = oracle.run(pb)
    assert r["status"] == 0
    assert np.abs(r["avg"] - pb["state"]["avg"]).max() <= 1e-14 * np.abs(pb["state"]["avg"]).max()
    assert np.abs(r["sx"]).max() < 1e-12 and np.abs(r["sy"]).max() < 1e-12
    assert np.abs(r["sigx"]).max() == 0.0


def test_conservation_periodic_2d():
    """Discontinuous data on a periodic square: sums of the cell averages are
    conserved to round-off (flux differences telescope), and the line slopes
    sum to zero along every periodic line (Gauss's theorem)."""
    pb = W.quadrant_2d(W.random_quadrants(7), 16, 7, nsteps=6, bc="periodic")
    r = oracle.run(pb)
    assert r["status"] == 0
    s0 = pb["state"]["avg"].sum(axis=(1, 2))
    s1 = r["avg"].sum(axis=(1, 2))
    assert np.all(np.abs(s1 - s0) <= 1e-13 * np.abs(pb["state"]["avg"]).sum(axis=(1, 2)))
    assert np.abs(r["sx"].sum(axis=3)).max() < 1e-11
    assert np.abs(r["sy"].sum(axis=2)).max() < 1e-11
    assert r["stats"]["ao"] > 0


def _sod_2d(n, order, axis):
    left, right = (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1)
    if axis == 0:
        st = [left, right, right, left]
    else:
        st = [left, left, right, right]
    pb = W.quadrant_2d(st, n, order, nsteps=8)
    pb["grid"]["bc"] = ["transmissive", "transmissive", "periodic", "periodic"] if axis == 0 else \
        ["periodic", "periodic", "transmissive", "transmissive"]
    return pb


@pytest.mark.parametrize("order", [5, 9])
def test_2d_y_independent_equals_1d(order):
    n = 16
    p1 = W.shock_tube("sod", n, order)
    p1["run"]["nsteps"] = 8
    p1["run"]["t_end"] = 0.0
    r1 = oracle.run(p1)
    r2 = oracle.run(_sod_2d(n, order, 0))
    assert np.abs(r2["avg"][0] - r1["avg"][0][None, :]).max() < 1e-13
    assert np.abs(r2["avg"][3] - r1["avg"][2][None, :]).max() < 1e-12
    assert np.abs(r2["avg"][2]).max() < 1e-14
    r3 = oracle.run(_sod_2d(n, order, 1))
    assert np.abs(r3["avg"][0] - r1["avg"][0][:, None]).max() < 1e-13


def test_transposition_symmetry():
    pb = W.quadrant_2d(W.random_quadrants(5), 12, 7, nsteps=5)
    r = oracle.run(pb)
    pt = W.quadrant_2d(W.random_quadrants(5), 12, 7, nsteps=5)
    perm = [0, 2, 1, 3]
    st = pb["state"]
    pt["state"] = {"avg": st["avg"][perm].transpose(0, 2, 1).copy(),
                   "sx": st["sy"][perm].transpose(0, 1, 3, 2).copy(),
                   "sy": st["sx"][perm].transpose(0, 1, 3, 2).copy()}
    rt = oracle.run(pt)
    assert np.abs(rt["avg"] - r["avg"][perm].transpose(0, 2, 1)).max() < 1e-12
    assert np.abs(rt["sx"] - r["sy"][perm].transpose(0, 1, 3, 2)).max() < 1e-9


@pytest.mark.parametrize("name", ["sod", "lax"])
@pytest.mark.parametrize("order", [5, 7, 9])
def test_shock_tube_converges_to_exact(name, order):
    errs = []
    for n in (100, 200):
        pb = W.shock_tube(name, n, order)
        r = oracle.run(pb)
        assert r["status"] == 0
        assert abs(r["t"] - pb["run"]["t_end"]) < 1e-14
        rs = pb["riemann"]
        ex = cell_averages(rs["left"], rs["right"], rs["gamma"], rs["xs"], r["t"], 0.0, 1.0, n)
        errs.append(np.abs(r["avg"][0] - ex[0]).mean())
    assert errs[1] < errs[0]
    assert errs[0] < 0.02


@pytest.mark.parametrize("order", [5, 9])
def test_double_rarefaction_robustness(order):
    """Near-vacuum double rarefaction (Sec. 4.5): positive density and pressure
    throughout, L1 density error a few percent of the mean."""
    pb = W.shock_tube("double_rarefaction", 100, order)
    r = oracle.run(pb)
    assert r["status"] == 0
    g = pb["riemann"]["gamma"]
    p = (g - 1) * (r["avg"][2] - 0.5 * r["avg"][1] ** 2 / r["avg"][0])
    assert r["avg"][0].min() > 0 and p.min() > 0
    rs = pb["riemann"]
    ex = cell_averages(rs["left"], rs["right"], g, rs["xs"], r["t"], 0.0, 1.0, 100, sub=16)
    assert np.abs(r["avg"][0] - ex[0]).mean() < 0.03


def test_le_blanc_is_reported_not_silently_wrong():
    """Le Blanc (p ratio 1e9, Sec. 4.5).  With the readings adopted here the
    strengths of the previous step miss the front as it enters fresh cells and
    a near-vacuum cell average turns nonphysical within a few steps; the run
    must report it (status 4) and stop after that step."""
    pb = W.shock_tube("le_blanc", 200, 9)
    r = oracle.run(pb)
    assert r["status"] in (0, 4)
    if r["status"] == 4:
        k = r["stats"]["steps"]
        assert k < 10
        assert r["t"] < pb["run"]["t_end"]
        g = pb["riemann"]["gamma"]

        def physical(a):
            p = (g - 1) * (a[2] - 0.5 * a[1] ** 2 / a[0])
            return bool(np.all(np.isfinite(a)) and np.all(a[0] > 0) and np.all(p > 0))

        # the step that reports it is the first whose stage or final state
        # is nonphysical (A34: that step completes, then the run stops)
        prev = oracle.run(pb, nsteps=k - 1)
        assert prev["status"] == 0 and physical(prev["avg"])
        assert not physical(r["avg"])


@pytest.mark.parametrize("name,mach", [("shu_osher", 3.0), ("titarev_toro", None)])
def test_shock_density_wave_data(name, mach):
    """Sec. 4.3 initial data: the left state is the post-shock state of a
    shock running into the gas at rest (rho = 1, p = 1): mass, momentum and
    energy fluxes across it agree in the shock's frame (Rankine-Hugoniot, to
    the digits the paper prints; Shu-Osher's is Mach 3); the right side's cell
    averages integrate to the exact integral of 1 + amp sin(k (x - 5))."""
    d = W.SHOCK_WAVES[name]
    g = 1.4
    rl, ul, pl = d["left"]
    s = rl * ul / (rl - 1.0)                   # mass flux continuity (the right gas is at rest)
    el = pl / (g - 1) + 0.5 * rl * ul * ul
    er = 1.0 / (g - 1)
    assert abs((rl * ul * (ul - s) + pl) - (1.0 + 0.0)) <= 2e-5 * pl
    assert abs(((el + pl) * ul - s * el) - (-s * er)) <= 2e-5 * el * s
    if mach is not None:
        assert abs(s / math.sqrt(g) - mach) <= 1e-5
    pb = W.shock_wave_1d(name, order=5)
    n = pb["grid"]["nx"]
    h = 10.0 / n
    kf = int(round(d["xs"] / h))
    k, amp = d["k"], d["amp"]
    exact = (10.0 - d["xs"]) + amp * (math.cos(k * (d["xs"] - 5.0)) - math.cos(k * 5.0)) / k
    assert abs(pb["state"]["avg"][0, kf:].sum() * h - exact) <= 1e-12 * exact


@pytest.mark.parametrize("order", [5, 9])
def test_blast_wave_first_step(order):
    """Interacting blast waves (Sec. 4.4: p = 1000 | 0.01 | 100, rho = 1, u = 0,
    400 cells, reflective walls, CFL 0.5).  Fixed independently of the
    scheme: the first time step is CFL h / sqrt(gamma p_max / rho), and no
    mass crosses a reflective wall.  With the readings adopted here the first
    step then leaves one cell nonphysical, the second on the low-pressure
    side of the x = 0.1 jump (the strong-pressure-ratio failure of the 1-D
    Riemann batch); the run reports it (status 4) and stops after that
    step."""
    pb = W.blast_wave(order=order)
    r = oracle.run(pb)
    h = 1.0 / 400
    assert r["stats"]["steps"] == 1
    assert abs(r["t"] - 0.5 * h / math.sqrt(1.4 * 1000.0)) <= 1e-15
    assert abs(r["avg"][0].sum() * h - 1.0) <= 1e-14
    a = r["avg"]
    p = 0.4 * (a[2] - 0.5 * a[1] ** 2 / a[0])
    assert r["status"] == 4
    assert list(np.where((a[0] <= 0) | (p <= 0))[0]) == [41]


@pytest.mark.slow
@pytest.mark.parametrize("order,n,steps", [(9, 20, 150), (7, 20, 150)])
def test_cfl_half_is_stable_2d(order, n, steps):
    """The paper runs every order at CFL 0.5 (abstract, Sec. 4).  Smooth 2-D
    data stays bounded for many steps at CFL 0.5 with the Step 3 tangential
    fit of degree min(2m+1, 8) (A22); the degree-11 interpolant for m = 4
    blows up within a dozen steps here."""
    pb = W.fourier_2d(5, n, order, nsteps=steps, cfl=0.5)
    r = oracle.run(pb)
    assert r["status"] == 0 and r["stats"]["steps"] == steps
    assert np.abs(r["sx"]).max() < 2.0 * np.abs(pb["state"]["sx"]).max()
    assert abs(r["avg"][0].mean() - pb["state"]["avg"][0].mean()) < 1e-13


def test_zero_initial_strengths_reading():
    """Strengths of the step before the first set to zero (an alternative
    reading of Eq. 3.2 at t = 0): every DFF of the first step is 1 (Eq. 3.3,
    A = 0), so both stages of that step take the full-order linear stencil
    everywhere (Algorithm 1), where the default reading (strengths of the
    initial piecewise-constant data) sends the cells beside the jump to
    AO(5,3).  From the second step on the strengths come from the first
    step's fluxes and the run equals one started from explicit zero strengths."""
    n = 100
    pb = W.shock_tube("sod", n, 9)
    r0 = oracle.run(pb, nsteps=1, t_end=0.0)
    assert r0["stats"]["ao"] > 0
    pb4 = dict(pb, scheme=dict(pb["scheme"], reading_flags=4))
    r = oracle.run(pb4, nsteps=1, t_end=0.0)
    assert r["status"] == 0
    assert r["stats"]["ao"] == r["stats"]["linear5"] == r["stats"]["linear7"] == 0
    assert r["stats"]["linear9"] == 2 * (n + 2)
    a = oracle.run(pb4, nsteps=3, t_end=0.0)
    b = oracle.run(pb, nsteps=3, t_end=0.0, sigma=(np.zeros(n + 1), np.zeros(1)))
    assert np.array_equal(a["avg"], b["avg"]) and a["t"] == b["t"]
