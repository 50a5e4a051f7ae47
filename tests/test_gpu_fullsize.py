"""Parity at the full workload sizes, in the launch configuration bench.py
times: the GPU steps the whole grid; the oracle recomputes sampled cells.

One two-stage step moves information about ten cells (two stages of
reconstruction stencils, DFF strengths and Step 1/3 line data), so the
oracle, run with the GPU's time step on a window of the full initial state,
reproduces every cell at least MARGIN cells inside the window's artificial
edges.  Windows of periodic problems wrap around; windows of transmissive
problems keep the true boundary where they touch the domain edge.  The 1-D
batch compares whole sampled jobs."""
import functools

import numpy as np
import pytest

import oracle
from paper_2508_13705_amd import workloads as W

pytestmark = pytest.mark.gpu

WIN = 40       # window side (cells)
MARGIN = 13    # cells of each artificial edge that are not compared


def _say(msg):
    print(f"\n[fullsize] {msg}", flush=True)


def _window(pb, i0, j0, periodic):
    """Sub-problem on cells [i0, i0+WIN) x [j0, j0+WIN) (wrapped when periodic,
    clipped to the domain otherwise) and the mask of cells to compare."""
    g = pb["grid"]
    nx, ny = g["nx"], g["ny"]
    dx, dy = (g["x1"] - g["x0"]) / nx, (g["y1"] - g["y0"]) / ny
    if periodic:
        ii = (np.arange(WIN) + i0) % nx
        jj = (np.arange(WIN) + j0) % ny
        bc = ["periodic"] * 4
        keep_x = (np.arange(WIN) >= MARGIN) & (np.arange(WIN) < WIN - MARGIN)
        keep_y = keep_x
    else:
        i0 = min(max(i0, 0), nx - WIN)
        j0 = min(max(j0, 0), ny - WIN)
        ii, jj = np.arange(i0, i0 + WIN), np.arange(j0, j0 + WIN)
        art = [i0 > 0, i0 + WIN < nx, j0 > 0, j0 + WIN < ny]          # artificial sides
        bc = [g["bc"][k] if not art[k] else "transmissive" for k in range(4)]
        a = np.arange(WIN)
        keep_x = (a >= (MARGIN if art[0] else 0)) & (a < WIN - (MARGIN if art[1] else 0))
        keep_y = (a >= (MARGIN if art[2] else 0)) & (a < WIN - (MARGIN if art[3] else 0))
    st = pb["state"]
    sub = {"avg": st["avg"][:, jj][:, :, ii], "sx": st["sx"][:, :, jj][:, :, :, ii],
           "sy": st["sy"][:, :, jj][:, :, :, ii]}
    x0 = g["x0"] + ii[0] * dx
    y0 = g["y0"] + jj[0] * dy
    wpb = {"name": pb["name"] + f"_win{i0}_{j0}",
           "grid": {"dim": 2, "nx": WIN, "ny": WIN, "x0": x0, "x1": x0 + WIN * dx, "y0": y0, "y1": y0 + WIN * dy,
                    "bc": bc},
           "scheme": pb["scheme"], "state": sub, "run": {"nsteps": 1, "dt": 0.0, "t_end": 0.0}}
    return wpb, ii, jj, np.outer(keep_y, keep_x)


def _check_2d(pb, precision, samples, periodic, tol):
    from paper_2508_13705_amd import cgks
    _say(f"{pb['name']} {pb['grid']['nx']}x{pb['grid']['ny']} order {pb['scheme']['order']} {precision}: one step")
    s = cgks.Solver(pb, precision=precision)
    s.step(1)
    got = s.read()
    assert got["status"] == 0 and got["steps"] == 1
    dt = got["t"]
    worst = 0.0
    for (i0, j0) in samples:
        wpb, ii, jj, keep = _window(pb, i0, j0, periodic)
        ref = oracle.run(wpb, nsteps=1, dt=dt)
        assert ref["status"] == 0
        g_avg = got["avg"][:, jj][:, :, ii]
        g_sx = got["sx"][:, :, jj][:, :, :, ii]
        g_sy = got["sy"][:, :, jj][:, :, :, ii]
        norm = np.abs(ref["avg"][:, keep]).sum(axis=1)
        # a component at rest in the window (zero momentum) is measured against the mass scale
        norm = np.where(norm > 1e-12 * norm[0], norm, norm[0])
        e = (np.abs(g_avg[:, keep] - ref["avg"][:, keep]).sum(axis=1) / norm).max()
        h = (pb["grid"]["x1"] - pb["grid"]["x0"]) / pb["grid"]["nx"]
        m = ref["sx"].shape[1]
        es = max((h * np.abs(g_sx[:, :, keep] - ref["sx"][:, :, keep]).sum(axis=(1, 2)) / (m * norm)).max(),
                 (h * np.abs(g_sy[:, :, keep] - ref["sy"][:, :, keep]).sum(axis=(1, 2)) / (m * norm)).max())
        worst = max(worst, e, es)
        assert e <= tol and es <= tol, (i0, j0, e, es)
    _say(f"  {len(samples)} windows, worst rel-L1 {worst:.3e} (bar {tol:g})")


@functools.lru_cache(maxsize=1)
def _turbulence_2048():
    return W.turbulence_2d(seed=4, n=2048, order=9, nsteps=1, prandtl=0.72, quad=4)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32_flux", 1e-5)])
def test_turbulence_2048_order9(precision, tol):
    pb = _turbulence_2048()
    rng = np.random.default_rng(7)
    samples = [(int(a), int(b)) for a, b in rng.integers(0, 2048, size=(6, 2))] + [(2048 - WIN // 2, 2048 - WIN // 2)]
    _check_2d(pb, precision, samples, periodic=True, tol=tol)


def test_turbulence_2048_500_steps_fp32_flux_error():
    """The whole turbulence run (2048^2, order 9, Pr 0.72, 500 steps at CFL
    0.2): both precisions stay physical, and the FP32-flux state stays within
    1e-5 (rel-L1, averages and h-scaled slopes) of the FP64 path, which the
    windows above pin to the oracle step by step.  Both runs take the FP64
    path's first CFL step as a fixed step, so they are compared at one time."""
    from paper_2508_13705_amd import cgks
    pb = _turbulence_2048()
    h = 1.0 / pb["grid"]["nx"]
    probe = cgks.Solver(pb, precision="fp64")
    probe.step(1)
    dt = probe.read(sync_only=True)["t"]
    del probe
    _say(f"turbulence 2048^2: 500 steps of dt {dt:.4e}, FP32-flux against FP64")
    runs = {p: cgks.Solver(pb, precision=p) for p in ("fp64", "fp32_flux")}
    for s in runs.values():
        s.step(500, dt=dt)
    a, b = runs["fp32_flux"].read(), runs["fp64"].read()
    assert a["status"] == b["status"] == 0 and a["steps"] == b["steps"] == 500
    norm = np.abs(b["avg"]).reshape(4, -1).sum(axis=1)
    e = (np.abs(a["avg"] - b["avg"]).reshape(4, -1).sum(axis=1) / norm).max()
    m = b["sx"].shape[1]
    es = max((h * np.abs(a[k] - b[k]).reshape(4, -1).sum(axis=1) / (m * norm)).max() for k in ("sx", "sy"))
    _say(f"  rel-L1 averages {e:.3e}, slopes {es:.3e} (bar 1e-5)")
    assert e <= 1e-5 and es <= 1e-5, (e, es)


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_quadrant_1024_order7(precision):
    """Four-quadrant Riemann data (the 1024^2 order-7 workload): windows on
    the quadrant interfaces (AO branches), at a corner and at an edge of the
    domain (true transmissive boundary).  FP32-flux is compared with a loose
    bar here (non-smooth data); its smooth-data bar is the turbulence test."""
    pb = W.quadrant_random(seed=3, n=1024, order=7, nsteps=1)
    samples = [(512 - WIN // 2, 512 - WIN // 2), (512 - WIN // 2, 200), (300, 512 - WIN // 2), (0, 0),
               (1024 - WIN, 700), (100, 1024 - WIN)]
    _check_2d(pb, precision, samples, periodic=False, tol=1e-10 if precision == "fp64" else 1e-3)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32_flux", 1e-3)])
def test_riemann_batch_4096_sampled_jobs(precision, tol):
    """The full 4096-job 1-D batch, 10 captured batch steps; sampled jobs are
    rerun by the oracle (FP64) for the steps they took.  FP32-flux is held to
    the loose bar of discontinuous data and its error is reported."""
    from paper_2508_13705_amd import cgks
    probs = W.riemann_batch(seed=2, count=4096)
    _say(f"4096-job 1-D batch, {precision}, 10 steps")
    B = cgks.Batch(1, precision, max_jobs=4096)
    sol = [cgks.Solver(pb, precision=precision) for pb in probs]
    slots = [B.add(s, max_steps=10, t_end=pb["run"]["t_end"]) for s, pb in zip(sol, probs)]
    B.commit()
    B.capture(5)
    B.launch()
    B.launch()
    st = B.poll()
    rng = np.random.default_rng(11)
    picks = list(rng.choice(4096, size=8, replace=False))
    picks.append(int(np.argmax([pb["grid"]["nx"] for pb in probs])))     # the largest job
    worst = 0.0
    for k in picks:
        pb, s, sl = probs[k], sol[k], slots[k]
        got = s.read()
        ref = oracle.run(pb, nsteps=10)
        assert got["status"] == ref["status"], k
        assert got["steps"] == ref["stats"]["steps"] == st[sl]["steps"], k
        if ref["status"] != 0:
            continue
        norm = np.abs(ref["avg"]).sum(axis=1)
        e = (np.abs(got["avg"] - ref["avg"]).sum(axis=1) / norm).max()
        worst = max(worst, e)
        assert e <= tol, (k, e)
    _say(f"  {len(picks)} sampled jobs match the oracle, worst rel-L1 {worst:.3e} (bar {tol:g})")


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_double_mach_960x240(precision):
    """The double Mach reflection at the paper's mesh (Sec. 4.8): windows on
    the wall's breakpoint at x = 1/6 (post-shock inflow | reflecting wall),
    on the top boundary where it follows the shock, on the left inflow, on
    the interior shock and on the right outflow.  Windows that touch the
    domain edge keep its true (segmented, moving) boundary."""
    pb = W.double_mach(240, order=5)
    pb["run"]["t_end"] = 0.0
    samples = [(40 - WIN // 2, 0), (178 - WIN // 2, 240 - WIN), (0, 100), (109 - WIN // 2, 100), (960 - WIN, 50)]
    _check_2d(pb, precision, samples, periodic=False, tol=1e-10 if precision == "fp64" else 1e-3)
