"""Writes the oracle results that the full-step-count parity tests compare
against (tests/test_gpu_fullsteps.py).  It calls only the CPU oracle
(oracle/) and the seeded input generators (paper_2508_13705_amd.workloads,
which hold initial data and no arithmetic of the scheme); no value here comes
from the HIP path.

    python tests/golden/make_parity_fixtures.py [c2] [c2f] [c3] [c4]

Configurations, each run for its full step count on a grid the oracle
finishes in minutes:
  c2  1-D Riemann batch (4096 problems, seed 2, order 9, CFL 0.5, t_end 0.15):
      a fixed subset of 32 problems, the 16 with the least predicted work
      (cells x steps, the steps from the initial signal speed) and 16 drawn
      with a fixed seed from those below the median predicted work, each run
      to t_end; a problem whose cell averages turn nonphysical is stored at
      the step before (with the step on which it stops);
  c2f the first four problems of the same batch (pressure ratio above 1000)
      whose run turns nonphysical within 50 steps, stored at the step before;
  c3  four-quadrant Riemann problem (seed 3), order 7, CFL 0.5, 200 steps,
      on 128 x 128 cells;
  c4  2-D Navier-Stokes turbulence (seed 4), order 9, mu 1e-4, Pr 0.72,
      CFL 0.2, 500 steps, on 64 x 64 cells with the spectrum cut at |k| <= 8
      (the full workload's |k| <= 32 is not resolved on 64 cells).
Results are stored as compressed .npz (loaded with allow_pickle=False).
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2508_13705_amd import workloads as W  # noqa: E402

C2_COUNT, C2_SMALLEST, C2_RANDOM, C2_SEED = 4096, 16, 16, 22


def c2_subset(probs):
    """Indices of the fixed subset (see the module docstring)."""
    work = []
    for pb in probs:
        r = pb["riemann"]
        g = r["gamma"]
        s = max(abs(u) + math.sqrt(g * p / rho) for rho, u, p in (r["left"], r["right"]))
        n = pb["grid"]["nx"]
        work.append(n * pb["run"]["t_end"] * s * n / pb["scheme"]["cfl"])
    work = np.array(work)
    order = np.argsort(work, kind="stable")
    small = [int(k) for k in order[:C2_SMALLEST]]
    med = np.median(work)
    pool = [k for k in range(len(probs)) if work[k] <= med and k not in small]
    rng = np.random.default_rng(C2_SEED)
    pick = sorted(int(k) for k in rng.choice(pool, size=C2_RANDOM, replace=False))
    return sorted(small + pick)


def make_c2():
    probs = W.riemann_batch(seed=2, count=C2_COUNT)
    idx = c2_subset(probs)
    rows = {"index": [], "status": [], "steps": [], "t": [], "nx": []}
    avg, sx = [], []
    for k in idx:
        pb = probs[k]
        t0 = time.time()
        r = oracle.run(pb)
        status, steps = r["status"], r["stats"]["steps"]
        if status != 0:
            # the state the run held before the step that turned it nonphysical
            r = oracle.run(pb, nsteps=steps - 1)
            assert r["status"] == 0
        rows["index"].append(k)
        rows["status"].append(status)
        rows["steps"].append(steps)
        rows["t"].append(r["t"])
        rows["nx"].append(pb["grid"]["nx"])
        avg.append(r["avg"])
        sx.append(r["sx"])
        print(f"c2 job {k}: nx {pb['grid']['nx']} status {status} steps {steps} ({time.time() - t0:.1f} s)",
              flush=True)
    np.savez_compressed(os.path.join(HERE, "c2_riemann_subset_o9.npz"),
                        **{key: np.array(v) for key, v in rows.items()},
                        avg=np.concatenate(avg, axis=1), sx=np.concatenate(sx, axis=1))


def make_c2_failing(count=4, scan_steps=50):
    """The first `count` problems of the batch (in index order, among those
    with a pressure ratio above 1000) whose oracle run turns nonphysical
    within `scan_steps` steps: the step on which each stops and the state on
    the step before."""
    probs = W.riemann_batch(seed=2, count=C2_COUNT)
    rows = {"index": [], "steps": [], "t": [], "nx": []}
    avg, sx = [], []
    for k, pb in enumerate(probs):
        r = pb["riemann"]
        if max(r["left"][2], r["right"][2]) / min(r["left"][2], r["right"][2]) < 1000.0:
            continue
        res = oracle.run(pb, nsteps=scan_steps)
        if res["status"] == 0:
            continue
        steps = res["stats"]["steps"]
        prev = oracle.run(pb, nsteps=steps - 1)
        assert prev["status"] == 0
        rows["index"].append(k)
        rows["steps"].append(steps)
        rows["t"].append(prev["t"])
        rows["nx"].append(pb["grid"]["nx"])
        avg.append(prev["avg"])
        sx.append(prev["sx"])
        print(f"c2 failing job {k}: nx {pb['grid']['nx']} stops nonphysical on step {steps}", flush=True)
        if len(rows["index"]) == count:
            break
    np.savez_compressed(os.path.join(HERE, "c2_riemann_failing_o9.npz"),
                        **{key: np.array(v) for key, v in rows.items()},
                        avg=np.concatenate(avg, axis=1), sx=np.concatenate(sx, axis=1))


def c3_problem():
    return W.quadrant_random(seed=3, n=128, order=7, nsteps=200)


def c4_problem():
    return W.turbulence_2d(seed=4, n=64, order=9, nsteps=500, kmax=8, mu=1e-4, prandtl=0.72, cfl=0.2, quad=4)


def make_2d(name, pb):
    t0 = time.time()
    r = oracle.run(pb)
    print(f"{name}: status {r['status']} steps {r['stats']['steps']} t {r['t']:.6f} ({time.time() - t0:.0f} s)",
          flush=True)
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), avg=r["avg"], sx=r["sx"], sy=r["sy"], t=r["t"],
                        steps=r["stats"]["steps"], status=r["status"],
                        stats=np.array([r["stats"][k] for k in ("fallback", "ao", "linear5", "linear7", "linear9")]))


if __name__ == "__main__":
    want = sys.argv[1:] or ["c2", "c2f", "c3", "c4"]
    if "c3" in want:
        make_2d("c3_quadrant128_o7_200", c3_problem())
    if "c4" in want:
        make_2d("c4_turbulence64_o9_500", c4_problem())
    if "c2" in want:
        make_c2()
    if "c2f" in want:
        make_c2_failing()
