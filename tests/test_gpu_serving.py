"""Serving loop (continuous batching under an HBM budget): every job's result
is bit-identical to the same job run alone, jobs overlap on the device, and
admission waits for memory."""
import numpy as np
import pytest

from paper_2508_13705_amd import workloads as W

pytestmark = pytest.mark.gpu


def _trace():
    # small sides (16..64), every order, both kinds of initial data, 4-20 steps
    tr = W.serving_trace(seed=5, count=12, rate=1e4, nmin_log2=4.0, nmax_log2=6.0, steps=(4, 20))
    return tr


@pytest.mark.parametrize("lanes", [(512, 1024), (24, 40)], ids=["one-lane", "three-lanes"])
def test_each_result_is_the_same_alone_and_in_the_mix(lanes):
    """With lane limits (24, 40) the 16-64 sided jobs spread over three
    lanes, whose graphs run concurrently on their own streams."""
    from paper_2508_13705_amd import cgks, serving
    tr = _trace()
    sizes = sorted(serving.job_bytes(j, "fp64") for j in tr)
    budget = sum(sizes[-3:])       # about three jobs at a time: admission must wait for memory
    print(f"\n[serving] {len(tr)} jobs, budget {budget} bytes, lanes {lanes}", flush=True)
    loop = serving.ServingLoop(2, "fp64", hbm_budget=budget, max_jobs=6, graph_steps=3, prep_workers=2,
                               keep_results=True, lane_sides=lanes)
    rep = loop.run(tr)
    used = {sum(1 for m in lanes if r["job"]["n"] > m) for r in rep["records"]}
    assert len(used) == (1 if lanes == (512, 1024) else 3)
    print("[serving] p50 %.3f s p99 %.3f s, max running %d" % (rep["latency_p50_s"], rep["latency_p99_s"],
                                                                rep["max_running"]), flush=True)
    assert rep["jobs"] == len(tr) and rep["rejected"] == 0
    assert rep["max_running"] >= 2            # jobs shared the device
    assert any(r["waited_for_memory"] for r in rep["records"])   # admission waited for memory
    assert rep["latency_p99_s"] >= rep["latency_p50_s"] > 0
    for r in rep["records"]:
        job = r["job"]
        alone = cgks.Solver(W.serving_problem(job))
        alone.step(job["nsteps"])
        a = alone.read()
        got = r["result"]
        assert got["status"] == a["status"]
        if a["status"] != 0:     # stopped after the same step in both runs
            assert got["steps"] == a["steps"]
            continue
        assert got["steps"] == a["steps"] == job["nsteps"]
        for k in ("avg", "sx", "sy", "sigx", "sigy"):
            assert np.array_equal(got[k], a[k]), (job, k)


def test_oversized_job_is_rejected():
    from paper_2508_13705_amd import serving
    tr = _trace()[:3]
    big = dict(tr[0], id=99, n=64, order=9)
    budget = serving.job_bytes(big, "fp64") - 1
    loop = serving.ServingLoop(2, "fp64", hbm_budget=budget, max_jobs=4, graph_steps=2, tune=False)
    rep = loop.run([j for j in tr if serving.job_bytes(j, "fp64") <= budget] + [big])
    assert rep["rejected"] == 1
