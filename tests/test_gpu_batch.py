"""Batched execution through the C ABI (cgks_batch_*): every job's result in a
batch -- stepped eagerly, replayed from a captured hipGraph, joined or left
mid-run, under any launch shape -- is bit-identical to the same job stepped
alone with cgks_step, and the batch path matches the FP64 oracle like the
single-grid path does."""
import numpy as np
import pytest

import oracle
from paper_2508_13705_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _say(msg):
    print(f"\n[batch] {msg}", flush=True)


def _same(a, b, dim):
    keys = ("avg", "sx", "sigx") + (("sy", "sigy") if dim == 2 else ())
    for k in keys:
        assert np.array_equal(a[k], b[k]), (k, np.abs(a[k] - b[k]).max())
    assert a["t"] == b["t"] and a["steps"] == b["steps"] and a["status"] == b["status"]


def _mixed_2d():
    """Uneven 2-D jobs: sizes, orders, boundary conditions and data differ."""
    return [
        W.quadrant_2d(W.random_quadrants(11), 23, 5, nsteps=0, name="q23o5"),
        W.fourier_2d(12, 17, 7, nsteps=0),
        W.quadrant_2d(W.CONFIG3, 40, 9, nsteps=0, name="c3n40o9"),
        W.quadrant_2d(W.random_quadrants(13), 31, 7, nsteps=0, name="q31o7"),
        W.fourier_2d(14, 16, 9, nsteps=0),
    ]


def _alone(pb, precision, nsteps, **kw):
    from paper_2508_13705_amd import cgks
    s = cgks.Solver(pb, precision=precision)
    s.step(nsteps, **kw)
    return s.read()


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_batch_2d_equals_alone(precision):
    from paper_2508_13705_amd import cgks
    pbs = _mixed_2d()
    steps = [6, 4, 5, 3, 6]
    _say(f"2-D mixed batch of {len(pbs)} jobs, {precision}")
    b = cgks.Batch(2, precision, max_jobs=8)
    sol = [cgks.Solver(pb, precision=precision) for pb in pbs]
    slots = [b.add(s, max_steps=k) for s, k in zip(sol, steps)]
    b.commit()
    b.step(7)   # one more step than the longest job: the finished jobs idle
    st = b.poll()
    for s, k, sl in zip(sol, steps, slots):
        assert st[sl]["status"] == 1 and st[sl]["steps"] == k
    for pb, s, k in zip(pbs, sol, steps):
        _same(s.read(), _alone(pb, precision, k), 2)


def test_batch_2d_matches_oracle():
    from paper_2508_13705_amd import cgks
    pbs = _mixed_2d()[:3]
    _say("2-D batch vs oracle")
    b = cgks.Batch(2, "fp64", max_jobs=4)
    sol = [cgks.Solver(pb) for pb in pbs]
    for s in sol:
        b.add(s, max_steps=4)
    b.commit()
    b.step(4)
    for pb, s in zip(pbs, sol):
        got = s.read()
        ref = oracle.run(pb, nsteps=4)
        assert got["status"] == ref["status"] == 0
        norm = np.abs(ref["avg"]).sum(axis=(1, 2))
        e = (np.abs(got["avg"] - ref["avg"]).sum(axis=(1, 2)) / norm).max()
        assert e <= TOL64, (pb["name"], e)


def test_batch_1d_riemann_equals_alone():
    """Uneven 1-D Riemann jobs of the batch workload (cell counts cut)."""
    from paper_2508_13705_amd import cgks
    pbs = W.riemann_batch(seed=2, count=12)
    small = []
    for pb in pbs:
        n = pb["grid"]["nx"] // 8 + 20
        L, R = pb["riemann"]["left"], pb["riemann"]["right"]
        small.append(W.riemann_1d(L, R, n, 9, 0.15, xs=(n // 2) / n))
    _say(f"1-D batch of {len(small)} jobs")
    for precision in ("fp64", "fp32_flux"):
        b = cgks.Batch(1, precision, max_jobs=16)
        sol = [cgks.Solver(pb, precision=precision) for pb in small]
        for s in sol:
            b.add(s, max_steps=25, t_end=0.15)
        b.commit()
        b.step(26)
        for pb, s in zip(small, sol):
            _same(s.read(), _alone(pb, precision, 25, t_end=0.15), 1)


def test_graph_replays_equal_eager():
    """A captured multi-step graph replayed several times, with eager work and
    synchronisations between replays, gives the eager result after every
    replay."""
    import torch
    from paper_2508_13705_amd import cgks
    pbs = _mixed_2d()
    _say("graph replay vs eager")
    bg = cgks.Batch(2, "fp64", max_jobs=8)
    be = cgks.Batch(2, "fp64", max_jobs=8)
    sg = [cgks.Solver(pb) for pb in pbs]
    se = [cgks.Solver(pb) for pb in pbs]
    for a, c in zip(sg, se):
        bg.add(a, max_steps=100)
        be.add(c, max_steps=100)
    bg.commit()
    be.commit()
    bg.capture(2)
    for rep in range(3):
        bg.launch()
        be.step(2)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
        for a, c in zip(sg, se):
            _same(a.read(), c.read(), 2)
        _say(f"replay {rep} ok")


def test_join_and_leave_mid_run():
    """Jobs admitted while others run, and retired while others continue,
    give their alone results (continuous batching)."""
    from paper_2508_13705_amd import cgks
    pbs = _mixed_2d()
    _say("join/leave")
    b = cgks.Batch(2, "fp64", max_jobs=3)
    s0, s1 = cgks.Solver(pbs[0]), cgks.Solver(pbs[1])
    k0 = b.add(s0, max_steps=5)
    b.commit()
    b.capture(1)
    b.launch()
    b.launch()
    k1 = b.add(s1, max_steps=6)   # joins after s0 has taken 2 steps
    b.commit()
    for _ in range(5):
        b.launch()                 # the graph captured before the join serves the new table
    st = b.poll()
    assert st[k0]["status"] == 1 and st[k0]["steps"] == 5
    assert st[k1]["steps"] == 5
    b.remove(k0)
    s2 = cgks.Solver(pbs[2])
    k2 = b.add(s2, max_steps=3)
    b.commit()
    b.step(3)
    st = b.poll()
    assert st[k1]["status"] == 1 and st[k1]["steps"] == 6
    assert st[k2]["status"] == 1 and st[k2]["steps"] == 3
    _same(s0.read(), _alone(pbs[0], "fp64", 5), 2)
    _same(s1.read(), _alone(pbs[1], "fp64", 6), 2)
    _same(s2.read(), _alone(pbs[2], "fp64", 3), 2)


def test_every_launch_shape_gives_the_same_result():
    from paper_2508_13705_amd import cgks
    pbs = _mixed_2d()[:3]
    _say("launch shapes and autotuner")
    ref = [_alone(pb, "fp32_flux", 8) for pb in pbs]
    for mult, remap in ((1, 0), (2, 1), (4, 0)):
        b = cgks.Batch(2, "fp32_flux", max_jobs=4)
        b.set_tuning(mult, remap)
        sol = [cgks.Solver(pb, precision="fp32_flux") for pb in pbs]
        for s in sol:
            b.add(s, max_steps=8)
        b.commit()
        b.step(8)
        for s, r in zip(sol, ref):
            _same(s.read(), r, 2)
    # the autotuner's trial steps are ordinary steps
    b = cgks.Batch(2, "fp32_flux", max_jobs=4)
    sol = [cgks.Solver(pb, precision="fp32_flux") for pb in pbs]
    for s in sol:
        b.add(s, max_steps=8)
    b.commit()
    t = b.tune(1)                  # 6 tile-shape and 6 launch candidates x 1 step
    assert t["grid_mult"] in (1, 2, 4) and t["ms_per_step"] > 0
    assert t["face_tile"] in (0, 1, 2) and t["line_tile"] in (0, 1)
    b.step(2)
    for s, r in zip(sol, ref):
        _same(s.read(), r, 2)


@pytest.mark.parametrize("precision", ["fp64", "fp32_flux"])
def test_every_tile_shape_gives_the_same_result(precision):
    """The batched face kernels in each tile shape (16 x NT, 32 x NT/2,
    8 x 2 NT faces x lines) and the Step 1 kernel in each (32 x 8, 16 x 16)
    compute every face and cell as the job alone does: bit for bit, for
    uneven jobs of every order; a change of shape between steps is taken
    after a commit."""
    from paper_2508_13705_amd import cgks
    pbs = _mixed_2d()
    ref = [_alone(pb, precision, 6) for pb in pbs]
    for ft in range(3):
        for lt in range(2):
            _say(f"tile shapes face {ft} lines {lt}, {precision}")
            b = cgks.Batch(2, precision, max_jobs=8)
            b.set_tuning(2, 1, ft, lt)
            sol = [cgks.Solver(pb, precision=precision) for pb in pbs]
            for q in sol:
                b.add(q, max_steps=6)
            b.commit()
            b.step(3)
            # switch shapes half way (the table is uploaded again)
            b.set_tuning(1, 0, (ft + 1) % 3, 1 - lt)
            b.commit()
            b.step(3)
            assert b.tuning()["face_tile"] == (ft + 1) % 3
            for q, r in zip(sol, ref):
                _same(q.read(), r, 2)


def test_t_end_and_nonphysical_jobs_stop_alone():
    """A job that reaches t_end, and a job that goes nonphysical, stop; the
    others are unaffected."""
    from paper_2508_13705_amd import cgks
    sod = W.shock_tube("sod", 60, 5)
    blanc = W.shock_tube("le_blanc", 120, 9)
    smooth = W.fourier_1d(n=64)
    _say("t_end / nonphysical")
    b = cgks.Batch(1, "fp64", max_jobs=4)
    s_sod, s_bl, s_sm = cgks.Solver(sod), cgks.Solver(blanc), cgks.Solver(smooth)
    k_sod = b.add(s_sod, max_steps=0, t_end=0.05)
    k_bl = b.add(s_bl, max_steps=400)
    k_sm = b.add(s_sm, max_steps=40)
    b.commit()
    b.step(400)
    st = b.poll()
    assert st[k_sod]["status"] == 1 and st[k_sod]["t"] == pytest.approx(0.05, rel=0, abs=1e-15)
    assert st[k_sm]["status"] == 1 and st[k_sm]["steps"] == 40
    assert st[k_bl]["status"] in (1, 2)
    r = _alone(sod, "fp64", st[k_sod]["steps"], t_end=0.05)
    _same(s_sod.read(), r, 1)
    _same(s_sm.read(), _alone(smooth, "fp64", 40), 1)
    al = cgks.Solver(blanc)
    if st[k_bl]["status"] == 1:
        al.step(st[k_bl]["steps"])
        _same(s_bl.read(), al.read(), 1)
    else:   # the batch stopped it after the step that went nonphysical
        al.step(st[k_bl]["steps"] + 1)
        a = al.read()
        assert a["status"] == s_bl.read()["status"] != 0
        assert a["steps"] == st[k_bl]["steps"]


def test_budget_and_slots():
    from paper_2508_13705_amd import cgks
    pb = W.fourier_2d(12, 17, 7, nsteps=0)
    s = cgks.Solver(pb)
    need = s.plan.state_bytes + s.plan.work_bytes
    b = cgks.Batch(2, "fp64", max_jobs=2, hbm_budget=need * 2 - 1)
    b.add(s, max_steps=1)
    s2 = cgks.Solver(pb)
    with pytest.raises(cgks.CgksError) as e:
        b.add(s2, max_steps=1)
    assert e.value.status == cgks.EBUDGET
    assert b.info()["bytes_used"] == need
    b2 = cgks.Batch(2, "fp64", max_jobs=1)
    b2.add(s, max_steps=1)
    with pytest.raises(cgks.CgksError) as e:
        b2.add(s2, max_steps=1)
    assert e.value.status == cgks.EBUDGET
    with pytest.raises(cgks.CgksError) as e:
        b2.step(1)                # added but not committed
    assert e.value.status == cgks.ESTATE
    b3 = cgks.Batch(1, "fp64", max_jobs=1)
    with pytest.raises(cgks.CgksError) as e:
        b3.add(s, max_steps=1)    # 2-D job in a 1-D batch
    assert e.value.status == cgks.EINVAL
