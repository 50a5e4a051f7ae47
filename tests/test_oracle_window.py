"""The windowing the full-size GPU parity tests rely on: one step of the
oracle on a window of a grid reproduces the whole-grid step, bit for bit, on
every cell at least MARGIN cells inside the window's artificial edges."""
import numpy as np

import oracle
from paper_2508_13705_amd import workloads as W

from test_gpu_fullsize import MARGIN, WIN, _window


def _compare(pb, samples, periodic):
    full = oracle.run(pb, nsteps=1)
    dt = full["t"]
    for i0, j0 in samples:
        wpb, ii, jj, keep = _window(pb, i0, j0, periodic)
        w = oracle.run(wpb, nsteps=1, dt=dt)
        f_avg = full["avg"][:, jj][:, :, ii]
        f_sx = full["sx"][:, :, jj][:, :, :, ii]
        assert np.array_equal(w["avg"][:, keep], f_avg[:, keep]), (i0, j0)
        assert np.array_equal(w["sx"][:, :, keep], f_sx[:, :, keep]), (i0, j0)
        # the margin is needed: cells next to an artificial edge do differ
        if periodic:
            assert not np.array_equal(w["avg"], f_avg)


def test_window_periodic_turbulence():
    pb = W.turbulence_2d(seed=4, n=64, order=9, nsteps=1, kmax=8, prandtl=0.72, quad=4)
    _compare(pb, [(5, 9), (40, 50)], periodic=True)


def test_window_transmissive_quadrants():
    pb = W.quadrant_random(seed=3, n=64, order=7, nsteps=1)
    _compare(pb, [(32 - WIN // 2, 32 - WIN // 2), (0, 0), (64 - WIN, 10)], periodic=False)
