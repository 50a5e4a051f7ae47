"""The allocation-free conservation totals (cgks_conservation_sums_static,
for callers that cannot allocate) against the workspace entry point
(cgks_conservation_sums), through the C ABI: equal bit for bit on two calls
in a row, the second on a smaller grid, and a grid beyond the scratch limit
is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

from paper_2508_13705_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sums_both(s):
    import torch
    from paper_2508_13705_amd import cgks
    L = cgks.lib()
    nv = s.dims[0] + 2
    a = torch.full((nv,), float("nan"), dtype=torch.float64, device=s.device)
    b = torch.full((nv,), float("nan"), dtype=torch.float64, device=s.device)
    st = cgks._stream_handle(s.stream)
    sp = ctypes.c_void_p(s.state.data_ptr())
    cgks.check(L.cgks_conservation_sums(s.plan.handle, sp, ctypes.c_void_p(s.work.data_ptr()),
                                        ctypes.c_void_p(a.data_ptr()), st))
    cgks.check(L.cgks_conservation_sums_static(s.plan.handle, sp, ctypes.c_void_p(b.data_ptr()), st))
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_static_sums_equal_workspace_sums_twice():
    from paper_2508_13705_amd import cgks
    big = cgks.Solver(W.turbulence_2d(seed=4, n=520, order=9, nsteps=2, quad=4), precision="fp32_flux")
    big.step(2)
    small = cgks.Solver(W.quadrant_2d(W.random_quadrants(6), 37, 7, nsteps=3))
    small.step(3)
    for s in (big, small):         # the second call takes a smaller grid
        print(f"\n[no-alloc] {s.problem['name']} {s.dims}", flush=True)
        a, b = _sums_both(s)
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), (a, b)
        ref = s.read()["avg"].reshape(a.size, -1).sum(axis=1)
        assert np.allclose(a, ref, rtol=1e-13, atol=1e-13 * np.abs(s.read()["avg"]).sum())


def test_static_sums_1d_and_oversized_grid_refused():
    from paper_2508_13705_amd import cgks
    s = cgks.Solver(W.fourier_1d(n=700))
    s.step(4)
    a, b = _sums_both(s)
    assert np.array_equal(a, b)
    # 8200 x 8200 interior cells exceed 2^26: refused (plan only, no buffers)
    pb = {"grid": {"dim": 2, "nx": 8200, "ny": 8200, "x0": 0.0, "x1": 1.0, "y0": 0.0, "y1": 1.0,
                   "bc": ["periodic"] * 4},
          "scheme": W.default_scheme(5)}
    plan = cgks.Plan(pb)
    L = cgks.lib()
    st = L.cgks_conservation_sums_static(plan.handle, ctypes.c_void_p(s.state.data_ptr()),
                                         ctypes.c_void_p(s.state.data_ptr()), None)
    assert st == cgks.EINVAL
    assert "too large" in L.cgks_last_error().decode()
