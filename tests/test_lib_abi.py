"""The C-ABI library loads and exports every symbol include/cgks.h declares;
host-side plan validation (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2508_13705_amd import cgks, workloads

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cgks.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgks_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(cgks.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = cgks.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def _plan(pb, precision="fp64"):
    return cgks.Plan(pb, precision)


def test_plan_sizes_match_layout():
    pb = workloads.quadrant_2d(workloads.CONFIG3, 20, 9, nsteps=1)
    p = _plan(pb)
    NX = NY = 26
    cells = NX * NY
    assert p.state_bytes == 8 * 4 * cells * (1 + 2 * 4)
    assert p.work_bytes >= 8 * (2 * 4 * cells * 9 + 2 * 4 * 4 * cells)
    pb1 = workloads.fourier_1d(n=64)
    p1 = _plan(pb1)
    assert p1.state_bytes == 8 * 3 * 70 * 2


@pytest.mark.parametrize("mutate,frag", [
    (lambda g, s: s.update(order=6), "order"),
    (lambda g, s: s.update(gamma=1.0), "gamma"),
    (lambda g, s: g.update(nx=4), "5 cells"),
    (lambda g, s: g.update(bc=["periodic", "transmissive", "periodic", "periodic"]), "periodic"),
    (lambda g, s: s.update(prandtl=0.0), "prandtl"),
    (lambda g, s: s.update(sigma_thres=0.0), "sigma_thres"),
    (lambda g, s: g["bc"].__setitem__(0, {"type": "inflow", "prim": [-1.0, 0.0, 0.0, 1.0]}), "rho > 0"),
    (lambda g, s: g["bc"].__setitem__(0, {"type": "inflow", "prim": [1.0, 0.0, 0.0, 0.0]}), "p > 0"),
    (lambda g, s: g["bc"].__setitem__(2, {"segments": ["reflective", "noslip"], "ends": []}), "segments"),
    (lambda g, s: g["bc"].__setitem__(2, {"segments": ["reflective", "noslip"], "ends": [[float("nan"), 0.0]]}),
     "finite"),
])
def test_plan_rejects_bad_descriptors(mutate, frag):
    pb = workloads.quadrant_2d(workloads.CONFIG3, 12, 7, nsteps=1)
    mutate(pb["grid"], pb["scheme"])
    with pytest.raises(cgks.CgksError) as e:
        _plan(pb)
    assert e.value.status == cgks.EINVAL
    assert frag in str(e.value)


def test_status_strings():
    L = cgks.lib()
    assert L.cgks_status_string(0) == b"ok"
    assert L.cgks_status_string(4) == b"nonphysical state"


@pytest.mark.parametrize("dim,prec,cap,frag", [
    (3, 0, 4, "dim"),
    (2, 7, 4, "precision"),
    (2, 0, 0, "max_jobs"),
])
def test_batch_create_rejects_bad_arguments(dim, prec, cap, frag):
    """Argument checks come before any device call (no GPU needed)."""
    L = cgks.lib()
    h = ctypes.c_void_p()
    st = L.cgks_batch_create(dim, prec, cap, 0, ctypes.byref(h))
    assert st == cgks.EINVAL
    assert frag in L.cgks_last_error().decode()
    assert not h.value


def test_batch_calls_reject_null_batch():
    L = cgks.lib()
    assert L.cgks_batch_commit(None, None) == cgks.EINVAL
    assert L.cgks_batch_step(None, 1, None) == cgks.EINVAL
    assert L.cgks_batch_launch(None, None) == cgks.EINVAL
    assert L.cgks_batch_remove(None, 0) == cgks.EINVAL
    assert L.cgks_batch_destroy(None) == cgks.OK


def test_plan_accepts_wall_inflow_and_moving_sides():
    for pb in (workloads.double_mach(12), workloads.viscous_shock_tube(20), workloads.jet(80, 24)):
        p = _plan(pb)
        assert p.work_bytes > 0
