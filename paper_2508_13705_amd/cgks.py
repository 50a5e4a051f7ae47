"""Thin ctypes binding of libcgks.so (C ABI in include/cgks.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels
of the library.  PyTorch provides the device buffers and the stream.  There
is no fallback: without the built library (or without a GPU) every call
raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CGKS_LIB", os.path.join(_HERE, "libcgks.so"))

OK, EINVAL, ENOMEM, EHIP, ENONPHYSICAL, ESTATE, EBUDGET = range(7)
BC = {"periodic": 0, "transmissive": 1, "reflective": 2, "noslip": 3}
BC_INFLOW, BC_SEGMENTED = 4, 5
MAX_SEGMENTS = 3
TAU = {"zero": 0, "inviscid": 1, "viscous": 2}
PRECISION = {"fp64": 0, "fp32_flux": 1}
GAUSS_M = {5: 2, 7: 3, 9: 4}

# every symbol include/cgks.h declares
EXPORTS = ["cgks_plan_create", "cgks_plan_sizes", "cgks_init_state", "cgks_step", "cgks_step_timed",
           "cgks_kernel_name", "cgks_read_state", "cgks_conservation_sums", "cgks_conservation_sums_static",
           "cgks_query_health",
           "cgks_plan_destroy", "cgks_status_string", "cgks_last_error",
           "cgks_batch_create", "cgks_batch_destroy", "cgks_batch_add", "cgks_batch_remove", "cgks_batch_commit",
           "cgks_batch_step", "cgks_batch_capture", "cgks_batch_launch", "cgks_batch_poll", "cgks_batch_info",
           "cgks_batch_set_tuning", "cgks_batch_get_tuning", "cgks_batch_tune"]


class CgksError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"cgks status {status}: {msg}")
        self.status = status


class BcSide(ctypes.Structure):
    _fields_ = [("nseg", ctypes.c_int), ("type", ctypes.c_int * MAX_SEGMENTS),
                ("prim", (ctypes.c_double * 4) * MAX_SEGMENTS),
                ("end0", ctypes.c_double * (MAX_SEGMENTS - 1)), ("speed", ctypes.c_double * (MAX_SEGMENTS - 1))]


class GridDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("bc", ctypes.c_int * 4), ("side", BcSide * 4)]


_SEG_KIND = {"transmissive": 1, "reflective": 2, "noslip": 3, "inflow": BC_INFLOW}


def bc_code(spec, side):
    """Code of one side for cgks_grid_desc.bc; a prescribed state or a
    segmented side also fills ``side``.  ``spec``: "periodic",
    "transmissive", "reflective", "noslip", {"type": "inflow", "prim": [rho,
    u, v, p]} (1-D: [rho, u, p]), or {"segments": [...], "ends": [[end0,
    speed], ...]} (segment k < last: cell centres below end0 + speed t)."""
    if isinstance(spec, str):
        return BC[spec]
    if "segments" not in spec:
        if spec.get("type") != "inflow":
            raise ValueError(f"unknown boundary {spec}")
        side.nseg = 1
        side.type[0] = BC_INFLOW
        for v, x in enumerate(spec["prim"]):
            side.prim[0][v] = float(x)
        return BC_INFLOW
    segs, ends = spec["segments"], spec.get("ends", [])
    side.nseg = len(segs)
    for k, sg in enumerate(segs[:MAX_SEGMENTS]):
        kind = sg if isinstance(sg, str) else sg["type"]
        side.type[k] = _SEG_KIND[kind]
        if kind == "inflow":
            for v, x in enumerate(sg["prim"]):
                side.prim[k][v] = float(x)
    for k, (e, c) in enumerate(ends[:MAX_SEGMENTS - 1]):
        side.end0[k] = float(e)
        side.speed[k] = float(c)
    if len(ends) != len(segs) - 1:
        side.nseg = 0      # rejected by the library
    return BC_SEGMENTED


class SchemeDesc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("gamma", ctypes.c_double), ("tau_model", ctypes.c_int),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("mu", ctypes.c_double),
                ("prandtl", ctypes.c_double), ("sigma_thres", ctypes.c_double), ("gamma_hi", ctypes.c_double),
                ("gamma_lo", ctypes.c_double), ("weno_eps", ctypes.c_double), ("precision", ctypes.c_int),
                ("reading_flags", ctypes.c_int)]


class Health(ctypes.Structure):
    _fields_ = [("nonphysical", ctypes.c_longlong), ("fallbacks", ctypes.c_longlong), ("steps", ctypes.c_longlong),
                ("recon_total", ctypes.c_longlong), ("dff_lt1", ctypes.c_longlong),
                ("ao_branch", ctypes.c_longlong), ("linear", ctypes.c_longlong * 3),
                ("near_ties", ctypes.c_longlong)]


class JobStatus(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("steps", ctypes.c_longlong),
                ("status", ctypes.c_int), ("in_use", ctypes.c_int)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("grid_mult", ctypes.c_int), ("xcd_remap", ctypes.c_int), ("face_tile", ctypes.c_int),
                ("line_tile", ctypes.c_int), ("ms_per_step", ctypes.c_float)]


_lib = None


def lib():
    """Load libcgks.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # One HIP runtime per process: PyTorch's libamdhip64 (the same soname
        # as the one this library needs) is loaded first and serves both;
        # loading this library first would bring in a second runtime that
        # then finds no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.cgks_plan_create.argtypes = [ctypes.POINTER(GridDesc), ctypes.POINTER(SchemeDesc), ctypes.POINTER(vp)]
        L.cgks_plan_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
        L.cgks_init_state.argtypes = [vp, vp, vp, dp, dp, dp, dp, dp, ctypes.c_double, vp]
        L.cgks_step.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp]
        L.cgks_step_timed.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp, dp,
                                      ctypes.POINTER(ctypes.c_int)]
        L.cgks_kernel_name.restype = ctypes.c_char_p
        L.cgks_kernel_name.argtypes = [vp, ctypes.c_int]
        L.cgks_read_state.argtypes = [vp, vp, vp, dp, dp, dp, dp, dp, dp, dp, dp,
                                      ctypes.POINTER(ctypes.c_longlong), vp]
        L.cgks_conservation_sums.argtypes = [vp, vp, vp, vp, vp]
        L.cgks_conservation_sums_static.argtypes = [vp, vp, vp, vp]
        L.cgks_query_health.argtypes = [vp, vp, ctypes.POINTER(Health), vp]
        L.cgks_plan_destroy.argtypes = [vp]
        L.cgks_batch_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.cgks_batch_destroy.argtypes = [vp]
        L.cgks_batch_add.argtypes = [vp, vp, vp, vp, ctypes.c_longlong, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.cgks_batch_remove.argtypes = [vp, ctypes.c_int]
        L.cgks_batch_commit.argtypes = [vp, vp]
        L.cgks_batch_step.argtypes = [vp, ctypes.c_int, vp]
        L.cgks_batch_capture.argtypes = [vp, ctypes.c_int]
        L.cgks_batch_launch.argtypes = [vp, vp]
        L.cgks_batch_poll.argtypes = [vp, ctypes.POINTER(JobStatus), vp]
        L.cgks_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int)]
        L.cgks_batch_set_tuning.argtypes = [vp, ctypes.POINTER(BatchTuning)]
        L.cgks_batch_get_tuning.argtypes = [vp, ctypes.POINTER(BatchTuning)]
        L.cgks_batch_tune.argtypes = [vp, ctypes.c_int, vp, ctypes.POINTER(BatchTuning)]
        L.cgks_status_string.restype = ctypes.c_char_p
        L.cgks_status_string.argtypes = [ctypes.c_int]
        L.cgks_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("cgks_status_string", "cgks_last_error", "cgks_kernel_name"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(status):
    if status != OK:
        raise CgksError(status, lib().cgks_last_error().decode())
    return status


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def descriptors(problem, precision="fp64"):
    """C descriptors of a workload dict (see paper_2508_13705_amd.workloads)."""
    g, s = problem["grid"], problem["scheme"]
    gd = GridDesc()
    gd.dim = g["dim"]
    gd.nx = g["nx"]
    gd.ny = g.get("ny", 1) if g["dim"] == 2 else 1
    gd.x0, gd.x1 = g["x0"], g["x1"]
    gd.y0, gd.y1 = g.get("y0", 0.0), g.get("y1", 1.0)
    for k in range(4):
        gd.bc[k] = bc_code(g["bc"][k], gd.side[k]) if k < len(g["bc"]) else 0
    sd = SchemeDesc()
    sd.order = s["order"]
    sd.gamma = s.get("gamma", 1.4)
    sd.tau_model = TAU[s.get("tau", "zero")]
    sd.c1, sd.c2, sd.mu = s.get("c1", 0.05), s.get("c2", 1.0), s.get("mu", 0.0)
    sd.prandtl = s.get("prandtl", 1.0)
    sd.sigma_thres = s.get("sigma_thres", 1.0)
    sd.gamma_hi, sd.gamma_lo = s.get("gamma_hi", 0.85), s.get("gamma_lo", 0.6)
    sd.weno_eps = s.get("weno_eps", 1e-8)
    sd.precision = PRECISION[precision]
    sd.reading_flags = int(s.get("reading_flags", 0))
    return gd, sd


class Plan:
    def __init__(self, problem, precision="fp64"):
        self.problem = problem
        self.precision = precision
        self.gd, self.sd = descriptors(problem, precision)
        h = ctypes.c_void_p()
        check(lib().cgks_plan_create(ctypes.byref(self.gd), ctypes.byref(self.sd), ctypes.byref(h)))
        self.handle = h
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().cgks_plan_sizes(h, ctypes.byref(sb), ctypes.byref(wb)))
        self.state_bytes, self.work_bytes = sb.value, wb.value

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.cgks_plan_destroy(self.handle)
            self.handle = None


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One grid's state on the GPU: torch-owned device buffers, library kernels."""

    def __init__(self, problem, precision="fp64", device="cuda:0", stream=None, sigma=None, t0=0.0):
        import torch
        self.torch = torch
        self.plan = Plan(problem, precision)
        self.problem = problem
        self.device = torch.device(device)
        self.stream = stream
        self.state = torch.empty(self.plan.state_bytes // 8, dtype=torch.float64, device=self.device)
        self.work = torch.empty(self.plan.work_bytes // 8, dtype=torch.float64, device=self.device)
        self.init(problem["state"], sigma=sigma, t0=t0)

    @property
    def dims(self):
        g = self.problem["grid"]
        return g["dim"], g["nx"], (g.get("ny", 1) if g["dim"] == 2 else 1), \
            (GAUSS_M[self.problem["scheme"]["order"]] if g["dim"] == 2 else 1)

    def init(self, state, sigma=None, t0=0.0):
        dim, nx, ny, m = self.dims
        avg = np.ascontiguousarray(state["avg"], dtype=np.float64)
        sx = np.ascontiguousarray(state["sx"], dtype=np.float64)
        sy = np.ascontiguousarray(state["sy"], dtype=np.float64) if dim == 2 else None
        sgx = sgy = None
        if sigma is not None:
            sgx = np.ascontiguousarray(sigma[0], dtype=np.float64)
            sgy = np.ascontiguousarray(sigma[1], dtype=np.float64) if dim == 2 else None
        with self.torch.cuda.device(self.device):
            check(lib().cgks_init_state(self.plan.handle, ctypes.c_void_p(self.state.data_ptr()),
                                        ctypes.c_void_p(self.work.data_ptr()), _dptr(avg), _dptr(sx), _dptr(sy),
                                        _dptr(sgx), _dptr(sgy), float(t0), _stream_handle(self.stream)))

    def step(self, n=1, dt=0.0, cfl=None, t_end=0.0):
        """Enqueue n steps (asynchronous)."""
        if cfl is None:
            cfl = self.problem["scheme"].get("cfl", 0.5)
        st = _stream_handle(self.stream)
        L = lib()
        sp, wp = ctypes.c_void_p(self.state.data_ptr()), ctypes.c_void_p(self.work.data_ptr())
        for _ in range(n):
            check(L.cgks_step(self.plan.handle, sp, wp, float(dt), float(cfl), float(t_end), st))

    def step_timed(self, dt=0.0, cfl=None, t_end=0.0):
        """One step with per-launch HIP event timing; returns [(name, ms), ...]."""
        if cfl is None:
            cfl = self.problem["scheme"].get("cfl", 0.5)
        ms = (ctypes.c_double * 16)()
        n = ctypes.c_int()
        check(lib().cgks_step_timed(self.plan.handle, ctypes.c_void_p(self.state.data_ptr()),
                                    ctypes.c_void_p(self.work.data_ptr()), float(dt), float(cfl), float(t_end),
                                    _stream_handle(self.stream), ms, ctypes.byref(n)))
        return [(lib().cgks_kernel_name(self.plan.handle, k).decode(), ms[k]) for k in range(n.value)]

    def run(self, nsteps=None, dt=None, t_end=None):
        """Advance as the problem's run block says (nsteps, fixed dt or CFL, t_end)."""
        r = self.problem.get("run", {})
        nsteps = r.get("nsteps", -1) if nsteps is None else nsteps
        dt = r.get("dt", 0.0) if dt is None else dt
        t_end = r.get("t_end", 0.0) if t_end is None else t_end
        if nsteps is None or nsteps < 0:
            # until t_end, or until the device stops the run (a nonphysical
            # state): poll the device time and status every few hundred steps
            while True:
                r = self.read(sync_only=True)
                if r["status"] != OK or r["t"] >= t_end * (1 - 1e-15):
                    break
                self.step(256, dt=dt, t_end=t_end)
        else:
            self.step(nsteps, dt=dt, t_end=t_end)

    def read(self, sync_only=False):
        dim, nx, ny, m = self.dims
        nv = dim + 2
        t = ctypes.c_double()
        steps = ctypes.c_longlong()
        if sync_only:
            st = lib().cgks_read_state(self.plan.handle, ctypes.c_void_p(self.state.data_ptr()),
                                       ctypes.c_void_p(self.work.data_ptr()), None, None, None, None, None, None,
                                       None, ctypes.byref(t), ctypes.byref(steps), _stream_handle(self.stream))
            if st not in (OK, ENONPHYSICAL):
                check(st)
            return {"t": t.value, "steps": steps.value, "status": st}
        avg = np.zeros((nv, ny, nx) if dim == 2 else (nv, nx))
        gx = np.zeros_like(avg)
        gy = np.zeros_like(avg) if dim == 2 else None
        sx = np.zeros((nv, m, ny, nx) if dim == 2 else (nv, nx))
        sy = np.zeros((nv, m, ny, nx)) if dim == 2 else None
        sgx = np.zeros((ny, nx + 1) if dim == 2 else (nx + 1,))
        sgy = np.zeros((ny + 1, nx)) if dim == 2 else None
        st = lib().cgks_read_state(self.plan.handle, ctypes.c_void_p(self.state.data_ptr()),
                                   ctypes.c_void_p(self.work.data_ptr()), _dptr(avg), _dptr(gx), _dptr(gy),
                                   _dptr(sx), _dptr(sy), _dptr(sgx), _dptr(sgy), ctypes.byref(t),
                                   ctypes.byref(steps), _stream_handle(self.stream))
        if st not in (OK, ENONPHYSICAL):
            check(st)
        return {"avg": avg, "gx": gx, "gy": gy, "sx": sx, "sy": sy, "sigx": sgx, "sigy": sgy, "t": t.value,
                "steps": steps.value, "status": st}

    def conservation_sums(self, out=None):
        """Enqueue the device totals of the conserved variables into ``out`` (a
        float64 device tensor of nv entries, allocated here if None); returns it."""
        nv = self.dims[0] + 2
        if out is None:
            out = self.torch.empty(nv, dtype=self.torch.float64, device=self.device)
        check(lib().cgks_conservation_sums(self.plan.handle, ctypes.c_void_p(self.state.data_ptr()),
                                           ctypes.c_void_p(self.work.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           _stream_handle(self.stream)))
        return out

    def health(self):
        h = Health()
        st = lib().cgks_query_health(self.plan.handle, ctypes.c_void_p(self.work.data_ptr()), ctypes.byref(h),
                                     _stream_handle(self.stream))
        if st not in (OK, ENONPHYSICAL):
            check(st)
        return {"nonphysical": h.nonphysical, "fallbacks": h.fallbacks, "steps": h.steps,
                "recon_total": h.recon_total, "dff_lt1": h.dff_lt1, "ao": h.ao_branch, "linear5": h.linear[0],
                "linear7": h.linear[1], "linear9": h.linear[2], "near_ties": h.near_ties, "status": st}


class Batch:
    """Many Solver states of one dimension and precision advanced together by
    the library's persistent batched kernels (include/cgks.h, cgks_batch_*).

    Jobs are Solver objects (their plan and torch-owned buffers); the batch
    keeps a reference to each job until it is removed and committed."""

    def __init__(self, dim, precision="fp64", max_jobs=64, hbm_budget=0, stream=None):
        import torch
        self.torch = torch
        self.dim = dim
        self.precision = precision
        self.max_jobs = max_jobs
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib().cgks_batch_create(dim, PRECISION[precision], max_jobs, int(hbm_budget), ctypes.byref(h)))
        self.handle = h
        self.jobs = {}
        self._status = (JobStatus * max_jobs)()

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.cgks_batch_destroy(self.handle)
            self.handle = None

    def add(self, solver, max_steps=0, dt=0.0, cfl=None, t_end=0.0):
        """Admit a Solver (takes effect at commit); returns its slot.  Raises
        CgksError with status EBUDGET when the budget or slot table is full."""
        if cfl is None:
            cfl = solver.problem["scheme"].get("cfl", 0.5)
        slot = ctypes.c_int(-1)
        check(lib().cgks_batch_add(self.handle, solver.plan.handle, ctypes.c_void_p(solver.state.data_ptr()),
                                   ctypes.c_void_p(solver.work.data_ptr()), int(max_steps), float(dt), float(cfl),
                                   float(t_end), ctypes.byref(slot)))
        self.jobs[slot.value] = solver
        return slot.value

    def remove(self, slot):
        check(lib().cgks_batch_remove(self.handle, int(slot)))
        return self.jobs.pop(slot)

    def commit(self):
        check(lib().cgks_batch_commit(self.handle, _stream_handle(self.stream)))

    def step(self, n=1):
        check(lib().cgks_batch_step(self.handle, int(n), _stream_handle(self.stream)))

    def capture(self, n):
        check(lib().cgks_batch_capture(self.handle, int(n)))

    def launch(self):
        check(lib().cgks_batch_launch(self.handle, _stream_handle(self.stream)))

    def poll(self):
        """{slot: {t, dt, steps, status}} of the jobs held (synchronises)."""
        check(lib().cgks_batch_poll(self.handle, self._status, _stream_handle(self.stream)))
        out = {}
        for k in range(self.max_jobs):
            s = self._status[k]
            if s.in_use:
                out[k] = {"t": s.t, "dt": s.dt, "steps": s.steps, "status": s.status}
        return out

    def info(self):
        n, used, tb, gf = ctypes.c_int(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int()
        check(lib().cgks_batch_info(self.handle, ctypes.byref(n), ctypes.byref(used), ctypes.byref(tb),
                                    ctypes.byref(gf)))
        return {"njobs": n.value, "bytes_used": used.value, "table_bytes": tb.value, "grid_face": gf.value}

    @staticmethod
    def _tuning_dict(t):
        return {"grid_mult": t.grid_mult, "xcd_remap": t.xcd_remap, "face_tile": t.face_tile,
                "line_tile": t.line_tile, "ms_per_step": t.ms_per_step}

    def tuning(self):
        t = BatchTuning()
        check(lib().cgks_batch_get_tuning(self.handle, ctypes.byref(t)))
        return self._tuning_dict(t)

    def set_tuning(self, grid_mult=1, xcd_remap=1, face_tile=0, line_tile=0):
        """Set the launch and tile shapes; a change of tile shape needs a commit
        before the next step."""
        t = BatchTuning(int(grid_mult), int(xcd_remap), int(face_tile), int(line_tile), 0.0)
        check(lib().cgks_batch_set_tuning(self.handle, ctypes.byref(t)))

    def tune(self, steps_per_trial=1):
        """Autotune tile shapes (2-D) and launch shape on the committed jobs
        (real steps); returns the chosen tuning."""
        t = BatchTuning()
        check(lib().cgks_batch_tune(self.handle, int(steps_per_trial), _stream_handle(self.stream), ctypes.byref(t)))
        return self._tuning_dict(t)
