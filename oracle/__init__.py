"""Plain FP64 CPU oracle of the ASE-DFF compact gas-kinetic scheme (arXiv 2508.13705).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU product
path (``paper_2508_13705_amd``) never imports it and shares no code, header,
table or constant generator with it.

The arithmetic lives in ``cgks_oracle.c`` (plain C, FP64, OpenMP over cells);
this module only marshals arguments through ctypes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cgks_oracle.c")
_LIB = os.path.join(_HERE, "libcgks_oracle.so")

BC = {"periodic": 0, "transmissive": 1, "reflective": 2, "noslip": 3}
SEG_TYPE = {"transmissive": 1, "reflective": 2, "noslip": 3, "inflow": 4}
MAXSEG = 3
TAU = {"zero": 0, "inviscid": 1, "viscous": 2}
STENCIL = {"S0": 0, "S1": 1, "S2": 2, "R5": 3, "R7": 4, "R9": 5}


def build(force=True):
    """Compile the oracle with gcc (no fast-math: IEEE FP64 throughout)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Side(ctypes.Structure):
    _fields_ = [("nseg", ctypes.c_int), ("type", ctypes.c_int * MAXSEG), ("prim", (ctypes.c_double * 4) * MAXSEG),
                ("end0", ctypes.c_double * MAXSEG), ("speed", ctypes.c_double * MAXSEG)]


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("order", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("bc", ctypes.c_int * 4),
        ("gamma", ctypes.c_double),
        ("tau_model", ctypes.c_int),
        ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("sigma_thres", ctypes.c_double), ("gamma_hi", ctypes.c_double), ("gamma_lo", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("x0", ctypes.c_double), ("y0", ctypes.c_double),
        ("side", Side * 4),
        ("reading_flags", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                              ctypes.c_double, ctypes.c_double, dp, ctypes.POINTER(ctypes.c_long)]
        L.orc_flux_point.argtypes = [ctypes.POINTER(Params), ctypes.c_int, dp, dp, ctypes.c_double, dp]
        L.orc_micro_solve.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp, dp]
        L.orc_psi_moment.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_u_moments.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp]
        L.orc_xi_moments.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.orc_stencil_fit.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_recon_poly.restype = ctypes.c_int
        L.orc_recon_poly.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp]
        L.orc_poly_eval.restype = ctypes.c_double
        L.orc_poly_eval.argtypes = [dp, ctypes.c_double, ctypes.c_int]
        L.orc_beta.restype = ctypes.c_double
        L.orc_beta.argtypes = [dp, ctypes.c_int]
        L.orc_dff.restype = ctypes.c_double
        L.orc_dff.argtypes = [ctypes.c_int, dp, ctypes.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def gauss_count(order):
    return {5: 2, 7: 3, 9: 4}[order]


def _side(spec, side):
    """Boundary code of one side; a prescribed state or a segmented side is
    written into ``side`` (code 5).  ``spec``: a name of ``BC``, or
    {"type": "inflow", "prim": [rho, u, v, p]} (1-D: [rho, u, p]), or
    {"segments": [...], "ends": [[end0, speed], ...]} with one end per
    segment but the last (segment k: centres below end0 + speed * t)."""
    if isinstance(spec, str):
        return BC[spec]
    segs = spec["segments"] if "segments" in spec else [spec]
    ends = spec.get("ends", [])
    if not 1 <= len(segs) <= MAXSEG or len(ends) != len(segs) - 1:
        raise ValueError(f"bad boundary segments: {spec}")
    side.nseg = len(segs)
    for k, sg in enumerate(segs):
        name = sg if isinstance(sg, str) else sg["type"]
        side.type[k] = SEG_TYPE[name]
        if name == "inflow":
            for v, x in enumerate(sg["prim"]):
                side.prim[k][v] = float(x)
    for k, (e, c) in enumerate(ends):
        side.end0[k] = float(e)
        side.speed[k] = float(c)
    return 5


def make_params(grid, scheme):
    """Fill the C parameter block from a problem's grid and scheme dicts."""
    p = Params()
    p.dim = grid["dim"]
    p.nx = grid["nx"]
    p.ny = grid.get("ny", 1)
    p.order = scheme["order"]
    p.dx = (grid["x1"] - grid["x0"]) / grid["nx"]
    p.dy = (grid["y1"] - grid["y0"]) / p.ny if grid["dim"] == 2 else 1.0
    bc = grid["bc"]
    for k in range(4):
        p.bc[k] = _side(bc[k], p.side[k]) if k < len(bc) else 0
    p.x0 = grid["x0"]
    p.y0 = grid.get("y0", 0.0)
    p.gamma = scheme.get("gamma", 1.4)
    p.tau_model = TAU[scheme.get("tau", "zero")]
    p.c1 = scheme.get("c1", 0.05)
    p.c2 = scheme.get("c2", 1.0)
    p.mu = scheme.get("mu", 0.0)
    p.prandtl = scheme.get("prandtl", 1.0)
    p.sigma_thres = scheme.get("sigma_thres", 1.0)
    p.gamma_hi = scheme.get("gamma_hi", 0.85)
    p.gamma_lo = scheme.get("gamma_lo", 0.6)
    p.weno_eps = scheme.get("weno_eps", 1e-8)
    p.cfl = scheme.get("cfl", 0.5)
    p.reading_flags = int(scheme.get("reading_flags", 0))
    return p


def run(problem, nsteps=None, dt=None, t_end=None, sigma=None, t0=0.0):
    """Advance ``problem`` (a workload dict) and return the new state.

    nsteps / dt / t_end default to ``problem['run']``.  ``sigma`` = (sigx, sigy)
    continues from stored interface strengths; None starts a fresh run.
    Returns dict(avg, sx, sy, sigx, sigy, t, status, stats).
    """
    grid, scheme, st = problem["grid"], problem["scheme"], problem["state"]
    runp = problem.get("run", {})
    if nsteps is None:
        nsteps = runp.get("nsteps", -1)
    if dt is None:
        dt = runp.get("dt", 0.0)
    if t_end is None:
        t_end = runp.get("t_end", 0.0)
    p = make_params(grid, scheme)
    dim, nx, ny = p.dim, p.nx, p.ny
    m = gauss_count(p.order) if dim == 2 else 1
    avg = _f64(st["avg"]).copy()
    sx = _f64(st["sx"]).copy()
    sy = _f64(st["sy"]).copy() if dim == 2 else np.zeros(1)
    if sigma is None:
        sigx = np.zeros((ny, nx + 1)) if dim == 2 else np.zeros(nx + 1)
        sigy = np.zeros((ny + 1, nx)) if dim == 2 else np.zeros(1)
        init = 1
    else:
        sigx, sigy = _f64(sigma[0]).copy(), (_f64(sigma[1]).copy() if dim == 2 else np.zeros(1))
        init = 0
    t = ctypes.c_double(t0)
    stats = (ctypes.c_long * 6)()
    status = lib().orc_run(ctypes.byref(p), _ptr(avg), _ptr(sx), _ptr(sy), _ptr(sigx), _ptr(sigy), init,
                           int(nsteps), float(dt), float(t_end), ctypes.byref(t), stats)
    return {
        "avg": avg, "sx": sx, "sy": sy if dim == 2 else None, "sigx": sigx, "sigy": sigy if dim == 2 else None,
        "t": t.value, "status": status,
        "stats": {"fallback": stats[0], "ao": stats[1], "linear5": stats[2], "linear7": stats[3],
                  "linear9": stats[4], "steps": stats[5]},
    }


# ---- single routines, for the pins ----------------------------------------

def flux_point(scheme, dim, Wl, Wr, dt):
    """Interface results at one Gauss point.  Wl, Wr: [6][4] (value, d_n, d_t,
    d_nn, d_nt, d_tt) x conservative variables in the face frame."""
    p = make_params({"dim": dim, "nx": 1, "ny": 1, "x0": 0, "x1": 1, "y0": 0, "y1": 1, "bc": ["periodic"] * 4},
                    dict(scheme, order=scheme.get("order", 5)))
    a = np.zeros((6, 4)); a[:, :np.shape(Wl)[1]] = Wl
    b = np.zeros((6, 4)); b[:, :np.shape(Wr)[1]] = Wr
    out = np.zeros(22)
    lib().orc_flux_point(ctypes.byref(p), dim, _ptr(_f64(a)), _ptr(_f64(b)), float(dt), _ptr(out))
    nv = dim + 2
    return {"Fh": out[0:nv], "F1": out[4:4 + nv], "W0": out[8:8 + nv], "Wh": out[12:12 + nv],
            "W1": out[16:16 + nv], "sigma": out[20], "tau": out[21]}


def micro_solve(dim, W, gamma, b):
    a = np.zeros(4)
    lib().orc_micro_solve(dim, _ptr(_f64(np.pad(W, (0, 4 - len(W))))), gamma,
                          _ptr(_f64(np.pad(b, (0, 4 - len(b))))), _ptr(a))
    return a[:dim + 2]


def psi_moment(dim, W, gamma, pa, pb, region):
    out = np.zeros(4)
    lib().orc_psi_moment(dim, _ptr(_f64(np.pad(W, (0, 4 - len(W))))), gamma, pa, pb, region, _ptr(out))
    return out[:dim + 2]


def u_moments(U, lam, region, nmax):
    out = np.zeros(nmax + 1)
    lib().orc_u_moments(U, lam, region, nmax, _ptr(out))
    return out


def xi_moments(K, lam, cmax):
    out = np.zeros(cmax + 1)
    lib().orc_xi_moments(K, lam, cmax, _ptr(out))
    return out


def gauss_legendre(m):
    x = np.zeros(4); w = np.zeros(4)
    lib().orc_gauss_legendre(m, _ptr(x), _ptr(w))
    return x[:m], w[:m]


def stencil_fit(which, q, hq):
    c = np.zeros(9)
    lib().orc_stencil_fit(STENCIL[which], _ptr(_f64(q)), _ptr(_f64(hq)), _ptr(c))
    return c


def recon_poly(scheme, q, hq, sig):
    p = make_params({"dim": 1, "nx": 1, "x0": 0, "x1": 1, "bc": ["periodic"] * 2}, scheme)
    c = np.zeros(9)
    br = lib().orc_recon_poly(ctypes.byref(p), _ptr(_f64(q)), _ptr(_f64(hq)), _ptr(_f64(sig)), _ptr(c))
    return c, br


def poly_eval(c, xi, d=0):
    return lib().orc_poly_eval(_ptr(_f64(c)), float(xi), int(d))


def beta(c, deg):
    return lib().orc_beta(_ptr(_f64(c)), int(deg))


def dff(which, sig, thres=1.0):
    return lib().orc_dff(STENCIL[which], _ptr(_f64(sig)), float(thres))
