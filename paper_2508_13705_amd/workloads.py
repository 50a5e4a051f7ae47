"""Seeded synthetic workloads shaped like the paper's test problems.

This module holds only initial data: grids, scheme parameters and the exact
projection of analytic initial fields onto cell averages and line-averaged
slopes.  It contains none of the scheme's arithmetic, and both the HIP path
and the CPU oracle take their inputs from here.

Every problem is a plain dict::

    {"name": str,
     "grid":   {"dim", "nx", "ny", "x0", "x1", "y0", "y1", "bc": [xlo, xhi, ylo, yhi]},
     "scheme": {"order", "gamma", "tau", "c1", "c2", "mu", "prandtl", "sigma_thres",
                "gamma_hi", "gamma_lo", "weno_eps", "cfl"},
     "state":  {"avg": [nv][ny][nx], "sx": [nv][m][ny][nx], "sy": [nv][m][ny][nx]}
               (1-D: avg [3][nx], sx [3][nx] = cell-averaged slope),
     "run":    {"nsteps", "dt", "t_end"}}

Line-averaged slopes (Sec. 3.3): sx[v][l][j][i] is the x-derivative averaged
along the horizontal Gauss line y = y_j + xi_l dy of cell (i, j), i.e.
(W(x_{i+1/2}, y_l) - W(x_{i-1/2}, y_l)) / dx; sy likewise along vertical lines.
Gauss-Legendre points with m = 2, 3, 4 for orders 5, 7, 9.
"""
import math

import numpy as np

GAUSS_M = {5: 2, 7: 3, 9: 4}


def gauss_legendre(m):
    """Gauss-Legendre nodes on [-1/2, 1/2] and weights summing to 1."""
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * x, 0.5 * w


def default_scheme(order, **kw):
    s = {"order": order, "gamma": 1.4, "tau": "zero", "c1": 0.05, "c2": 1.0, "mu": 0.0, "prandtl": 1.0,
         "sigma_thres": 1.0, "gamma_hi": 0.85, "gamma_lo": 0.6, "weno_eps": 1e-8, "cfl": 0.5}
    s.update(kw)
    return s


def _cons(rho, u, v, p, gamma, dim):
    if dim == 1:
        return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def _sinc(z):
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = np.abs(z) > 1e-300
    out[nz] = np.sin(z[nz]) / z[nz]
    return out


# ---------------------------------------------------------------------------
# 1-D
# ---------------------------------------------------------------------------

def _fourier_rho_1d(modes, x0, x1, n):
    """Exact cell averages and face values of rho = 1 + sum a sin(pi k x + phi)."""
    dx = (x1 - x0) / n
    xc = x0 + (np.arange(n) + 0.5) * dx
    xf = x0 + np.arange(n + 1) * dx
    avg = np.ones(n)
    face = np.ones(n + 1)
    for a, k, ph in modes:
        w = math.pi * k
        avg += a * np.sin(w * xc + ph) * _sinc(0.5 * w * dx)
        face += a * np.sin(w * xf + ph)
    return avg, face, dx


def smooth_1d(modes, n, order, u=1.0, p=1.0, gamma=1.4, x0=0.0, x1=2.0, nsteps=100, dt=0.0, t_end=0.0,
              name="smooth_1d", **scheme_kw):
    """Density wave on a periodic line: W is linear in rho, so exact cell
    averages follow from those of rho, and the cell-averaged slope is the
    difference of the face values over dx."""
    ra, rf, dx = _fourier_rho_1d(modes, x0, x1, n)
    ones = np.ones_like
    avg = _cons(ra, u * ones(ra), None, p * ones(ra), gamma, 1)
    face = _cons(rf, u * ones(rf), None, p * ones(rf), gamma, 1)
    sx = (face[:, 1:] - face[:, :-1]) / dx
    return {"name": name,
            "grid": {"dim": 1, "nx": n, "ny": 1, "x0": x0, "x1": x1, "y0": 0.0, "y1": 1.0,
                     "bc": ["periodic", "periodic"]},
            "scheme": default_scheme(order, gamma=gamma, tau="zero", **scheme_kw),
            "state": {"avg": avg, "sx": sx},
            "run": {"nsteps": nsteps, "dt": dt, "t_end": t_end},
            "modes": modes}


def advection_1d(order, n, t_end=2.0, c=0.3):
    """Accuracy test of Sec. 4.1: rho = 1 + 0.2 sin(pi x), U = 1, p = 1 on
    [0, 2], periodic; dt = c dx^(r/4) rounded down to divide t_end."""
    dx = 2.0 / n
    dt0 = c * dx ** (order / 4.0)
    nsteps = int(math.ceil(t_end / dt0 - 1e-12))
    return smooth_1d([(0.2, 1.0, 0.0)], n, order, nsteps=nsteps, dt=t_end / nsteps, t_end=0.0,
                     name=f"advection_1d_r{order}_n{n}")


def fourier_1d(seed=1, n=256, order=5, nsteps=100, cfl=0.5):
    """rho = 1 + sum of 4 seeded Fourier modes (total amplitude 0.2), u = 1, p = 1
    on periodic [0, 2]; CFL time step."""
    rng = np.random.default_rng(seed)
    ks = rng.choice(np.arange(1, 9), size=4, replace=False)
    w = rng.uniform(0.0, 1.0, size=4)
    a = 0.2 * w / w.sum()
    ph = rng.uniform(0.0, 2.0 * math.pi, size=4)
    modes = [(float(a[j]), float(ks[j]), float(ph[j])) for j in range(4)]
    return smooth_1d(modes, n, order, nsteps=nsteps, dt=0.0, name=f"fourier_1d_s{seed}", cfl=cfl)


def riemann_1d(left, right, n, order, t_end, x0=0.0, x1=1.0, xs=0.5, gamma=1.4, tau="inviscid", cfl=0.5,
               bc="transmissive", nsteps=-1, name="riemann_1d", **scheme_kw):
    """Piecewise-constant (rho, u, p) states split at the face nearest xs;
    exact cell averages, zero slopes."""
    dx = (x1 - x0) / n
    kf = int(round((xs - x0) / dx))
    rho = np.where(np.arange(n) < kf, left[0], right[0]).astype(np.float64)
    u = np.where(np.arange(n) < kf, left[1], right[1]).astype(np.float64)
    p = np.where(np.arange(n) < kf, left[2], right[2]).astype(np.float64)
    avg = _cons(rho, u, None, p, gamma, 1)
    return {"name": name,
            "grid": {"dim": 1, "nx": n, "ny": 1, "x0": x0, "x1": x1, "y0": 0.0, "y1": 1.0, "bc": [bc, bc]},
            "scheme": default_scheme(order, gamma=gamma, tau=tau, cfl=cfl, **scheme_kw),
            "state": {"avg": avg, "sx": np.zeros_like(avg)},
            "run": {"nsteps": nsteps, "dt": 0.0, "t_end": t_end},
            "riemann": {"left": tuple(left), "right": tuple(right), "xs": x0 + kf * dx, "gamma": gamma}}


SHOCK_TUBES = {
    # Sec. 4.2 and 4.5
    "sod": dict(left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), t_end=0.2),
    "lax": dict(left=(0.445, 0.698, 3.528), right=(0.5, 0.0, 0.571), t_end=0.14),
    "double_rarefaction": dict(left=(1.0, -2.0, 0.1), right=(1.0, 2.0, 0.1), t_end=0.1),
    "le_blanc": dict(left=(1.0, 0.0, 2.0 / 3.0 * 1e-1), right=(1e-3, 0.0, 2.0 / 3.0 * 1e-10), t_end=6.0,
                     x0=0.0, x1=9.0, xs=3.0, gamma=5.0 / 3.0),
}


def shock_tube(name, n, order, **kw):
    d = dict(SHOCK_TUBES[name])
    d.update(kw)
    return riemann_1d(n=n, order=order, name=name, **d)


def blast_wave(n=400, order=9, t_end=0.038, cfl=0.5, nsteps=-1):
    """Interacting blast waves (Sec. 4.4): rho = 1 and u = 0 on [0, 1], p = 1000
    for x < 0.1, 0.01 up to x = 0.9 and 100 beyond; reflective walls at both
    ends; exact cell averages (the jumps fall on faces), zero slopes."""
    dx = 1.0 / n
    xc = (np.arange(n) + 0.5) * dx
    p = np.where(xc < 0.1, 1000.0, np.where(xc < 0.9, 0.01, 100.0))
    rho = np.ones(n)
    avg = _cons(rho, np.zeros(n), None, p, 1.4, 1)
    return {"name": "blast_wave",
            "grid": {"dim": 1, "nx": n, "ny": 1, "x0": 0.0, "x1": 1.0, "y0": 0.0, "y1": 1.0,
                     "bc": ["reflective", "reflective"]},
            "scheme": default_scheme(order, gamma=1.4, tau="inviscid", cfl=cfl),
            "state": {"avg": avg, "sx": np.zeros_like(avg)},
            "run": {"nsteps": nsteps, "dt": 0.0, "t_end": t_end}}


SHOCK_WAVES = {
    # Sec. 4.3: a shock entering a density wave at rest (p = 1, u = 0),
    # rho = 1 + amp sin(k (x - 5)) on [xs, 10]
    "shu_osher": dict(left=(3.857134, 2.629369, 10.33333), xs=1.0, amp=0.2, k=5.0, n=200, t_end=1.8),
    "titarev_toro": dict(left=(1.515695, 0.523346, 1.805), xs=0.5, amp=0.1, k=20.0 * math.pi, n=1000, t_end=5.0),
}


def shock_wave_1d(name, order=9, n=None, t_end=None, cfl=0.5, nsteps=-1):
    """Shock / density-wave interaction of Sec. 4.3 on [0, 10] (the shock
    starts at a face).  Exact cell averages and cell-averaged slopes (the
    difference of face values over dx) of the initial data, zero on the
    constant left side; transmissive ends (the inflow side holds the
    post-shock state, the far side is at rest)."""
    d = SHOCK_WAVES[name]
    n = d["n"] if n is None else n
    t_end = d["t_end"] if t_end is None else t_end
    dx = 10.0 / n
    kf = int(round(d["xs"] / dx))
    xf = np.arange(n + 1) * dx
    amp, k = d["amp"], d["k"]
    rho_f = 1.0 + amp * np.sin(k * (xf - 5.0))
    rho = 1.0 + amp * (np.cos(k * (xf[:-1] - 5.0)) - np.cos(k * (xf[1:] - 5.0))) / (k * dx)
    u = np.zeros(n)
    p = np.ones(n)
    rl, ul, pl = d["left"]
    rho[:kf], u[:kf], p[:kf] = rl, ul, pl
    avg = _cons(rho, u, None, p, 1.4, 1)
    sx = np.zeros_like(avg)
    sx[0, kf:] = (rho_f[kf + 1:] - rho_f[kf:-1]) / dx
    return {"name": name,
            "grid": {"dim": 1, "nx": n, "ny": 1, "x0": 0.0, "x1": 10.0, "y0": 0.0, "y1": 1.0,
                     "bc": ["transmissive", "transmissive"]},
            "scheme": default_scheme(order, gamma=1.4, tau="inviscid", cfl=cfl),
            "state": {"avg": avg, "sx": sx},
            "run": {"nsteps": nsteps, "dt": 0.0, "t_end": t_end}}


def riemann_batch(seed=2, count=4096, nmin=200, nmax=4000, order=9, t_end=0.15, cfl=0.5):
    """Independent 1-D Riemann problems on [0, 1], interface at the face nearest
    x = 0.5, transmissive ends."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    rl = rng.uniform(0.1, 1.0, size=count)
    rr = rng.uniform(0.1, 1.0, size=count)
    pl = 10.0 ** rng.uniform(-2.0, 3.0, size=count)
    pr = 10.0 ** rng.uniform(-2.0, 3.0, size=count)
    ul = rng.uniform(-2.0, 2.0, size=count)
    ur = rng.uniform(-2.0, 2.0, size=count)
    out = []
    for b in range(count):
        n = int(ns[b])
        xs = math.floor(n / 2) / n
        out.append(riemann_1d((rl[b], ul[b], pl[b]), (rr[b], ur[b], pr[b]), n, order, t_end, xs=xs, cfl=cfl,
                              name=f"riemann_batch_s{seed}_{b}"))
    return out


# ---------------------------------------------------------------------------
# 2-D
# ---------------------------------------------------------------------------

def _grid2(nx, ny, x0, x1, y0, y1):
    dx = (x1 - x0) / nx
    dy = (y1 - y0) / ny
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    return dx, dy, xc, yc


def _sin_grid(ax, by, ph):
    """sin(ax[i] + by[j] + ph) on the [j][i] grid, by the angle-addition
    identity (outer products of 1-D arrays instead of n^2 sines)."""
    return np.outer(np.cos(by + ph), np.sin(ax)) + np.outer(np.sin(by + ph), np.cos(ax))


def _cos_grid(ax, by, ph):
    """cos(ax[i] + by[j] + ph) on the [j][i] grid."""
    return np.outer(np.cos(by + ph), np.cos(ax)) - np.outer(np.sin(by + ph), np.sin(ax))


def smooth_2d(modes, n, order, u=1.0, v=1.0, p=1.0, gamma=1.4, L=2.0, nsteps=100, dt=0.0, t_end=0.0,
              name="smooth_2d", **scheme_kw):
    """rho = 1 + sum a sin(pi (kx x + ky y) + phi), constant (u, v, p), periodic
    [0, L]^2 with integer (kx, ky) when L = 2.  W is linear in rho: exact cell
    averages by the product of sinc factors; the line slopes are exact
    differences of face values, sin(w(x+h)) - sin(w(x-h)) = 2 cos(wx) sin(wh)."""
    m = GAUSS_M[order]
    xg, _ = gauss_legendre(m)
    dx, dy, xc, yc = _grid2(n, n, 0.0, L, 0.0, L)
    ravg = np.ones((n, n))
    for a, kx, ky, ph in modes:
        wx, wy = math.pi * kx, math.pi * ky
        ravg += a * _sin_grid(wx * xc, wy * yc, ph) * _sinc(0.5 * wx * dx) * _sinc(0.5 * wy * dy)
    # W = (rho, rho u, rho v, p/(gamma-1) + rho (u^2+v^2)/2) is affine in rho
    dW = np.array([1.0, u, v, 0.5 * (u * u + v * v)])
    one = np.ones_like(ravg)
    avg = _cons(ravg, u * one, v * one, p * one, gamma, 2)
    sx = np.empty((4, m, n, n))
    sy = np.empty((4, m, n, n))
    for l in range(m):
        gx = np.zeros((n, n))
        gy = np.zeros((n, n))
        for a, kx, ky, ph in modes:
            wx, wy = math.pi * kx, math.pi * ky
            gx += (2.0 * a * math.sin(0.5 * wx * dx) / dx) * _cos_grid(wx * xc, wy * (yc + xg[l] * dy), ph)
            gy += (2.0 * a * math.sin(0.5 * wy * dy) / dy) * _cos_grid(wx * (xc + xg[l] * dx), wy * yc, ph)
        sx[:, l] = dW[:, None, None] * gx
        sy[:, l] = dW[:, None, None] * gy
    return {"name": name,
            "grid": {"dim": 2, "nx": n, "ny": n, "x0": 0.0, "x1": L, "y0": 0.0, "y1": L, "bc": ["periodic"] * 4},
            "scheme": default_scheme(order, gamma=gamma, tau="zero", **scheme_kw),
            "state": {"avg": avg, "sx": sx, "sy": sy},
            "run": {"nsteps": nsteps, "dt": dt, "t_end": t_end},
            "modes": modes, "velocity": (u, v)}


def advection_2d(order, n, t_end=2.0, c=0.3):
    """Accuracy test of Sec. 4.6: rho = 1 + 0.2 sin(pi (x + y)), (U, V) = (1, 1),
    p = 1 on [0, 2]^2, periodic, tau = 0, dt = c dx^(r/4)."""
    dx = 2.0 / n
    dt0 = c * dx ** (order / 4.0)
    nsteps = int(math.ceil(t_end / dt0 - 1e-12))
    return smooth_2d([(0.2, 1.0, 1.0, 0.0)], n, order, nsteps=nsteps, dt=t_end / nsteps,
                     name=f"advection_2d_r{order}_n{n}")


def fourier_2d(seed, n, order, nsteps=100, cfl=0.5):
    """2-D analogue of the 1-D Fourier wave: 4 seeded modes, total amplitude
    0.2, (u, v) = (1, 1), p = 1, periodic [0, 2]^2, tau = 0, CFL step."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(-4, 5, size=(4, 2))
    for j in range(4):
        if ks[j, 0] == 0 and ks[j, 1] == 0:
            ks[j, 0] = 1
    w = rng.uniform(0.0, 1.0, size=4)
    a = 0.2 * w / w.sum()
    ph = rng.uniform(0.0, 2.0 * math.pi, size=4)
    modes = [(float(a[j]), float(ks[j, 0]), float(ks[j, 1]), float(ph[j])) for j in range(4)]
    return smooth_2d(modes, n, order, nsteps=nsteps, dt=0.0, cfl=cfl, name=f"fourier_2d_s{seed}_n{n}")


def quadrant_2d(states, n, order, nsteps=200, t_end=0.0, split=(0.5, 0.5), gamma=1.4, tau="inviscid", cfl=0.5,
                bc="transmissive", name="quadrant_2d"):
    """Four-quadrant Riemann data on [0, 1]^2.  states[q] = (rho, u, v, p) for
    q = 0: x<xs,y<ys; 1: x>=xs,y<ys; 2: x>=xs,y>=ys; 3: x<xs,y>=ys.  The split
    sits on the faces nearest (xs, ys); exact averages, zero slopes."""
    m = GAUSS_M[order]
    kx = int(round(split[0] * n))
    ky = int(round(split[1] * n))
    I, J = np.meshgrid(np.arange(n), np.arange(n))
    q = np.where(J < ky, np.where(I < kx, 0, 1), np.where(I < kx, 3, 2))
    S = np.asarray(states, dtype=np.float64)
    rho, u, v, p = (S[q, k] for k in range(4))
    avg = _cons(rho, u, v, p, gamma, 2)
    return {"name": name,
            "grid": {"dim": 2, "nx": n, "ny": n, "x0": 0.0, "x1": 1.0, "y0": 0.0, "y1": 1.0, "bc": [bc] * 4},
            "scheme": default_scheme(order, gamma=gamma, tau=tau, cfl=cfl),
            "state": {"avg": avg, "sx": np.zeros((4, m, n, n)), "sy": np.zeros((4, m, n, n))},
            "run": {"nsteps": nsteps, "dt": 0.0, "t_end": t_end}}


def random_quadrants(seed):
    rng = np.random.default_rng(seed)
    return [(rng.uniform(0.1, 2.0), rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5), rng.uniform(0.03, 1.5))
            for _ in range(4)]


def quadrant_random(seed=3, n=1024, order=7, nsteps=200):
    """Four-quadrant Riemann problem with per-quadrant rho in [0.1, 2], p in
    [0.03, 1.5], velocities in [-1.5, 1.5] drawn from the seed."""
    return quadrant_2d(random_quadrants(seed), n, order, nsteps=nsteps, name=f"quadrant_s{seed}_n{n}")


# Configuration 3 of Sec. 4.7 (the paper's timing workload)
# Sec. 4.7 (a): four rarefaction waves, split at (0.5, 0.5), t = 0.2
CONFIG2 = [(1.0, -0.7259, -0.7259, 1.0), (0.5197, 0.0, -0.7259, 0.4), (1.0, 0.0, 0.0, 1.0), (0.5197, -0.7259, 0.0, 0.4)]
CONFIG3 = [(0.138, 1.206, 1.206, 0.029), (0.5323, 0.0, 1.206, 0.3), (1.5, 0.0, 0.0, 1.5), (0.5323, 1.206, 0.0, 0.3)]


# ---------------------------------------------------------------------------
# Wall, inflow and moving boundaries (Sec. 4.8-4.10).  A side is a name
# ("periodic", "transmissive", "reflective", "noslip"), a prescribed state
# {"type": "inflow", "prim": [rho, u, v, p]}, or {"segments": [...], "ends":
# [[end0, speed], ...]}: segment k holds the ghost cells whose centre (along
# the side: y on x-sides, x on y-sides) lies below end0 + speed * t.
# Discontinuous initial data crossing cells: each cell takes the state at its
# centre; zero slopes.
# ---------------------------------------------------------------------------

def _inflow(prim):
    return {"type": "inflow", "prim": [float(x) for x in prim]}


def _piecewise_2d(nx, ny, x0, x1, y0, y1, region, states, gamma, order, bc, name, t_end, tau, cfl, **scheme_kw):
    """region(X, Y) -> index into states (rho, u, v, p) at the cell centres."""
    m = GAUSS_M[order]
    dx, dy, xc, yc = _grid2(nx, ny, x0, x1, y0, y1)
    X, Y = np.meshgrid(xc, yc)
    q = region(X, Y)
    S = np.asarray(states, dtype=np.float64)
    rho, u, v, p = (S[q, k] for k in range(4))
    avg = _cons(rho, u, v, p, gamma, 2)
    return {"name": name,
            "grid": {"dim": 2, "nx": nx, "ny": ny, "x0": x0, "x1": x1, "y0": y0, "y1": y1, "bc": bc},
            "scheme": default_scheme(order, gamma=gamma, tau=tau, cfl=cfl, **scheme_kw),
            "state": {"avg": avg, "sx": np.zeros((4, m, ny, nx)), "sy": np.zeros((4, m, ny, nx))},
            "run": {"nsteps": -1, "dt": 0.0, "t_end": t_end}}


# Mach 10 shock at 60 degrees to the wall (Sec. 4.8)
DMR_PRE = (1.4, 0.0, 0.0, 1.0)
DMR_POST = (8.0, 8.25 * math.cos(math.pi / 6), -8.25 * math.sin(math.pi / 6), 116.5)


def double_mach(ny=240, order=5, t_end=0.2, cfl=0.5):
    """[0, 4] x [0, 1], 4 ny x ny cells.  The shock meets the bottom at
    x = 1/6 and stands at x = 1/6 + (y + 20 t)/sqrt(3).  Left: post-shock
    inflow; right: transmissive; bottom: post-shock for x < 1/6, reflecting
    wall beyond; top: post-shock behind the exact shock position, pre-shock
    ahead of it (a breakpoint moving at 20/sqrt(3))."""
    r3 = math.sqrt(3.0)
    bc = [_inflow(DMR_POST), "transmissive",
          {"segments": [_inflow(DMR_POST), "reflective"], "ends": [[1.0 / 6.0, 0.0]]},
          {"segments": [_inflow(DMR_POST), _inflow(DMR_PRE)], "ends": [[1.0 / 6.0 + 1.0 / r3, 20.0 / r3]]}]
    region = lambda X, Y: np.where(X < 1.0 / 6.0 + Y / r3, 1, 0)
    return _piecewise_2d(4 * ny, ny, 0.0, 4.0, 0.0, 1.0, region, [DMR_PRE, DMR_POST], 1.4, order, bc,
                         f"double_mach_n{ny}_o{order}", t_end, "inviscid", cfl)


def viscous_shock_tube(nx=500, order=5, t_end=1.0, re=200.0, cfl=0.5):
    """[0, 1] x [0, 0.5], nx x nx/2 cells; a membrane at x = 0.5 separates
    (120, 0, 0, 120/gamma) from (1.2, 0, 0, 1.2/gamma); mu = 1/Re, Pr = 1.
    No-slip adiabatic walls left, right and bottom; symmetry (slip) on top."""
    g = 1.4
    bc = ["noslip", "noslip", "noslip", "reflective"]
    region = lambda X, Y: np.where(X < 0.5, 0, 1)
    return _piecewise_2d(nx, nx // 2, 0.0, 1.0, 0.0, 0.5, region, [(120.0, 0.0, 0.0, 120.0 / g), (1.2, 0.0, 0.0, 1.2 / g)],
                         g, order, bc, f"viscous_shock_tube_n{nx}_o{order}", t_end, "viscous", cfl, mu=1.0 / re,
                         prandtl=1.0)


JETS = {
    # Sec. 4.10: (domain x1, y1), jet band on the left side, jet state, t_end, cells
    80: dict(x1=2.0, y1=1.0, band=(0.45, 0.55), jet=(5.0, 30.0, 0.0, 0.4127), t_end=0.07, nx=448),
    2000: dict(x1=1.0, y1=0.5, band=(0.2, 0.3), jet=(5.0, 800.0, 0.0, 0.4127), t_end=1e-3, nx=800),
}
JET_AMBIENT = (0.5, 0.0, 0.0, 0.4127)


def jet(mach=80, nx=None, order=5, cfl=0.5):
    """Ambient gas (gamma = 5/3) at rest; the left side prescribes the jet
    state inside the band and the ambient state outside it; the other sides
    are outflow (transmissive)."""
    d = JETS[mach]
    nx = nx or d["nx"]
    ny = nx // 2
    bc = [{"segments": [_inflow(JET_AMBIENT), _inflow(d["jet"]), _inflow(JET_AMBIENT)],
           "ends": [[d["band"][0], 0.0], [d["band"][1], 0.0]]}, "transmissive", "transmissive", "transmissive"]
    region = lambda X, Y: np.zeros(X.shape, dtype=int)
    return _piecewise_2d(nx, ny, 0.0, d["x1"], 0.0, d["y1"], region, [JET_AMBIENT], 5.0 / 3.0, order, bc,
                         f"jet_mach{mach}_n{nx}_o{order}", d["t_end"], "inviscid", cfl)


def _spectral_velocity(seed, n, kmax, urms):
    """Solenoidal random-phase field on the unit periodic square: stream
    function modes on integer wavevectors 1 <= |k| <= kmax with shell energy
    E(k) ~ k^(-5/3); returns the Fourier coefficient arrays of u and v."""
    rng = np.random.default_rng(seed)
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    KX, KY = np.meshgrid(k1, k1)  # [j][i]
    K = np.sqrt(KX ** 2 + KY ** 2)
    shell = (K >= 1.0) & (K <= kmax)
    amp = np.zeros_like(K)
    amp[shell] = np.sqrt(K[shell] ** (-5.0 / 3.0) / (2.0 * math.pi * K[shell]))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=K.shape)
    psi_hat = np.zeros_like(K, dtype=np.complex128)
    psi_hat[shell] = amp[shell] / (2.0 * math.pi * K[shell]) * np.exp(1j * phase[shell])
    # real field: Hermitian symmetrisation through the real part of the inverse transform
    uh = 2j * math.pi * KY * psi_hat      # u = d psi / dy
    vh = -2j * math.pi * KX * psi_hat     # v = -d psi / dx
    u0 = np.real(np.fft.ifft2(uh))
    v0 = np.real(np.fft.ifft2(vh))
    s = urms / math.sqrt(np.mean(u0 ** 2 + v0 ** 2))
    return uh * s, vh * s, KX, KY


def _eval_shifted(coef, KX, KY, sx, sy, n):
    """Real part of the Fourier series on the grid shifted by (sx, sy) (units of
    the cell size), sampled at the points (i + sx, j + sy) / n."""
    ph = np.exp(2j * math.pi * (KX * sx + KY * sy) / n)
    return np.real(np.fft.ifft2(coef * ph))


def turbulence_2d(seed=4, n=2048, order=9, nsteps=500, kmax=32, mach=0.3, mu=1e-4, prandtl=0.72, gamma=1.4,
                  cfl=0.2, quad=5):
    """Decaying 2-D turbulence on the periodic unit square: rho = 1, p = 1/gamma
    (sound speed 1), solenoidal velocity with u_rms = Mach.  Cell averages by
    quad x quad Gauss quadrature of the band-limited field, line slopes from
    point values at the face Gauss points.

    CFL 0.2, the paper's number for its viscous case (Sec. 4.9).  At CFL 0.5
    this smooth vortical flow does not stay stable.  With the Prandtl-number
    fix and a collision time of about one step (2048^2 with mu = 1e-4), it
    goes nonphysical near step 200; the oracle breaks down on the same step
    as the GPU path; with Pr 1 the same field runs on.  The paper runs CFL
    0.5 only on problems with shocks, and uses a far smaller step for its
    smooth accuracy tests."""
    m = GAUSS_M[order]
    xg, _ = gauss_legendre(m)
    qx, qw = gauss_legendre(quad)
    uh, vh, KX, KY = _spectral_velocity(seed, n, kmax, mach)
    h = 1.0 / n
    p0 = 1.0 / gamma

    def cons_shift(sx, sy):
        # cell centres sit at (i + 1/2) h: shift by 1/2 + offset
        u = _eval_shifted(uh, KX, KY, 0.5 + sx, 0.5 + sy, n)
        v = _eval_shifted(vh, KX, KY, 0.5 + sx, 0.5 + sy, n)
        one = np.ones_like(u)
        return _cons(one, u, v, p0 * one, gamma, 2)

    avg = np.zeros((4, n, n))
    for a in range(quad):
        for b in range(quad):
            avg += qw[a] * qw[b] * cons_shift(qx[a], qx[b])
    sx = np.zeros((4, m, n, n))
    sy = np.zeros((4, m, n, n))
    for l in range(m):
        sx[:, l] = (cons_shift(0.5, xg[l]) - cons_shift(-0.5, xg[l])) / h
        sy[:, l] = (cons_shift(xg[l], 0.5) - cons_shift(xg[l], -0.5)) / h
    return {"name": f"turbulence_s{seed}_n{n}",
            "grid": {"dim": 2, "nx": n, "ny": n, "x0": 0.0, "x1": 1.0, "y0": 0.0, "y1": 1.0, "bc": ["periodic"] * 4},
            "scheme": default_scheme(order, gamma=gamma, tau="viscous", mu=mu, prandtl=prandtl, cfl=cfl),
            "state": {"avg": avg, "sx": sx, "sy": sy},
            "run": {"nsteps": nsteps, "dt": 0.0, "t_end": 0.0}}


def serving_trace(seed=5, count=200, rate=None, nmin_log2=7.0, nmax_log2=11.0, steps=(50, 500)):
    """Job descriptions for the serving mix: Poisson arrivals, side
    round(2^U[7, 11]), order from {5, 7, 9}, smooth or four-quadrant data,
    50-500 steps.  Returns a list of dicts (arrival time, side, order, kind,
    data seed, steps); the problem itself is built by ``serving_problem``."""
    rng = np.random.default_rng(seed)
    rate = 1.0 if rate is None else rate
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for k in range(count):
        out.append({"id": k, "arrival": float(t[k]),
                    "n": int(round(2.0 ** rng.uniform(nmin_log2, nmax_log2))),
                    "order": int(rng.choice([5, 7, 9])),
                    "kind": "smooth" if rng.uniform() < 0.5 else "riemann",
                    "seed": int(rng.integers(0, 2 ** 31 - 1)),
                    "nsteps": int(rng.integers(steps[0], steps[1] + 1))})
    return out


def serving_problem(job):
    if job["kind"] == "smooth":
        return fourier_2d(job["seed"], job["n"], job["order"], nsteps=job["nsteps"])
    return quadrant_2d(random_quadrants(job["seed"]), job["n"], job["order"], nsteps=job["nsteps"],
                       name=f"quadrant_s{job['seed']}_n{job['n']}")
