"""Pins of three parts of the oracle that the paper fixes only in part: the
linear weights of the AO(5,3) reconstruction (Eq. 3.12, which as printed do
not sum to one; reading A3), the WENO-Z weights built on the global
indicator tau_Z (Eq. 3.14-3.16, reading A4) and the CFL time step (Sec. 4,
reading A19).

Each pin checks a property the paper or the mathematics fixes, chosen so that
a plausible slip fails it:
  - mirror symmetry: reflecting the data x -> -x must reflect the
    reconstruction and the whole solution (an asymmetric weight, a swapped
    sub-stencil or index fails it);
  - the ENO property: at an isolated jump the nonlinear weights select the
    one sub-stencil that does not cross it;
  - a worked example on linear data, where every intermediate quantity of
    Eq. 3.12-3.17 has a closed form (a wrong tau_Z scale, a wrong share of
    the linear weights or indicators taken from the unscaled members fail it);
  - the time step of uniform and two-state data against the formula of
    Sec. 4 evaluated from the primitive states (|U| + |V| in place of
    sqrt(U^2 + V^2), the wrong grid spacing or the wrong density in the
    viscous bound fail it).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2508_13705_amd import workloads as W


def _mirror_data(q, hq, sig):
    """x -> -x: cell k <-> cell -k, derivative averages change sign; face f
    (left face of cell f, at x_{f-1/2}) <-> face 1 - f."""
    return q[::-1].copy(), -hq[::-1].copy(), sig[::-1].copy()


def _mirror_poly(c):
    """p(xi) -> p(-xi)"""
    return np.array([c[j] * (-1) ** j for j in range(9)])


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("flags", [0, 2])
def test_ao_reconstruction_is_mirror_symmetric(seed, flags):
    """Reconstructing mirrored data gives the mirrored polynomial (Eq. 3.11-3.17,
    3.19 with the AO branch taken).  The sub-stencils S0 = {i-1, i} and
    S1 = {i, i+1} are mirror images of each other, so their linear weights
    must be equal; the central S2 and the fifth-order member map to
    themselves.  Indicators of the unscaled members (an alternative reading)
    keep the symmetry; gamma_1 taking the gamma_Lo share (the other) breaks
    it, test_gamma1_reading_is_not_mirror_symmetric."""
    rng = np.random.default_rng(100 + seed)
    sch = dict(W.default_scheme(5), reading_flags=flags)
    q = rng.normal(size=5)
    hq = rng.normal(size=5)
    sig = rng.uniform(0.0, 0.8, size=6)
    sig[2] += 0.6   # A(r5) > 1: the AO branch
    c, br = oracle.recon_poly(sch, q, hq, sig)
    assert br == 0
    cm, brm = oracle.recon_poly(sch, *_mirror_data(q, hq, sig))
    assert brm == 0
    scale = np.abs(c).max()
    assert np.abs(cm - _mirror_poly(c)).max() <= 1e-13 * scale, (cm, _mirror_poly(c))


def test_gamma1_reading_is_not_mirror_symmetric():
    """With gamma_1 = (1 - gamma_Hi) gamma_Lo (the printed form of Eq. 3.12
    completed to sum to one) the mirror images S0 and S1 carry different
    linear weights, so mirrored data no longer give the mirrored polynomial:
    the reason the default reading gives the gamma_Lo share to S2."""
    rng = np.random.default_rng(100)
    sch = dict(W.default_scheme(5), reading_flags=1)
    worst = 0.0
    for _ in range(6):
        q, hq = rng.normal(size=5), rng.normal(size=5)
        sig = rng.uniform(0.0, 0.8, size=6)
        sig[2] += 0.6
        c, br = oracle.recon_poly(sch, q, hq, sig)
        cm, _ = oracle.recon_poly(sch, *_mirror_data(q, hq, sig))
        assert br == 0
        worst = max(worst, np.abs(cm - _mirror_poly(c)).max() / np.abs(c).max())
    assert worst > 1e-3


def _riemann(left, right, n, order, nsteps):
    pb = W.riemann_1d(left, right, n, order, t_end=0.0, nsteps=nsteps)
    pb["run"] = {"nsteps": nsteps, "dt": 0.0, "t_end": 0.0}
    return pb


@pytest.mark.parametrize("order", [5, 9])
def test_riemann_problem_is_mirror_symmetric(order):
    """A 1-D Riemann problem and its mirror image (states swapped, velocities
    negated, on the domain reflected about its centre) give mirrored
    solutions, cell by cell, with the AO branch active: rho and rho E even,
    rho u odd; the cell-averaged slopes the other way round."""
    n, steps = 60, 24
    L, R = (1.0, 0.75, 1.0), (0.125, -0.3, 0.1)
    r = oracle.run(_riemann(L, R, n, order, steps))
    rm = oracle.run(_riemann((R[0], -R[1], R[2]), (L[0], -L[1], L[2]), n, order, steps))
    assert r["status"] == rm["status"] == 0
    assert r["stats"]["ao"] > 0
    assert abs(r["t"] - rm["t"]) <= 1e-15 * r["t"]
    par = np.array([1.0, -1.0, 1.0])[:, None]
    mir_avg = par * rm["avg"][:, ::-1]
    mir_sx = -par * rm["sx"][:, ::-1]
    scale = np.abs(r["avg"]).max(axis=1, keepdims=True)
    assert np.all(np.abs(r["avg"] - mir_avg) <= 1e-12 * scale)
    sscale = np.abs(r["sx"]).max(axis=1, keepdims=True)
    assert np.all(np.abs(r["sx"] - mir_sx) <= 1e-10 * sscale)


def _jump_data(k, a, J, jump_right):
    """Cell averages and h-scaled derivative averages (xi units) of
    a sin(k xi) plus a jump of height J at the face +1/2 (jump_right) or
    -1/2 of the reconstructed cell; inside every cell the data are smooth."""
    F = lambda x: -a * np.cos(k * x) / k       # antiderivative of the smooth part
    f = lambda x: a * np.sin(k * x)
    js = np.arange(-2, 3)
    q = np.array([F(j + 0.5) - F(j - 0.5) for j in js])
    hq = np.array([f(j + 0.5) - f(j - 0.5) for j in js])
    q = q + J * ((js >= 1) if jump_right else (js >= 0))
    return q, hq


@pytest.mark.parametrize("jump_right", [True, False])
def test_ao_weights_pick_the_smooth_substencil_at_a_jump(jump_right):
    """ENO property of the WENO-Z weights (Eq. 3.14-3.17): with a jump beside
    the cell, the only sub-stencil that does not cross it (S0 for a jump at
    the right face, S1 for a jump at the left face) takes almost all of the
    weight, so the face value tends to that member's DFF-scaled value
    (Eq. 3.19) as the smooth side gets smoother."""
    sch = W.default_scheme(5)
    sig = np.zeros(6)
    sig[3 if jump_right else 2] = 2.0     # the strength of the jump face
    member = "S0" if jump_right else "S1"
    # DFF of the member: A = eta sigma over its faces (A7): S0 has the
    # right face with eta 1, S1 the left face with eta 1
    alpha = oracle.dff(member, sig, 1.0)
    assert alpha == pytest.approx(0.5)
    devs = []
    for k in (0.4, 0.2, 0.1):
        q, hq = _jump_data(k, 0.1, 1.0, jump_right)
        c, br = oracle.recon_poly(sch, q, hq, sig)
        assert br == 0
        pm = oracle.stencil_fit(member, q, hq)
        want = q[2] + alpha * (oracle.poly_eval(pm, 0.5) - q[2])
        devs.append(abs(oracle.poly_eval(c, 0.5) - want))
        # the fifth-order member alone is far off (it crosses the jump)
        p5 = oracle.stencil_fit("R5", q, hq)
        assert abs(oracle.poly_eval(p5, 0.5) - oracle.poly_eval(pm, 0.5)) > 0.05
    assert devs[0] < 1e-2
    assert devs[0] > devs[1] > devs[2]
    assert devs[2] < 1e-4


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_weno_z_weights_worked_example(flags):
    """Linear data q_j = j, h Q_x = 1 (the cell's polynomial is xi for every
    member, by polynomial exactness), with the strength 0.6 on the face +3/2
    only.  Then, by Eq. 3.3-3.4 with the face weights of A7:
      A(S0) = 0, A(S1) = 2 * 0.6, A(S2) = 0.6, A(r5) = 2 * 0.6, so
      alpha = (1, 5/6, 1, 5/6) and the scaled members are alpha_k xi (Eq. 3.19);
      beta_k = alpha_k^2 (the indicator of a linear member is its slope squared),
      = (1, 25/36, 1, 25/36);
      tau_Z = (|b3 - b0| + |b3 - b1| + |b3 - b2|) / 3 = (2 * 11/36) / 3 = 11/54 (Eq. 3.15);
      gamma = (0.03, 0.03, 0.09, 0.85) for gamma_Hi = 0.85, gamma_Lo = 0.6 (Eq. 3.12, A3);
      omega_k = gamma_k (1 + tau_Z^2 / (beta_k + eps)^2), normalised (Eq. 3.14, 3.16);
    and the AO polynomial (Eq. 3.17) is s xi with
      s = w3 / g3 (alpha_3 - sum_{k<3} g_k alpha_k) + sum_{k<3} w_k alpha_k.
    The alternative readings change one input each: gamma_1 taking the
    gamma_Lo share gives gamma = (0.03, 0.09, 0.03, 0.85); indicators of the
    unscaled members are all 1, so tau_Z = 0, the weights stay linear and
    s = alpha_3 = 5/6 whatever the linear weights."""
    sch = dict(W.default_scheme(5), reading_flags=flags)
    q = np.arange(-2, 3, dtype=np.float64)
    hq = np.ones(5)
    sig = np.zeros(6)
    sig[4] = 0.6
    alpha = [1.0, 5.0 / 6.0, 1.0, 5.0 / 6.0]
    for name, a in zip(("S0", "S1", "S2", "R5"), alpha):
        assert oracle.dff(name, sig, 1.0) == pytest.approx(a, rel=1e-15)
    beta = [a * a for a in alpha]
    tau_z = 11.0 / 54.0
    assert tau_z == pytest.approx((abs(beta[3] - beta[0]) + abs(beta[3] - beta[1]) + abs(beta[3] - beta[2])) / 3.0)
    eps = sch["weno_eps"]

    def slope(g, tz, b):
        om = [g[k] * (1.0 + tz ** 2 / (b[k] + eps) ** 2) for k in range(4)]
        w = [o / sum(om) for o in om]
        return w[3] / g[3] * (alpha[3] - sum(g[k] * alpha[k] for k in range(3))) + \
            sum(w[k] * alpha[k] for k in range(3))

    g = [0.03, 0.09, 0.03, 0.85] if flags & 1 else [0.03, 0.03, 0.09, 0.85]
    s = 5.0 / 6.0 if flags & 2 else slope(g, tau_z, beta)
    c, br = oracle.recon_poly(sch, q, hq, sig)
    assert br == 0
    assert abs(c[0]) < 1e-15 and np.abs(c[2:]).max() < 1e-14
    assert c[1] == pytest.approx(s, rel=1e-14, abs=0.0)
    if flags:
        return
    g = [0.03, 0.03, 0.09, 0.85]
    # the example tells the reading apart from plausible slips, each of which
    # moves the slope by far more than the tolerance above: tau_Z without its
    # 1/3; S2 taking the (1 - gamma_Lo) share; indicators of the unscaled
    # members (all 1, so tau_Z = 0 and the weights stay linear: slope 5/6)
    for alt in (slope(g, 3.0 * tau_z, beta), slope([0.045, 0.045, 0.06, 0.85], tau_z, beta), 5.0 / 6.0):
        assert abs(alt - s) > 1e-5


def _uniform_2d(prim, nx, ny, order, x1=1.0, y1=1.0, tau="inviscid", mu=0.0, cfl=0.5):
    reg = lambda X, Y: np.zeros(X.shape, dtype=int)
    return W._piecewise_2d(nx, ny, 0.0, x1, 0.0, y1, reg, [prim], 1.4, order, ["periodic"] * 4, "uniform2d", 0.0,
                           tau, cfl, mu=mu)


def _first_dt(pb):
    r = oracle.run(pb, nsteps=1, t_end=0.0)
    assert r["status"] == 0 and r["stats"]["steps"] == 1
    return r["t"]


def _speed(prim, gamma=1.4):
    rho, u, v, p = prim
    return math.hypot(u, v) + math.sqrt(gamma * p / rho)


def test_cfl_dt_uniform_diagonal_flow():
    """dt = CFL dx / (||U|| + a_s) (Sec. 4) with ||U|| the magnitude of the
    velocity: a diagonal flow tells sqrt(U^2 + V^2) apart from |U| + |V|."""
    prim = (1.2, 0.8, -0.6, 0.9)
    pb = _uniform_2d(prim, 8, 8, 5, cfl=0.5)
    dx = 1.0 / 8
    assert _first_dt(pb) == pytest.approx(0.5 * dx / _speed(prim), rel=1e-15)


def test_cfl_dt_uses_the_smaller_spacing():
    """On a grid with dy < dx the step is set by the smaller spacing (A19)."""
    prim = (1.0, 0.3, 0.4, 1.0)
    pb = _uniform_2d(prim, 8, 10, 5, x1=1.0, y1=0.5, cfl=0.4)
    dy = 0.5 / 10
    assert _first_dt(pb) == pytest.approx(0.4 * dy / _speed(prim), rel=1e-15)


def test_cfl_dt_two_states_and_viscous_bound():
    """Quadrants with different states: the largest signal speed sets the
    inviscid bound; the viscous bound dx^2 / (4 nu) with nu = mu / rho is
    set by the smallest density (Sec. 4), both times the CFL number."""
    fast = (1.5, 1.0, 1.0, 1.0)        # largest ||U|| + a_s
    light = (0.25, 0.0, 0.0, 0.05)     # smallest rho, slow
    states = [fast, light, fast, light]
    n = 10
    dx = 1.0 / n
    s_max = max(_speed(fast), _speed(light))
    for mu, cfl in ((1e-4, 0.5), (2e-2, 0.3)):
        pb = W.quadrant_2d(states, n, 5, nsteps=1, tau="viscous", cfl=cfl, bc="periodic")
        pb["scheme"]["mu"] = mu
        want = cfl * min(dx / s_max, dx * dx * 0.25 / (4.0 * mu))
        assert _first_dt(pb) == pytest.approx(want, rel=1e-15), mu
    # the second case is bound by the viscous limit, the first by the inviscid one
    assert dx * dx * 0.25 / (4.0 * 2e-2) < dx / s_max < dx * dx * 0.25 / (4.0 * 1e-4)
