"""Pins of the oracle's gas-kinetic interface flux (Eq. 2.6-2.8, 2.11, 2.12,
2.15) against closed forms: free stream, the Euler flux and its
Cauchy-Kovalevskaya time derivative, compatibility W(0) = Q0, mirror symmetry
and the discontinuity strength of Eq. 3.2."""
import numpy as np
import pytest

import oracle

GAMMA = 1.4


def cons1(rho, u, p, g=GAMMA):
    return np.array([rho, rho * u, p / (g - 1) + 0.5 * rho * u * u])


def cons2(rho, u, v, p, g=GAMMA):
    return np.array([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])


def euler_flux(W, dim, g=GAMMA):
    rho = W[0]
    u = W[1] / rho
    if dim == 1:
        p = (g - 1) * (W[2] - 0.5 * rho * u * u)
        return np.array([rho * u, rho * u * u + p, u * (W[2] + p)])
    v = W[2] / rho
    p = (g - 1) * (W[3] - 0.5 * rho * (u * u + v * v))
    return np.array([rho * u, rho * u * u + p, rho * u * v, u * (W[3] + p)])


def euler_flux_y(W, g=GAMMA):
    rho, u, v = W[0], W[1] / W[0], W[2] / W[0]
    p = (g - 1) * (W[3] - 0.5 * rho * (u * u + v * v))
    return np.array([rho * v, rho * u * v, rho * v * v + p, v * (W[3] + p)])


def jacobian(f, W):
    """Complex-step Jacobian (exact to rounding)."""
    n = len(W)
    J = np.zeros((n, n))
    h = 1e-30
    for k in range(n):
        Wc = W.astype(np.complex128)
        Wc[k] += 1j * h
        J[:, k] = np.imag(f(Wc)) / h
    return J


SCHEMES = [dict(tau="zero"), dict(tau="inviscid", c1=0.05, c2=1.0), dict(tau="viscous", mu=1e-3, c2=1.0)]


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dim", [1, 2])
def test_free_stream(scheme, dim):
    W = cons1(0.7, 0.4, 1.3) if dim == 1 else cons2(0.7, 0.4, -0.9, 1.3)
    Wk = np.zeros((6, dim + 2))
    Wk[0] = W
    dt = 0.01
    r = oracle.flux_point(scheme, dim, Wk, Wk, dt)
    F = euler_flux(W, dim)
    assert np.allclose(r["Fh"], 0.5 * dt * F, rtol=1e-13, atol=1e-16)
    assert np.allclose(r["F1"], dt * F, rtol=1e-13, atol=1e-16)
    for k in ("W0", "Wh", "W1"):
        assert np.allclose(r[k], W, rtol=1e-13, atol=1e-15)
    assert r["sigma"] == 0.0


@pytest.mark.parametrize("scheme", SCHEMES)
def test_initial_interface_value_is_kinetic_equilibrium(scheme):
    """W(0) = Q0 = int_{u>0} psi g^l + int_{u<0} psi g^r for any tau."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        Wl = cons2(*rng.uniform([0.2, -1, -1, 0.1], [2, 1, 1, 3]))
        Wr = cons2(*rng.uniform([0.2, -1, -1, 0.1], [2, 1, 1, 3]))
        A = np.zeros((6, 4)); B = np.zeros((6, 4))
        A[0], B[0] = Wl, Wr
        A[1:] = rng.normal(scale=0.3, size=(5, 4)); B[1:] = rng.normal(scale=0.3, size=(5, 4))
        r = oracle.flux_point(scheme, 2, A, B, 0.02)
        Q0 = oracle.psi_moment(2, Wl, GAMMA, 0, 0, +1) + oracle.psi_moment(2, Wr, GAMMA, 0, 0, -1)
        assert np.allclose(r["W0"], Q0, rtol=1e-12, atol=1e-13)


def test_smooth_tau0_flux_is_euler_cauchy_kovalevskaya_1d():
    """tau = 0 with one smooth state on both sides: the flux integral is
    F delta + F_t delta^2 / 2 with F_t = A W_t, W_t = -A W_x (A the Euler
    Jacobian), and the interface value moves with W_t."""
    W = cons1(1.1, 0.35, 0.9)
    Wx = np.array([0.3, -0.2, 0.5])
    Wxx = np.array([0.1, 0.4, -0.3])
    Wk = np.zeros((6, 3)); Wk[0], Wk[1], Wk[3] = W, Wx, Wxx
    A = jacobian(lambda w: euler_flux(w, 1), W)
    Wt = -A @ Wx
    Ft = A @ Wt
    F = euler_flux(W, 1)
    for dt in (1e-2, 3e-3):
        r = oracle.flux_point(dict(tau="zero"), 1, Wk, Wk, dt)
        assert np.allclose(r["F1"], F * dt + 0.5 * Ft * dt * dt, rtol=1e-12, atol=1e-15)
        assert np.allclose(r["Fh"], F * dt / 2 + 0.125 * Ft * dt * dt, rtol=1e-12, atol=1e-15)
        Wt_fit = (4 * r["Wh"] - 3 * r["W0"] - r["W1"]) / dt
        assert np.allclose(Wt_fit, Wt, rtol=1e-9, atol=1e-11)
        assert np.allclose(r["W0"], W, rtol=1e-14)


def test_smooth_tau0_flux_is_euler_cauchy_kovalevskaya_2d():
    W = cons2(0.9, -0.25, 0.6, 1.2)
    Wx = np.array([0.2, -0.1, 0.3, 0.4])
    Wy = np.array([-0.15, 0.25, 0.05, -0.2])
    Wk = np.zeros((6, 4)); Wk[0], Wk[1], Wk[2] = W, Wx, Wy
    Wk[3:] = np.array([[0.1, 0.2, -0.1, 0.05], [0.02, -0.3, 0.1, 0.2], [-0.1, 0.05, 0.2, 0.1]])
    A = jacobian(lambda w: euler_flux(w, 2), W)
    B = jacobian(euler_flux_y, W)
    Wt = -(A @ Wx + B @ Wy)
    Ft = A @ Wt
    F = euler_flux(W, 2)
    dt = 5e-3
    r = oracle.flux_point(dict(tau="zero"), 2, Wk, Wk, dt)
    assert np.allclose(r["F1"], F * dt + 0.5 * Ft * dt * dt, rtol=1e-12, atol=1e-15)
    Wt_fit = (4 * r["Wh"] - 3 * r["W0"] - r["W1"]) / dt
    assert np.allclose(Wt_fit, Wt, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_mirror_symmetry(scheme):
    """x -> -x: the mirrored left/right pair (normal momentum and odd
    derivatives negated) gives the mirrored flux; this also pins the use of
    a^r (not a^l) for u < 0 (A14)."""
    rng = np.random.default_rng(5)
    M = np.array([1, -1, 1, 1.0])          # parity of (rho, rho u_n, rho u_t, rho E)
    D = np.array([1, -1, 1, 1, -1, 1.0])   # parity of (value, d_n, d_t, d_nn, d_nt, d_tt)
    for _ in range(4):
        Wl = np.zeros((6, 4)); Wr = np.zeros((6, 4))
        Wl[0] = cons2(*rng.uniform([0.3, -1, -1, 0.2], [2, 1, 1, 2]))
        Wr[0] = cons2(*rng.uniform([0.3, -1, -1, 0.2], [2, 1, 1, 2]))
        Wl[1:] = rng.normal(scale=0.3, size=(5, 4)); Wr[1:] = rng.normal(scale=0.3, size=(5, 4))
        r = oracle.flux_point(scheme, 2, Wl, Wr, 0.01)
        ml = (D[:, None] * M[None, :]) * Wr
        mr = (D[:, None] * M[None, :]) * Wl
        s = oracle.flux_point(scheme, 2, ml, mr, 0.01)
        for k in ("Fh", "F1"):
            assert np.allclose(s[k], -M * r[k], rtol=1e-11, atol=1e-14)
        for k in ("W0", "Wh", "W1"):
            assert np.allclose(s[k], M * r[k], rtol=1e-11, atol=1e-14)
        assert abs(s["sigma"] - r["sigma"]) <= 1e-13 * r["sigma"]


def test_tau_limit_is_continuous():
    rng = np.random.default_rng(9)
    Wl = np.zeros((6, 4)); Wr = np.zeros((6, 4))
    Wl[0] = cons2(1.0, 0.2, 0.1, 1.0); Wr[0] = cons2(0.9, 0.25, 0.05, 0.95)
    Wl[1:] = rng.normal(scale=0.1, size=(5, 4)); Wr[1:] = rng.normal(scale=0.1, size=(5, 4))
    a = oracle.flux_point(dict(tau="zero"), 2, Wl, Wr, 0.01)
    b = oracle.flux_point(dict(tau="inviscid", c1=1e-9, c2=0.0), 2, Wl, Wr, 0.01)
    assert np.allclose(a["F1"], b["F1"], rtol=1e-8, atol=1e-12)
    assert np.allclose(a["W1"], b["W1"], rtol=1e-8, atol=1e-12)


def test_sigma_formula():
    """Eq. 3.2 on a hand-computed pair (1-D: no tangential Mach number)."""
    g = GAMMA
    Wl = np.zeros((6, 3)); Wr = np.zeros((6, 3))
    Wl[0] = cons1(1.0, 0.5, 1.0); Wr[0] = cons1(0.5, -0.2, 0.25)
    cl, cr = np.sqrt(g * 1.0 / 1.0), np.sqrt(g * 0.25 / 0.5)
    expect = 0.75 / 1.0 + 0.75 / 0.25 + (0.5 / cl + 0.2 / cr) ** 2
    r = oracle.flux_point(dict(tau="zero"), 1, Wl, Wr, 0.01)
    assert abs(r["sigma"] - expect) <= 1e-14 * expect


def test_tau_models():
    g = GAMMA
    Wl = np.zeros((6, 3)); Wr = np.zeros((6, 3))
    Wl[0] = cons1(1.0, 0.0, 1.0); Wr[0] = cons1(0.5, 0.0, 0.5)
    dt = 0.02
    r = oracle.flux_point(dict(tau="inviscid", c1=0.05, c2=1.0), 1, Wl, Wr, dt)
    assert abs(r["tau"] - (0.05 * dt + (0.5 / 1.5) * dt)) < 1e-15
    r = oracle.flux_point(dict(tau="zero"), 1, Wl, Wr, dt)
    assert r["tau"] == 0.0


def test_prandtl_fix_invariants():
    """Prandtl fix of the energy flux (not in the paper; its rate is pinned in
    test_oracle_prandtl.py):
    no effect at Pr = 1 or in a uniform state, only the energy flux changes,
    and the change is proportional to (1/Pr - 1)."""
    rng = np.random.default_rng(4)
    Wl = np.zeros((6, 4)); Wr = np.zeros((6, 4))
    Wl[0] = cons2(1.0, 0.2, 0.1, 0.7); Wr[0] = cons2(1.02, 0.21, 0.09, 0.71)
    Wl[1:] = rng.normal(scale=0.2, size=(5, 4)); Wr[1:] = rng.normal(scale=0.2, size=(5, 4))
    base = dict(tau="viscous", mu=1e-3, c2=1.0)
    a = oracle.flux_point(dict(base, prandtl=1.0), 2, Wl, Wr, 0.01)
    b = oracle.flux_point(dict(base, prandtl=0.72), 2, Wl, Wr, 0.01)
    c = oracle.flux_point(dict(base, prandtl=0.5), 2, Wl, Wr, 0.01)
    assert np.array_equal(a["F1"][:3], b["F1"][:3]) and np.array_equal(a["W1"], b["W1"])
    db, dc = b["F1"][3] - a["F1"][3], c["F1"][3] - a["F1"][3]
    assert db != 0.0
    assert abs(db / dc - (1 / 0.72 - 1) / (1 / 0.5 - 1)) < 1e-9
    U = np.zeros((6, 4)); U[0] = Wl[0]
    u1 = oracle.flux_point(dict(base, prandtl=1.0), 2, U, U, 0.01)
    u2 = oracle.flux_point(dict(base, prandtl=0.72), 2, U, U, 0.01)
    assert abs(u2["F1"][3] - u1["F1"][3]) < 1e-15
