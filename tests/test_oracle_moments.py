"""Pins of the oracle's Maxwellian moments and micro-coefficient solves
(Sec. 2.1, Eq. 2.2, 2.3, 2.8) against direct numerical quadrature."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


def _gauss_pdf(u, U, lam):
    return math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2)


@pytest.mark.parametrize("U,lam", [(0.0, 0.5), (0.7, 2.0), (-1.3, 0.35), (2.5, 7.0), (-0.05, 30.0)])
def test_u_moments_match_quadrature(U, lam):
    full = oracle.u_moments(U, lam, 0, 7)
    pos = oracle.u_moments(U, lam, +1, 7)
    neg = oracle.u_moments(U, lam, -1, 7)
    for n in range(8):
        f = lambda u: u ** n * _gauss_pdf(u, U, lam)
        qf = integrate.quad(f, -np.inf, np.inf, epsabs=0, epsrel=1e-13)[0]
        qp = integrate.quad(f, 0, np.inf, epsabs=0, epsrel=1e-13)[0]
        qn = integrate.quad(f, -np.inf, 0, epsabs=0, epsrel=1e-13)[0]
        scale = integrate.quad(lambda u: abs(u) ** n * _gauss_pdf(u, U, lam), -np.inf, np.inf)[0]
        assert abs(full[n] - qf) <= 1e-12 * scale
        assert abs(pos[n] - qp) <= 1e-12 * scale
        assert abs(neg[n] - qn) <= 1e-12 * scale
        assert abs(pos[n] + neg[n] - full[n]) <= 1e-13 * scale


@pytest.mark.parametrize("K", [1, 2, 3])
def test_xi_moments_match_product_quadrature(K):
    """<(xi^2)^c> for K internal degrees of freedom, each a Gaussian of
    variance 1/(2 lam): multinomial expansion over the K one-dimensional
    moments computed by quadrature."""
    lam = 0.8
    m1 = [integrate.quad(lambda x: x ** (2 * k) * _gauss_pdf(x, 0.0, lam), -np.inf, np.inf)[0] for k in range(4)]
    got = oracle.xi_moments(float(K), lam, 3)
    import itertools
    for c in range(4):
        s = 0.0
        for ks in itertools.product(range(c + 1), repeat=K):
            if sum(ks) != c:
                continue
            coef = math.factorial(c)
            prod = 1.0
            for k in ks:
                coef //= math.factorial(k)
                prod *= m1[k]
            s += coef * prod
        assert abs(got[c] - s) <= 1e-12 * s


@pytest.mark.parametrize("dim", [1, 2])
def test_conservative_moments_and_energy(dim):
    """int psi g = W: the internal degrees of freedom K = 2/(gamma-1) - D make
    the energy moment equal rho E = p/(gamma-1) + rho |U|^2 / 2 (A13)."""
    gamma = 1.4
    rho, u, v, p = 0.8, 0.3, -0.6, 1.7
    if dim == 1:
        W = np.array([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u])
    else:
        W = np.array([rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)])
    got = oracle.psi_moment(dim, W, gamma, 0, 0, 0)
    assert np.allclose(got, W, rtol=1e-14, atol=0)
    # flux moments int u psi g: the Euler flux
    F = oracle.psi_moment(dim, W, gamma, 1, 0, 0)
    if dim == 1:
        Fe = [rho * u, rho * u * u + p, u * (W[2] + p)]
    else:
        Fe = [rho * u, rho * u * u + p, rho * u * v, u * (W[3] + p)]
    assert np.allclose(F, Fe, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("dim", [1, 2])
def test_micro_solve_residual_by_quadrature(dim):
    """<a psi> = b (Eq. 2.8): check the solved coefficients by integrating
    psi * a * g with quadrature in u (and v), using the pinned xi moments."""
    gamma = 1.4
    rng = np.random.default_rng(11)
    rho, u, v, p = 1.3, -0.4, 0.9, 0.6
    K = 2.0 / (gamma - 1.0) - dim
    lam = rho / (2 * p)
    if dim == 1:
        W = np.array([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u])
    else:
        W = np.array([rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)])
    b = rng.normal(size=dim + 2)
    a = oracle.micro_solve(dim, W, gamma, b)
    x1, x2 = K / (2 * lam), K * (K + 2) / (4 * lam * lam)
    if dim == 1:
        def psi_a(uu):
            # returns the vector int psi a g over xi, as a function of u
            e = 0.5 * (uu * uu)
            aval0 = a[0] + a[1] * uu + a[2] * e            # a without xi part
            # a = a0 + a1 u + a2 (u^2 + xi^2)/2 ; psi = (1, u, (u^2+xi^2)/2)
            r0 = aval0 + a[2] * 0.5 * x1
            r2 = 0.5 * (uu * uu * r0 + aval0 * x1 + a[2] * 0.5 * x2)
            return np.array([r0, uu * r0, r2]) * rho * _gauss_pdf(uu, u, lam)
        got = np.array([integrate.quad(lambda s: psi_a(s)[k], -np.inf, np.inf, epsrel=1e-13)[0] for k in range(3)])
    else:
        def integrand(k, vv, uu):
            e = 0.5 * (uu * uu + vv * vv)
            a0 = a[0] + a[1] * uu + a[2] * vv + a[3] * e
            r0 = a0 + a[3] * 0.5 * x1
            vals = [r0, uu * r0, vv * r0, e * r0 + 0.5 * (a0 * x1 + a[3] * 0.5 * x2)]
            return vals[k] * rho * _gauss_pdf(uu, u, lam) * _gauss_pdf(vv, v, lam)
        got = np.array([integrate.dblquad(lambda vv, uu: integrand(k, vv, uu), u - 12 / math.sqrt(lam),
                                          u + 12 / math.sqrt(lam), v - 12 / math.sqrt(lam), v + 12 / math.sqrt(lam),
                                          epsabs=1e-13, epsrel=1e-12)[0] for k in range(4)])
    assert np.allclose(got, b, rtol=1e-9, atol=1e-10)
