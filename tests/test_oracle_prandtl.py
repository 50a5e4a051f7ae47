"""Pin of the oracle's Prandtl-number fix (reading A18) by Fourier heat
conduction: an entropy wave (density perturbation at rest, uniform pressure)
decays at the thermal diffusivity times k^2, nu k^2 / Pr for the BGK model
with the heat flux scaled to Prandtl number Pr.  The ratio of the decay rates
at Pr = 0.72 and Pr = 1 must be 1/Pr, whatever the scheme's own dissipation:
without the fix it is 1, with the correction's sign reversed it is below 1,
and with 1/Pr in place of 1/Pr - 1 it is about 2.4.  Collision time 0.15 of
the time step (the continuum regime the fix is meant for)."""
import math

import numpy as np

import oracle
from paper_2508_13705_amd import workloads as W


def _rate(prandtl, n=32, mu=2e-3, t_end=5.0):
    pb = W.smooth_1d([(0.01, 2.0, 0.0)], n, 5, u=0.0, p=1.0, x0=0.0, x1=1.0)
    pb["scheme"].update(tau="viscous", mu=mu, prandtl=prandtl, cfl=0.5)
    x = (np.arange(n) + 0.5) / n
    amp = lambda r: abs(np.sum((r - 1.0) * np.exp(-2j * math.pi * x))) * 2 / n
    r = oracle.run(pb, nsteps=-1, t_end=t_end)
    assert r["status"] == 0 and abs(r["t"] - t_end) < 1e-12
    return -math.log(amp(r["avg"][0]) / amp(pb["state"]["avg"][0])) / r["t"]


def test_entropy_wave_decay_scales_with_one_over_prandtl():
    k2 = (2 * math.pi) ** 2
    r1, r72 = _rate(1.0), _rate(0.72)
    assert abs(r1 / (2e-3 * k2) - 1.0) < 0.03          # nu k^2 at Pr = 1 (measured 1.4% above)
    assert abs((r72 / r1) * 0.72 - 1.0) < 0.01         # measured 0.4% below 1/Pr
