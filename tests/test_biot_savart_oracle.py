"""Pins of the oracle's Biot-Savart sum (Sec. 3.4 eq. nsode with the regularised
kernel K_eps of Sec. 5):

* Lamb-Oseen closed form: particles on a lattice carrying Gamma_i = omega(x_i) h^2
  of a Lamb-Oseen vortex (spread 4 nu t) induce, with the Gaussian-regularised
  kernel, the velocity of a Lamb-Oseen vortex of spread 4 nu t + eps^2 (the
  smoothing is a Gaussian convolution; the lattice sum of a smooth Gaussian
  integrand is exact to far below 1e-10 at eps = 3h);
* the kernel is odd (Sec. 3.4): sum_i Gamma_i u_i = 0, and with K(r).r = 0 also
  sum_i Gamma_i u_i . x_i = 0, for any cloud;
* K_eps(0) = 0: a lone particle does not move itself.
"""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("h", [0.04, 0.02])
def test_lattice_lamb_oseen_gives_the_smoothed_closed_form(orc, h):
    x, y = workloads.lattice(-1.0, 1.0, h)
    nu, t, G = 0.01, 1.0, 1.0
    g = workloads.lamb_oseen_omega(x, y, t, nu, G) * h * h
    eps = 3.0 * h
    sel = np.random.default_rng(1).choice(x.size, 400, replace=False)
    u, v = orc.biot_savart(x, y, g, eps, x[sel], y[sel])
    r2 = x[sel] ** 2 + y[sel] ** 2
    w = G / (2.0 * np.pi * r2) * (-np.expm1(-r2 / (4.0 * nu * t + eps * eps)))
    ue, ve = -y[sel] * w, x[sel] * w
    scale = np.abs(np.concatenate([ue, ve])).max()
    assert np.abs(u - ue).max() <= 1e-10 * scale
    assert np.abs(v - ve).max() <= 1e-10 * scale


def test_oddness_gives_zero_momentum_sums(orc):
    rng = np.random.default_rng(7)
    n = 2000
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    g = rng.normal(0, 1, n)
    u, v = orc.biot_savart(x, y, g, 0.05)
    scale = np.sum(np.abs(g) * (np.abs(u) + np.abs(v)))
    assert abs(np.sum(g * u)) <= 1e-12 * scale
    assert abs(np.sum(g * v)) <= 1e-12 * scale
    assert abs(np.sum(g * (u * x + v * y))) <= 1e-12 * np.sum(np.abs(g) * (np.abs(u * x) + np.abs(v * y)))


def test_lone_particle_does_not_move_itself(orc):
    u, v = orc.biot_savart(np.array([0.3]), np.array([-0.2]), np.array([2.0]), 0.1)
    assert u[0] == 0.0 and v[0] == 0.0
