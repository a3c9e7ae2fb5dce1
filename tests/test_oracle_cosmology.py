"""Pins of oracle.cosmology: closed forms (EdS), an independent growth ODE, sigma_8."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.cosmology import Cosmology, schedule, step_factors


def test_eds_closed_forms():
    c = Cosmology(1.0, 0.0)
    for a in (0.02, 0.1, 0.5, 1.0):
        assert c.D(a) == pytest.approx(a, rel=1e-10)
        assert c.f(a) == pytest.approx(1.0, rel=1e-9)
        assert float(c.E(a)) == pytest.approx(a**-1.5, rel=1e-14)
    a0, a1 = 0.02, 0.37
    assert c.kick_factor(a0, a1) == pytest.approx(2 * (a1**0.5 - a0**0.5), rel=1e-11)
    assert c.drift_factor(a0, a1) == pytest.approx(-2 * (a1**-0.5 - a0**-0.5), rel=1e-11)


def test_lcdm_growth_matches_ode():
    c = Cosmology(0.3, 0.7)
    # growth ODE in ln a: D'' + (2 + dlnE/dlna) D' - 1.5 Om / (a^3 E^2) D = 0, growing mode D ~ a early
    def rhs(lna, y):
        a = math.exp(lna)
        E2 = 0.3 / a**3 + 0.7
        dlnE = -1.5 * 0.3 / a**3 / E2
        return [y[1], -(2.0 + dlnE) * y[1] + 1.5 * 0.3 / (a**3 * E2) * y[0]]
    a_start = 1e-4
    sol = integrate.solve_ivp(rhs, (math.log(a_start), 0.0), [a_start, a_start], rtol=1e-11, atol=1e-16,
                              dense_output=True)
    d1 = sol.sol(0.0)[0]
    for a in (0.02, 0.1, 0.5, 0.8):
        y = sol.sol(math.log(a))
        assert c.D(a) == pytest.approx(y[0] / d1, rel=2e-6)
        assert c.f(a) == pytest.approx(y[1] / y[0], rel=2e-5)


def test_sigma8_normalisation_independent_integral():
    c = Cosmology(0.3, 0.7, h=0.7, sigma8=0.8)
    # integrate in k (not ln k) with a different rule
    k = np.logspace(-5, 2.5, 200001)
    integrand = k**2 * c.pk_linear(k) * c.tophat(8.0 * k) ** 2
    s2 = np.trapezoid(integrand, k) / (2 * math.pi**2)
    assert math.sqrt(s2) == pytest.approx(0.8, rel=1e-4)


def test_bbks_limits():
    c = Cosmology(0.3, 0.7, h=0.7)
    assert float(c.transfer_bbks(1e-7)) == pytest.approx(1.0, abs=1e-5)
    q = 1e5
    k = q * 0.3 * 0.7
    asym = math.log(2.34 * q) / (2.34 * q) / (6.71 * q)
    assert float(c.transfer_bbks(k)) == pytest.approx(asym, rel=1e-3)


def test_schedule_and_factors_cover_interval():
    c = Cosmology(1.0, 0.0)
    a, ah = schedule(0.02, 1.0, 50)
    assert a[0] == 0.02 and a[-1] == 1.0
    assert np.allclose(np.diff(np.log(a)), math.log(50.0) / 50)
    d0, kicks, drifts = step_factors(c, 0.02, 1.0, 50)
    # drifts chain a_0 -> a_1/2 -> ... -> a_n: their sum is the full drift integral
    assert d0 + drifts.sum() == pytest.approx(c.drift_factor(0.02, 1.0), rel=1e-10)
    assert kicks.sum() == pytest.approx(c.kick_factor(0.02, 1.0), rel=1e-10)


def test_velocity_dispersion_model_positive_and_ordered():
    c = Cosmology(0.3, 0.7)
    s0 = c.sigma_v2(1.0, 0.0)
    s8 = c.sigma_v2(1.0, 8.0)
    assert s0 > s8 > 0
    # linear-theory rms 3-D velocity today is a few hundred km/s for sigma_8 = 0.8
    assert 2.0 < math.sqrt(s0) < 8.0  # units of 100 km/s
    assert c.sigma_delta2(1.0, 8.0, 2.0) > 0
