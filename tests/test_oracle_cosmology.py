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


def _gaussian_spectrum(c, k0):
    """Replace the BBKS shape by P(k) = exp(-(k/k0)^2) with unit amplitude (closed-form integrals)."""
    c._pk_shape = lambda k: np.exp(-(np.asarray(k, dtype=np.float64) / k0) ** 2)
    c._amp = 1.0
    return c


def test_velocity_dispersion_closed_forms():
    """Eq. (vdisp) with P(k) = exp(-(k/k0)^2): without smoothing the integral of d^3k/(2 pi)^3 P/k^2
    is k0 sqrt(pi) / (4 pi^2) (over the oracle's range 1e-6 < k < 300 h/Mpc: times the difference of
    the error functions at the ends); the top-hat's expansion W^2 = 1 - x^2/5 + 3 x^4/175 gives the
    small-r change from the moments of P; the prefactor (a H f D)^2 is a in Einstein-de Sitter."""
    k0 = 0.8
    c = _gaussian_spectrum(Cosmology(1.0, 0.0), k0)
    s0 = c.sigma_v2(1.0, 0.0)
    span = math.erf(300.0 / k0) - math.erf(1e-6 / k0)
    assert s0 == pytest.approx(k0 * math.sqrt(math.pi) / (4.0 * math.pi**2) * span, rel=1e-9)
    for a in (0.02, 0.3):
        assert c.sigma_v2(a, 0.0) == pytest.approx(a * s0, rel=1e-7)
    r = 0.05 / k0
    m2 = math.sqrt(math.pi) * k0**3 / 4.0   # int k^2 P dk
    m4 = 3.0 * math.sqrt(math.pi) * k0**5 / 8.0  # int k^4 P dk
    drop = (r * r / 5.0 * m2 - 3.0 * r**4 / 175.0 * m4) / (2.0 * math.pi**2)
    assert s0 - c.sigma_v2(1.0, r) == pytest.approx(drop, rel=1e-5)
    # LCDM prefactor against its factors
    cl = _gaussian_spectrum(Cosmology(0.3, 0.7), k0)
    a = 0.5
    pref = (a * float(cl.E(a)) * cl.f(a) * cl.D(a)) ** 2
    assert cl.sigma_v2(a, 0.0) == pytest.approx(pref * s0, rel=1e-7)


def test_velocity_dispersion_difference_by_lattice_mode_sum():
    """Eq. (vdelta) as a sum over the modes of a periodic box (a 3-D lattice in k, no quadrature in
    ln k): (1/V) sum_k P/k^2 (W^2(k r_p) - W^2(k r_c)) with the BBKS spectrum."""
    c = Cosmology(0.3, 0.7)
    rp, rc = 1.5, 6.0
    L, n = 200.0, 192
    f = 2.0 * math.pi * np.fft.fftfreq(n, d=L / n)
    kx, ky, kz = np.meshgrid(f, f, f, indexing="ij", sparse=True)
    k = np.sqrt(kx**2 + ky**2 + kz**2)
    k = np.where(k == 0, 1.0, k)
    w = c.tophat(k * rp) ** 2 - c.tophat(k * rc) ** 2
    p = c.pk_linear(k, 1.0)
    s = (p / k**2 * w)
    s[0, 0, 0] = 0.0
    lattice = s.sum() / L**3
    model = c.sigma_delta2(1.0, rc, rp) / (float(c.E(1.0)) * c.f(1.0) * c.D(1.0)) ** 2
    assert model == pytest.approx(lattice, rel=2e-3)


@pytest.mark.parametrize("name", ["c1_pm32", "c2_pm128"])
def test_velocity_dispersion_model_matches_measured_ic(name):
    """The measured rms velocity about the coarse-cell mean of the initial conditions agrees with
    Eq. (vdelta) within a factor 1.5 (the paper reports good agreement, Sec. 2.2); the smoothing
    radii are those of spheres with a coarse cell's and a particle's volume. Measured ratios:
    C1 1.36, C2 1.27."""
    import synth
    from oracle import ic
    cfg = synth.WORKLOADS[name]
    c = Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])
    nm, npart, nc, L, a = cfg["nm_side"], cfg["np_side"], cfg["nc_side"], cfg["box"], cfg["a_init"]
    x, p, _ = ic.zeldovich(npart, nm, L, c, a, cfg["seed"])
    cell = np.floor(x / (nm // nc)).astype(np.int64) % nc
    cid = cell[:, 0] + nc * (cell[:, 1] + nc * cell[:, 2])
    cnt = np.bincount(cid, minlength=nc**3)
    mean = np.stack([np.bincount(cid, weights=p[:, d], minlength=nc**3) for d in range(3)]) / np.maximum(cnt, 1)
    dp2 = ((p - mean[:, cid].T) ** 2).sum(axis=1).mean()
    # p = a^2 dx/dt in fine cells x H0: peculiar velocity p / a, one fine cell x H0 = (L / nm) 100 km/s
    measured = dp2 / a**2 * (L / nm) ** 2
    sphere = (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
    model = c.sigma_delta2(a, sphere * L / nc, sphere * L / npart)
    assert 1.0 / 1.5 < measured / model < 1.5, measured / model
