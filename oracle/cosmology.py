"""Background cosmology, linear growth and linear power spectrum (FP64, scipy quadrature).

Test infrastructure only (see ``oracle/__init__``).

Units: H0 = 1. Time-integration factors are dimensionless integrals over the scale factor.
Wavenumbers for the power spectrum are in h/Mpc and lengths in Mpc/h.

Pins (tests/test_oracle_cosmology.py):
* E, D, f, kick and drift factors reduce to the Einstein-de Sitter closed forms
  (D = a, f = 1, K = 2 a^{1/2}, Delta = -2 a^{-1/2}).
* LCDM growth D(a) is checked against an independent ODE integration of the growth equation.
* sigma_8 normalisation reproduces sigma(8 Mpc/h) = sigma_8 by a separate integration.
* BBKS transfer function: T -> 1 as k -> 0 and the large-q asymptote ln(2.34q)/(2.34q)*(6.71q)^-1.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

_QUAD = dict(epsabs=0.0, epsrel=1e-12, limit=400)


def _quad_lnk(fun, lnk_min=math.log(1e-6), lnk_max=math.log(300.0), pieces=200):
    """Integral over ln k split into pieces (the top-hat window oscillates at high k)."""
    edges = np.linspace(lnk_min, lnk_max, pieces + 1)
    return sum(integrate.quad(fun, lo, hi, epsabs=1e-300, epsrel=1e-11, limit=500)[0]
               for lo, hi in zip(edges[:-1], edges[1:]))


class Cosmology:
    """Flat or curved matter + Lambda background with H0 = 1 (Sec. 2.2 uses a, H, D, f)."""

    def __init__(self, omega_m: float, omega_l: float | None = None, h: float = 0.7,
                 sigma8: float = 0.8, n_s: float = 1.0):
        self.omega_m = float(omega_m)
        self.omega_l = float(1.0 - omega_m if omega_l is None else omega_l)
        self.omega_k = 1.0 - self.omega_m - self.omega_l
        self.h = float(h)
        self.sigma8 = float(sigma8)
        self.n_s = float(n_s)
        self._d_norm = self._growth_unnormalised(1.0)
        self._amp = None

    # ---- background -------------------------------------------------------------------
    def E(self, a):
        """Dimensionless Hubble rate H(a)/H0."""
        a = np.asarray(a, dtype=np.float64)
        return np.sqrt(self.omega_m / a**3 + self.omega_k / a**2 + self.omega_l)

    # ---- linear growth (growing mode of a pressureless fluid with Lambda) -------------
    def _growth_unnormalised(self, a: float) -> float:
        # D(a) proportional to E(a) * int_0^a da' / (a' E(a'))^3  (valid for matter + Lambda + curvature)
        val, _ = integrate.quad(lambda x: 1.0 / (x * float(self.E(x)))**3, 0.0, a, **_QUAD)
        return float(self.E(a)) * val

    def D(self, a: float) -> float:
        """Linear growth factor, normalised to D(1) = 1."""
        return self._growth_unnormalised(a) / self._d_norm

    def f(self, a: float) -> float:
        """Growth rate f = d ln D / d ln a, from the derivative of the integral form of D."""
        E = float(self.E(a))
        integral, _ = integrate.quad(lambda x: 1.0 / (x * float(self.E(x)))**3, 0.0, a, **_QUAD)
        dlnE = -(3.0 * self.omega_m / a**3 + 2.0 * self.omega_k / a**2) / (2.0 * E * E)
        return dlnE + 1.0 / (a * a * E**3 * integral)

    # ---- leapfrog factors (Sec. 2.3.3 "timestep": DKKD operator splitting) -------------
    def kick_factor(self, a0: float, a1: float) -> float:
        """K = int_{a0}^{a1} da / (a^2 E): dp = -grad(phi) K for the momentum p = a^2 dx/dt."""
        val, _ = integrate.quad(lambda x: 1.0 / (x * x * float(self.E(x))), a0, a1, **_QUAD)
        return val

    def drift_factor(self, a0: float, a1: float) -> float:
        """Delta = int_{a0}^{a1} da / (a^3 E): dx = p Delta."""
        val, _ = integrate.quad(lambda x: 1.0 / (x**3 * float(self.E(x))), a0, a1, **_QUAD)
        return val

    # ---- linear power spectrum ----------------------------------------------------------
    def transfer_bbks(self, k):
        """BBKS (Bardeen, Bond, Kaiser & Szalay 1986) transfer function, shape Gamma = Omega_m h,
        k in h/Mpc; no baryon correction."""
        k = np.asarray(k, dtype=np.float64)
        q = k / (self.omega_m * self.h)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (np.log1p(2.34 * q) / (2.34 * q)
                 * (1.0 + 3.89 * q + (16.1 * q)**2 + (5.46 * q)**3 + (6.71 * q)**4) ** -0.25)
        return np.where(q > 0, t, 1.0)

    def _pk_shape(self, k):
        k = np.asarray(k, dtype=np.float64)
        return k**self.n_s * self.transfer_bbks(k) ** 2

    @staticmethod
    def tophat(x):
        """Fourier transform of a real-space spherical top-hat, W(x) = 3 (sin x - x cos x) / x^3."""
        x = np.asarray(x, dtype=np.float64)
        small = np.abs(x) < 1e-3
        xs = np.where(small, 1.0, x)
        w = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs**3
        return np.where(small, 1.0 - x * x / 10.0, w)

    def _sigma2_shape(self, r: float) -> float:
        # sigma^2(r) = 1/(2 pi^2) int k^2 P(k) W^2(kr) dk, integrated in ln k
        def integrand(lnk):
            k = math.exp(lnk)
            return k**3 * float(self._pk_shape(k)) * float(self.tophat(k * r)) ** 2
        return _quad_lnk(integrand) / (2.0 * math.pi**2)

    @property
    def amplitude(self) -> float:
        """A in P(k) = A k^n_s T^2(k), fixed by sigma(8 Mpc/h) = sigma_8 at a = 1."""
        if self._amp is None:
            self._amp = self.sigma8**2 / self._sigma2_shape(8.0)
        return self._amp

    def pk_linear(self, k, a: float = 1.0):
        """Linear matter power spectrum at scale factor a, (Mpc/h)^3, k in h/Mpc."""
        return self.amplitude * self._pk_shape(k) * self.D(a) ** 2

    def sigma_r(self, r: float, a: float = 1.0) -> float:
        return math.sqrt(self.amplitude * self._sigma2_shape(r)) * self.D(a)

    # ---- velocity dispersion model, Eqs. (vdisp), (vdelta) ----------------------------
    def sigma_v2(self, a: float, r: float) -> float:
        """Eq. (vdisp): (a H f D)^2 int d^3k/(2pi)^3 P(k)/k^2 W^2(kr), in (100 km/s)^2 with
        H = 100 h km/s/Mpc * E(a) (so the result is in units of (100 km/s)^2).
        Reading: the 1/(2 pi)^3 of the usual convention is taken although the printed equation
        omits it. r = 0 means no smoothing."""
        pref = (a * float(self.E(a)) * self.f(a) * self.D(a)) ** 2

        def integrand(lnk):
            k = math.exp(lnk)
            w = 1.0 if r == 0 else float(self.tophat(k * r))
            return k * float(self._pk_shape(k)) * w * w  # k^3 * P/k^2 * W^2, d ln k
        return pref * self.amplitude * _quad_lnk(integrand) / (2.0 * math.pi**2)

    def sigma_delta2(self, a: float, r_c: float, r_p: float) -> float:
        """Eq. (vdelta), 3-D variance of the velocity relative to the coarse-cell mean.
        Reading: the printed difference has its operands swapped (smoothing on the smaller
        particle scale r_p keeps more power, so sigma_v^2(r_p) > sigma_v^2(r_c)); the
        non-negative difference sigma_v^2(r_p) - sigma_v^2(r_c) is returned."""
        return self.sigma_v2(a, r_p) - self.sigma_v2(a, r_c)


def schedule(a_init: float, a_final: float, n_steps: int, spacing: int = 0):
    """Integer-step scale factors a_0..a_n and half-step a_{j+1/2} (geometric mean).

    spacing 0: uniform in ln a (default); 1: uniform in a.
    The DKD leapfrog keeps positions at half steps and momenta at integer steps (Sec. 2.3.3).
    """
    j = np.arange(n_steps + 1, dtype=np.float64)
    if spacing == 0:
        a = a_init * (a_final / a_init) ** (j / n_steps)
    else:
        a = a_init + (a_final - a_init) * j / n_steps
    a[0], a[-1] = a_init, a_final
    ah = np.sqrt(a[:-1] * a[1:])
    return a, ah


def step_factors(cosmo: Cosmology, a_init: float, a_final: float, n_steps: int, spacing: int = 0):
    """Per-step (kick, drift) factors of the DKD scheme with merged drifts.

    Returns (drift0, kicks, drifts): the initial half drift a_0 -> a_1/2, then for step j the
    kick a_j -> a_{j+1} (force evaluated at a_{j+1/2}) and the drift a_{j+1/2} -> a_{j+3/2}
    (the last one stops at a_n, completing the final half drift at the checkpoint)."""
    a, ah = schedule(a_init, a_final, n_steps, spacing)
    drift0 = cosmo.drift_factor(a[0], ah[0])
    kicks = [cosmo.kick_factor(a[j], a[j + 1]) for j in range(n_steps)]
    drifts = [cosmo.drift_factor(ah[j], ah[j + 1]) for j in range(n_steps - 1)]
    drifts.append(cosmo.drift_factor(ah[-1], a[-1]))
    return drift0, np.array(kicks), np.array(drifts)
