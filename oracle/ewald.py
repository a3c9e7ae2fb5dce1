"""Periodic direct-sum (Ewald) forces for a handful of particles, FP64.

Test infrastructure only (see ``oracle/__init__``).

Used to pin the PM force law of oracle.pm. A unit point mass with a neutralising background in
a periodic cube of side L (lap(phi) = 4 pi (delta_D - 1/L^3)) produces the Ewald acceleration
(Hernquist, Bouchet & Suto 1991)
  a(x) = - sum_n (x - nL)/r_n^3 [erfc(alpha r_n) + 2 alpha r_n / sqrt(pi) exp(-alpha^2 r_n^2)]
         - (4 pi / L^3) sum_{k != 0} k / k^2 exp(-k^2 / (4 alpha^2)) sin(k . x),
with k = 2 pi h / L. In the oracle's units (lap(phi) = 3/2 Omega_m delta, lengths in cells,
delta = rho/<rho> - 1 with N particles of unit mass) each particle carries the coupling
G_eff = 3/2 Omega_m L^3 / (4 pi N).

Pins (tests/test_oracle_pm.py): the sum tends to the bare 1/r^2 law at r << L and is odd in x.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc


def ewald_unit_accel(dx, box: float, alpha: float | None = None, nreal: int = 4, nk: int = 6):
    """Acceleration at offset dx (3,) from a unit mass, periodic box of side `box`."""
    dx = np.asarray(dx, dtype=np.float64)
    a = 2.0 / box if alpha is None else alpha
    acc = np.zeros(3)
    rng = np.arange(-nreal, nreal + 1)
    n = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3) * box
    r = dx[None, :] - n
    rn = np.sqrt((r * r).sum(1))
    ok = rn > 0
    r, rn = r[ok], rn[ok]
    fac = (erfc(a * rn) + 2.0 * a * rn / math.sqrt(math.pi) * np.exp(-(a * rn) ** 2)) / rn**3
    acc -= (r * fac[:, None]).sum(0)
    hr = np.arange(-nk, nk + 1)
    h = np.stack(np.meshgrid(hr, hr, hr, indexing="ij"), -1).reshape(-1, 3)
    h = h[(h != 0).any(1)]
    k = 2.0 * math.pi * h / box
    k2 = (k * k).sum(1)
    kfac = np.exp(-k2 / (4.0 * a * a)) / k2 * np.sin(k @ dx)
    acc -= 4.0 * math.pi / box**3 * (k * kfac[:, None]).sum(0)
    return acc


def ewald_accel(x, box: float, omega_m: float):
    """Accelerations (N,3) of N unit-mass particles in the oracle's PM units."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    geff = 1.5 * omega_m * box**3 / (4.0 * math.pi * n)
    out = np.zeros_like(x)
    for i in range(n):
        for j in range(n):
            if i != j:
                out[i] += geff * ewald_unit_accel(x[i] - x[j], box)
    return out
