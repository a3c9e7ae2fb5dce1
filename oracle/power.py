"""Auto power spectrum estimator (Sec. 3, Eq. (cps) and Delta^2(k)), FP64.

Test infrastructure only (see ``oracle/__init__``).

Particles are CIC-assigned to the fine mesh, delta = rho/<rho> - 1, and
P(k) = (L^3 / N_m^6) |delta_k|^2 for the unnormalised DFT delta_k = sum_x delta(x) e^{-ikx}.
Readings (the paper is silent on the estimator): shells b = nint(|n|) for b = 1 .. N_m/2 with
n the integer wavevector; in the half-spectrum layout (last axis halved) modes with n_x = 0 or
n_x = N_m/2 count once and every other mode twice (its conjugate partner); the shell reports
the weighted mean |k|, the weighted mean P and the mode count. No CIC deconvolution and no
shot-noise subtraction by default.

Pins (tests/test_oracle_power.py): a single cosine mode puts all its power in one shell with
the analytic amplitude; white noise gives a flat spectrum L^3/N at every shell within its
Gaussian scatter; the mode counts of all shells add up to the number of distinct modes
with |n| < N/2 + 1/2.
"""
from __future__ import annotations

import numpy as np


def shell_index(nm: int):
    """Integer |n| shell of every mode in the rfftn layout [z, y, x//2+1] and its weight."""
    nf = np.fft.fftfreq(nm) * nm
    nr = np.fft.rfftfreq(nm) * nm
    n2 = nf[:, None, None] ** 2 + nf[None, :, None] ** 2 + nr[None, None, :] ** 2
    nmag = np.sqrt(n2)
    b = np.floor(nmag + 0.5).astype(np.int64)
    w = np.full(n2.shape, 2.0)
    w[:, :, 0] = 1.0
    if nm % 2 == 0:
        w[:, :, -1] = 1.0
    return b, nmag, w


def power_spectrum(delta, box: float):
    """(k_mean [h/Mpc], P [(Mpc/h)^3], n_modes) for shells 1 .. N/2."""
    nm = delta.shape[0]
    dk = np.fft.rfftn(delta)
    p = (box**3 / float(nm) ** 6) * (dk.real**2 + dk.imag**2)
    b, nmag, w = shell_index(nm)
    nb = nm // 2
    sel = (b >= 1) & (b <= nb)
    bb = b[sel]
    ww = w[sel]
    nmodes = np.bincount(bb, weights=ww, minlength=nb + 1)[1:]
    ksum = np.bincount(bb, weights=ww * nmag[sel], minlength=nb + 1)[1:]
    psum = np.bincount(bb, weights=ww * p[sel], minlength=nb + 1)[1:]
    kf = 2.0 * np.pi / box
    with np.errstate(invalid="ignore", divide="ignore"):
        return kf * ksum / nmodes, psum / nmodes, nmodes


def dimensionless(k, pk):
    """Delta^2(k) = k^3 P(k) / (2 pi^2)."""
    return k**3 * pk / (2.0 * np.pi**2)
