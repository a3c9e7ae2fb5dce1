"""Auto and cross power spectrum estimators (Sec. 3, Eqs. (cps) and (ccc), Delta^2(k)), FP64.

Test infrastructure only (see ``oracle/__init__``).

Particles are CIC-assigned to the fine mesh, delta = rho/<rho> - 1, and
P(k) = (L^3 / N_m^6) |delta_k|^2 for the unnormalised DFT delta_k = sum_x delta(x) e^{-ikx}.
Readings (the paper is silent on the estimator): shells b = nint(|n|) for b = 1 .. N_m/2 with
n the integer wavevector; in the half-spectrum layout (last axis halved) modes with n_x = 0 or
n_x = N_m/2 count once and every other mode twice (its conjugate partner); the shell reports
the weighted mean |k|, the weighted mean P and the mode count. No CIC deconvolution and no
shot-noise subtraction by default.

Cross power P_ab (Eq. (cps) with two fields): (L^3 / (N_a^3 N_b^3)) Re(conj(delta_a,k) delta_b,k)
over the same shells, and the cross-correlation coefficient xi = P_ab / sqrt(P_aa P_bb)
(Eq. (ccc)). Reading for two meshes of different sizes over the same box: only the modes both
meshes hold unaliased enter, i.e. every signed component |n_i| < N_min/2 (the Nyquist planes of
the smaller mesh are dropped), shells 1 .. N_min/2; two meshes of one size use every mode, as
the auto spectrum does.

Pins (tests/test_oracle_power.py): a single cosine mode puts all its power in one shell with
the analytic amplitude; white noise gives a flat spectrum L^3/N at every shell within its
Gaussian scatter; the mode counts of all shells add up to the number of distinct modes
with |n| < N/2 + 1/2; xi of a field with itself is 1 and with its negative -1; two cosines
of one wavevector shifted by a phase theta give xi = cos(theta); independent noise fields give
xi within the Gaussian scatter of 0; a field sampled on a mesh of twice the size has the same
cross power with itself over the common modes.
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


def _signed(nm):
    """Signed integer frequency of each index (fftfreq times nm is not exact for every size)."""
    return np.rint(np.fft.fftfreq(nm) * nm).astype(np.int64)


def cross_spectrum(delta_a, delta_b, box: float):
    """(k_mean [h/Mpc], P_aa, P_bb, P_ab [(Mpc/h)^3], n_modes) for shells 1 .. N_min/2.

    delta_a and delta_b are cubic meshes over the same box, of sizes N_a and N_b."""
    na, nb_ = delta_a.shape[0], delta_b.shape[0]
    n = min(na, nb_)
    fa = np.fft.rfftn(delta_a)
    fb = np.fft.rfftn(delta_b)
    if na == nb_:
        b, nmag, w = shell_index(n)
        keep = np.ones(b.shape, dtype=bool)
        ca, cb = fa, fb
    else:
        # the modes with every |n_i| < N/2 of the smaller mesh, picked out of both spectra
        fz = _signed(n)
        fx = np.arange(n // 2 + 1)
        keep = (np.abs(fz)[:, None, None] < n / 2) & (np.abs(fz)[None, :, None] < n / 2) & \
            (fx[None, None, :] < n / 2)

        def take(f, m):
            iz = fz % m
            return f[np.ix_(iz, iz, fx)]

        ca, cb = take(fa, na), take(fb, nb_)
        n2 = fz[:, None, None] ** 2 + fz[None, :, None] ** 2 + fx[None, None, :] ** 2
        nmag = np.sqrt(n2)
        b = np.floor(nmag + 0.5).astype(np.int64)
        w = np.where(fx[None, None, :] == 0, 1.0, 2.0) * np.ones(n2.shape)
    nsh = n // 2
    sel = keep & (b >= 1) & (b <= nsh)
    bb, ww = b[sel], w[sel]
    sa, sb = ca[sel], cb[sel]
    va, vb = box**3 / float(na) ** 6, box**3 / float(nb_) ** 6
    vab = box**3 / (float(na) ** 3 * float(nb_) ** 3)

    def shells(x):
        return np.bincount(bb, weights=ww * x, minlength=nsh + 1)[1:]

    nmodes = shells(np.ones(bb.shape))
    ksum = shells(nmag[sel])
    paa = shells(va * (sa.real**2 + sa.imag**2))
    pbb = shells(vb * (sb.real**2 + sb.imag**2))
    pab = shells(vab * (sa.real * sb.real + sa.imag * sb.imag))
    kf = 2.0 * np.pi / box
    with np.errstate(invalid="ignore", divide="ignore"):
        return kf * ksum / nmodes, paa / nmodes, pbb / nmodes, pab / nmodes, nmodes


def correlation(paa, pbb, pab):
    """xi(k) = P_ab / sqrt(P_aa P_bb) (Eq. (ccc))."""
    with np.errstate(invalid="ignore", divide="ignore"):
        return pab / np.sqrt(paa * pbb)


def dimensionless(k, pk):
    """Delta^2(k) = k^3 P(k) / (2 pi^2)."""
    return k**3 * pk / (2.0 * np.pi**2)
