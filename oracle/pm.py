"""Plain FP64 particle-mesh N-body step on uncompressed particles.

Test infrastructure only (see ``oracle/__init__``).

This is the result CUBE's compressed step approximates (Sec. 2.3.3, Figs. code, update_xp,
update_vp; single-level PM, no PP force as in Sec. 3). Units: lengths in fine-mesh cells,
H0 = 1, momentum p = a^2 dx/dt.

Equations of motion (comoving): dx/da = p / (a^3 E), dp/da = -grad(phi) / (a^2 E) with
lap(phi) = (3/2) Omega_m delta. The leapfrog is DKD with merged drifts, i.e. the paper's
(DKKD)^n with the final half drift done at the checkpoint.

Readings (the paper defers the force kernels to CUBEP3M):
* CIC with cell centres at i + 1/2: i0 = floor(u - 1/2), d = u - 1/2 - i0, weights 1 - d, d;
  the same weights for deposit and interpolation.
* Green's function G(k) = -(3/2) Omega_m / |k|^2 with k_i = 2 pi n_i / N_m, G(0) = 0.
* Force = -grad(phi) by the 4-point central difference
  (8 (phi[i+1] - phi[i-1]) - (phi[i+2] - phi[i-2])) / 12 on the mesh, then CIC-interpolated.

Pins (tests/test_oracle_pm.py): single-particle CIC weights; mass conservation; momentum
conservation to 1e-12; plane-wave potential and the closed-form FD transfer function
(8 sin k - sin 2k)/6; the periodic direct sum (oracle.ewald) at separations > 4 cells; the exact
1-D Zel'dovich solution before shell crossing (oracle.zeldovich).
"""
from __future__ import annotations

import numpy as np

from .cosmology import Cosmology, step_factors


def cic_weights(x, nm: int):
    """Lower corner index (wrapped) and upper weight per dimension for positions x (N,3)."""
    u = np.asarray(x, dtype=np.float64) - 0.5
    i0 = np.floor(u)
    d = u - i0
    i0 = np.mod(i0.astype(np.int64), nm)
    return i0, d


def cic_deposit(x, nm: int, mass=None):
    """CIC mass assignment; returns rho[z, y, x] in particle-mass units."""
    i0, d = cic_weights(x, nm)
    n = len(i0)
    m = np.ones(n) if mass is None else np.asarray(mass, np.float64)
    rho = np.zeros(nm**3, dtype=np.float64)
    for cz in (0, 1):
        wz = d[:, 2] if cz else 1.0 - d[:, 2]
        iz = (i0[:, 2] + cz) % nm
        for cy in (0, 1):
            wy = d[:, 1] if cy else 1.0 - d[:, 1]
            iy = (i0[:, 1] + cy) % nm
            for cx in (0, 1):
                wx = d[:, 0] if cx else 1.0 - d[:, 0]
                ix = (i0[:, 0] + cx) % nm
                rho += np.bincount(ix + nm * (iy + nm * iz), weights=m * wx * wy * wz, minlength=nm**3)
    return rho.reshape(nm, nm, nm)


def density_contrast(rho, n_particles: int):
    """delta = rho / <rho> - 1 (Sec. 3)."""
    nm3 = rho.size
    return rho * (nm3 / n_particles) - 1.0


def kvectors(nm: int):
    """Angular wavenumbers (rad per cell) of the rfftn layout [z, y, x//2+1]."""
    k = 2.0 * np.pi * np.fft.fftfreq(nm)
    kr = 2.0 * np.pi * np.fft.rfftfreq(nm)
    return k[:, None, None], k[None, :, None], kr[None, None, :]


def green_function(nm: int, omega_m: float):
    kz, ky, kx = kvectors(nm)
    k2 = kx**2 + ky**2 + kz**2
    with np.errstate(divide="ignore"):
        g = -1.5 * omega_m / k2
    g[0, 0, 0] = 0.0
    return g


# Threads of the FFT: None uses numpy.fft (one thread; the stored golden spectra were made so); a
# number uses scipy.fft with that many threads (the host timing of the benchmark). The two differ
# by rounding only.
FFT_WORKERS = None


def poisson(delta, omega_m: float):
    """phi with lap(phi) = (3/2) Omega_m delta on the periodic mesh (FFT, FP64)."""
    nm = delta.shape[0]
    if FFT_WORKERS:
        import scipy.fft
        dk = scipy.fft.rfftn(delta, workers=FFT_WORKERS)
        return scipy.fft.irfftn(dk * green_function(nm, omega_m), s=delta.shape, axes=(0, 1, 2),
                                workers=FFT_WORKERS)
    dk = np.fft.rfftn(delta)
    return np.fft.irfftn(dk * green_function(nm, omega_m), s=delta.shape, axes=(0, 1, 2))


def gradient4(phi):
    """4-point central difference of phi along x, y, z (returns d phi / d x_i, arrays [z,y,x])."""
    out = []
    for axis in (2, 1, 0):  # x, y, z
        a = np.roll(phi, -1, axis) - np.roll(phi, 1, axis)
        b = np.roll(phi, -2, axis) - np.roll(phi, 2, axis)
        out.append((8.0 * a - b) / 12.0)
    return out


def cic_interp(field, x):
    """CIC interpolation of a mesh field [z, y, x] to positions x (N,3)."""
    nm = field.shape[0]
    i0, d = cic_weights(x, nm)
    f = field.reshape(-1)
    out = np.zeros(len(i0))
    for cz in (0, 1):
        wz = d[:, 2] if cz else 1.0 - d[:, 2]
        iz = (i0[:, 2] + cz) % nm
        for cy in (0, 1):
            wy = d[:, 1] if cy else 1.0 - d[:, 1]
            iy = (i0[:, 1] + cy) % nm
            for cx in (0, 1):
                wx = d[:, 0] if cx else 1.0 - d[:, 0]
                ix = (i0[:, 0] + cx) % nm
                out += wx * wy * wz * f[ix + nm * (iy + nm * iz)]
    return out


def force_field(x, nm: int, omega_m: float, n_particles: int | None = None):
    """Mesh force -grad(phi) (3 arrays) and phi for particles at x."""
    n = len(x) if n_particles is None else n_particles
    delta = density_contrast(cic_deposit(x, nm), n)
    phi = poisson(delta, omega_m)
    g = gradient4(phi)
    return [-gi for gi in g], phi


def pm_accel(x, nm: int, omega_m: float):
    """Force on each particle, F = -grad(phi) interpolated by CIC, shape (N,3)."""
    f, _ = force_field(x, nm, omega_m)
    return np.stack([cic_interp(fi, x) for fi in f], axis=1)


class PMRun:
    """DKD leapfrog with merged drifts over a fixed scale-factor schedule."""

    def __init__(self, x, p, nm: int, cosmo: Cosmology, a_init: float, a_final: float,
                 n_steps: int, spacing: int = 0):
        self.x = np.mod(np.asarray(x, np.float64), nm)
        self.p = np.asarray(p, np.float64).copy()
        self.nm = nm
        self.cosmo = cosmo
        self.drift0, self.kicks, self.drifts = step_factors(cosmo, a_init, a_final, n_steps, spacing)
        self.n_steps = n_steps
        self.j = -1  # -1: before the initial half drift

    def _drift(self, dfac):
        self.x = np.mod(self.x + self.p * dfac, self.nm)

    def advance(self):
        """One call = initial half drift (first call) or one kick+drift step."""
        if self.j < 0:
            self._drift(self.drift0)
            self.j = 0
            return
        j = self.j
        acc = pm_accel(self.x, self.nm, self.cosmo.omega_m)
        self.p = self.p + acc * self.kicks[j]
        self._drift(self.drifts[j])
        self.j += 1

    def run(self):
        while self.j < self.n_steps:
            self.advance()
        return self.x, self.p
