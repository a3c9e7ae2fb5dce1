"""Zel'dovich initial conditions on uncompressed particles (Sec. 2.3.2, Fig. ic), FP64.

Test infrastructure only (see ``oracle/__init__``).

Steps, in the paper's order:
1. Gaussian white noise w on the N_p^3 Lagrangian lattice (oracle.philox; lattice index
   x fastest), Fourier transformed and multiplied by the linear amplitude:
   delta_k = FFT(w) sqrt(N_p^3 P(k, a_i) / L^3), so that <|delta_k|^2> = N_p^6 P / L^3 in the
   unnormalised DFT convention.
2. Displacement potential from -lap(Phi) = delta_L, Phi_k = delta_k / k^2.
3. Psi = grad(Phi). Reading: the paper differentiates in real space with an unstated stencil;
   here the derivative is spectral, Psi_k = i k Phi_k, and the k = 0 mode and every mode on a
   Nyquist plane (any |n_i| = N_p/2) are zeroed.
4. Lattice point q = (i + 1/2) L / N_p; x = q + Psi; momentum p = a^2 E(a) f(a) Psi at a_i
   (growing mode: dx/dt = H f Psi).

Refined initial conditions (the PM-error reference of Sec. 3: the same initial conditions with
8 times more particles and cells): the noise of an N_p^3 run refined from an N_q^3 parent
(N_q divides N_p) takes, for every mode with all |n_i| < N_q/2, the parent's transformed noise
scaled by (N_p/N_q)^{3/2} (so both runs hold one Gaussian field on those scales); the other modes
come from the run's own noise, drawn with seed XOR REFINE_KEY. Reading: the paper does not say
how its higher-resolution run shares the initial conditions.

Output is in fine-mesh units (lengths in cells of the N_m mesh, H0 = 1), particles in
lattice order. Pins: tests/test_oracle_ic.py (a single-mode field reproduces the analytic
displacement; the measured P(k) of the IC density tracks the input spectrum).
"""
from __future__ import annotations

import numpy as np

from .cosmology import Cosmology
from .philox import white_noise_grid


def displacement_field(noise, box: float, cosmo: Cosmology, a: float):
    """Psi (3 arrays [z,y,x], Mpc/h) from white noise on an n^3 lattice."""
    n = noise.shape[0]
    wk = np.fft.rfftn(noise)
    nf = np.fft.fftfreq(n) * n
    nr = np.fft.rfftfreq(n) * n
    nz, ny, nx = nf[:, None, None], nf[None, :, None], nr[None, None, :]
    kf = 2.0 * np.pi / box
    kz, ky, kx = kf * nz, kf * ny, kf * nx
    k2 = kx**2 + ky**2 + kz**2
    kk = np.sqrt(k2)
    pk = np.zeros_like(kk)
    nz_mask = kk > 0
    pk[nz_mask] = cosmo.pk_linear(kk[nz_mask], a)
    amp = np.sqrt(n**3 * pk / box**3)
    dk = wk * amp
    half = n // 2
    nyq = (np.abs(nz) == half) | (np.abs(ny) == half) | (np.abs(nx) == half)
    dk = np.where(nyq, 0.0, dk)
    dk[0, 0, 0] = 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        phik = np.where(k2 > 0, dk / k2, 0.0)
    return [np.fft.irfftn(1j * kd * phik, s=noise.shape, axes=(0, 1, 2)) for kd in (kx, ky, kz)]


REFINE_KEY = 0x9E3779B97F4A7C15


def refined_noise(seed: int, n: int, parent_n: int):
    """White noise on the n^3 lattice whose modes with every |n_i| < parent_n/2 are the parent's
    (n^3 lattice noise of seed ^ REFINE_KEY elsewhere), as a real array [z, y, x]."""
    own = np.fft.rfftn(white_noise_grid(seed ^ REFINE_KEY, n))
    par = np.fft.rfftn(white_noise_grid(seed, parent_n))
    f = np.rint(np.fft.fftfreq(parent_n) * parent_n).astype(np.int64)
    keep = np.abs(f) < parent_n // 2
    fl = f[keep]
    fx = np.arange(parent_n // 2)
    own[np.ix_(fl % n, fl % n, fx)] = par[np.ix_(fl % parent_n, fl % parent_n, fx)] * (n / parent_n) ** 1.5
    return np.fft.irfftn(own, s=(n, n, n), axes=(0, 1, 2))


def zeldovich(np_side: int, nm_side: int, box: float, cosmo: Cosmology, a: float, seed: int,
              noise=None):
    """Positions x (N,3, fine units, wrapped) and momenta p (N,3) in lattice order."""
    if noise is None:
        noise = white_noise_grid(seed, np_side)
    psi = displacement_field(noise, box, cosmo, a)
    scale = nm_side / box  # Mpc/h -> fine cells
    psi = np.stack([ps.reshape(-1) * scale for ps in psi], axis=1)
    i = np.arange(np_side)
    qz, qy, qx = np.meshgrid(i, i, i, indexing="ij")
    cell = nm_side / np_side
    q = (np.stack([qx.reshape(-1), qy.reshape(-1), qz.reshape(-1)], axis=1) + 0.5) * cell
    x = np.mod(q + psi, nm_side)
    vfac = a * a * float(cosmo.E(a)) * cosmo.f(a)
    return x, vfac * psi, q
