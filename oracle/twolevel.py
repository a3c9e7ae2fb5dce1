"""Two-level particle-mesh potential: a short-range part on the fine mesh and a long-range part on
a mesh R = 4 times coarser that compensates it (Sec. 2.3.1, Sec. 2.3.3, Fig. update_vp).

Test infrastructure only (see ``oracle/__init__``).

The paper computes a fine-mesh force with a kernel that vanishes beyond the buffer region
(F_f(r > N_b) = 0) on each extended tile, plus a compensating coarse-mesh force from the coarse
density through a global FFT, and takes its kernels K_f, K_c from CUBEP3M without stating them.
Readings (one per open point):
* Split of the Green's function G(k) = -(3/2) Omega_m / k^2 (k in rad per fine cell): fine part
  G (1 - S), coarse part G S, with S(k) = exp(-k^2 r_s^2) and r_s in fine cells. The fine part's
  potential around a point mass falls as erfc(r / (2 r_s)) / r, so it is below 2e-5 of Newton's
  at r = 6 r_s: the paper's cut-off holds for N_b >= 6 r_s / R coarse cells.
* Coarse density: the fine CIC density contrast restricted to the coarse mesh with tent weights
  (every fine cell within R fine cells of a coarse cell centre along each axis, weight 1 - |d| / R,
  normalised), a coarse-mesh CIC of the fine density. Its transfer B(n) per mode is divided out.
* Coarse potential: phi_c(n) = G(n) S(n) R^3 D_c(n) / B(n) for the modes with every |n_i| < N_c/2,
  D_c the DFT of the coarse density; it joins the fine potential on the fine mesh by band-limited
  interpolation (its spectrum placed at the same integer frequencies), so that
      phi(n) = G(n) [(1 - S(n)) D_f(n) + S(n) R^3 D_c(n) / B(n)]   (|n_i| < N_c/2),
      phi(n) = G(n) (1 - S(n)) D_f(n)                              (otherwise).
  A density without power at or beyond the coarse Nyquist frequency gives exactly the
  single-level potential; the difference otherwise is the restriction's aliasing, weighted by S.
* The force is the single-level one's: the 4-point gradient of phi on the fine mesh, interpolated
  to the particles with CIC (oracle.pm), in one kick (the paper kicks with F_f and F_c in turn).
* On one device the fine part is solved with one FFT over the whole fine mesh: with a kernel that
  vanishes beyond the buffer that equals the tile-by-tile solve on the extended tiles.

Pins (tests/test_oracle_twolevel.py): a band-limited density gives the single-level potential to
rounding; the coarse-mesh transfer of single fine modes (restriction, aliasing) against the
closed form of the tent weights; the fine part's real-space cut-off; pair forces against the
periodic direct sum (oracle.ewald) at 4.5 - 14 fine cells within the single-level force's
tolerances; momentum conservation.
"""
from __future__ import annotations

import numpy as np

from . import pm


def tent_weights(R: int):
    """Offsets b (fine cells from a coarse cell's first fine cell) and normalised weights of the
    restriction along one axis: the fine cells whose centres lie within R of the coarse centre."""
    b = np.arange(-R // 2, R + R // 2)
    d = b - (R - 1) / 2.0  # distance from the coarse centre, fine cells
    w = np.clip(1.0 - np.abs(d) / R, 0.0, None)
    return b, w / w.sum()


def restrict(delta, nc: int):
    """Coarse density contrast [zc, yc, xc] from the fine one (tent weights along each axis)."""
    nm = delta.shape[0]
    R = nm // nc
    b, w = tent_weights(R)
    out = np.asarray(delta, np.float64)
    base = np.arange(0, nm, R)
    for ax in range(3):
        acc = 0.0
        for bi, wi in zip(b, w):
            acc = acc + wi * np.take(out, (base + bi) % nm, axis=ax)
        out = acc
    return out


def transfer(q, nm: int, R: int):
    """Restriction transfer along one axis for fine frequencies q: sum_b w_b exp(2 pi i q b / N_m)."""
    b, w = tent_weights(R)
    return (w[None, :] * np.exp(2j * np.pi * np.outer(np.asarray(q, np.float64), b) / nm)).sum(axis=1)


def split(nm: int, r_s: float):
    """S(k) on the rfftn layout of the fine mesh."""
    kz, ky, kx = pm.kvectors(nm)
    return np.exp(-(kx**2 + ky**2 + kz**2) * r_s * r_s)


def potential(delta, nc: int, omega_m: float, r_s: float, parts: bool = False):
    """Two-level potential on the fine mesh from the fine density contrast delta [z, y, x]."""
    delta = np.asarray(delta, np.float64)
    nm = delta.shape[0]
    R = nm // nc
    G = pm.green_function(nm, omega_m)
    S = split(nm, r_s)
    Df = np.fft.rfftn(delta)
    fine_k = G * (1.0 - S) * Df
    Dc = np.fft.rfftn(restrict(delta, nc))
    coarse_k = np.zeros_like(fine_k)
    f = np.fft.fftfreq(nm, 1.0 / nm).astype(np.int64)  # signed frequency of each index
    low = np.nonzero(np.abs(f) < nc // 2)[0]
    lowx = np.arange(nc // 2)
    t = transfer(f, nm, R)
    for iz in low:
        for iy in low:
            B = t[iz] * t[iy] * t[lowx]
            coarse_k[iz, iy, lowx] = (G[iz, iy, lowx] * S[iz, iy, lowx] * R**3
                                      * Dc[f[iz] % nc, f[iy] % nc, lowx] / B)
    phi = np.fft.irfftn(fine_k + coarse_k, s=delta.shape, axes=(0, 1, 2))
    if not parts:
        return phi
    return (phi, np.fft.irfftn(fine_k, s=delta.shape, axes=(0, 1, 2)),
            np.fft.irfftn(coarse_k, s=delta.shape, axes=(0, 1, 2)))


def accel(x, nm: int, nc: int, omega_m: float, r_s: float):
    """Two-level force on particles at x (N, 3): CIC density, two-level potential, 4-point gradient,
    CIC interpolation."""
    n = len(x)
    delta = pm.density_contrast(pm.cic_deposit(x, nm), n)
    phi = potential(delta, nc, omega_m, r_s)
    return np.stack([-pm.cic_interp(g, x) for g in pm.gradient4(phi)], axis=1)
