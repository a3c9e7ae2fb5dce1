"""Exact one-dimensional Zel'dovich plane wave before shell crossing (FP64).

Test infrastructure only (see ``oracle/__init__``).

For a planar perturbation the Zel'dovich approximation is exact until orbits cross:
x = q + D(a) Psi_1(q), p = a^2 E(a) f(a) D(a) Psi_1(q). With
Psi_1(q) = -sin(k q) / (k D_cross) the first crossing happens at D = D_cross (at q = 0).
Used to pin the integrator and the whole PM chain of oracle.pm (and, through the same
configuration, the GPU path).
"""
from __future__ import annotations

import numpy as np

from .cosmology import Cosmology


def plane_wave(np_side: int, nm_side: int, cosmo: Cosmology, a: float, a_cross: float):
    """Particles on the np_side^3 lattice (fine units) displaced along x by one mode k = 2 pi / N_m."""
    cell = nm_side / np_side
    i = np.arange(np_side)
    qz, qy, qx = np.meshgrid(i, i, i, indexing="ij")
    q = (np.stack([qx.reshape(-1), qy.reshape(-1), qz.reshape(-1)], axis=1) + 0.5) * cell
    k = 2.0 * np.pi / nm_side
    d_cross = cosmo.D(a_cross)
    psi1 = -np.sin(k * q[:, 0]) / (k * d_cross)
    D = cosmo.D(a)
    x = q.copy()
    x[:, 0] = np.mod(q[:, 0] + D * psi1, nm_side)
    p = np.zeros_like(q)
    p[:, 0] = a * a * float(cosmo.E(a)) * cosmo.f(a) * D * psi1
    return x, p, q, psi1
