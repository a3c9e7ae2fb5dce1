"""Offsets between the particles of two runs, Eq. (offset) of Sec. 3 ("Displacement of particles"),
FP64.

Test infrastructure only (see ``oracle/__init__``).

With particle IDs the same particle can be found in both runs. Its displacement is Psi = x - q
(Eulerian minus Lagrangian position), and the offset is Delta Psi = |Psi_i - Psi_0|. The Lagrangian
q is the same in both runs and cancels, so Delta Psi = |x_i - x_0|, where each component is the
shortest separation on the periodic box (the minimal image). Reading: positions and offsets are in
fine-mesh cells. The paper's grey reference curve is the displacement itself, |Psi_0| = |x_0 - q|,
taken with the same minimal image.

Pins (tests/test_oracle_displacement.py): the minimal-image offset equals a brute-force minimum
over the 27 periodic images; identical runs have zero offset; a pair straddling the box edge is
as close as its periodic distance; the lattice positions match the initial conditions' q.
"""
from __future__ import annotations

import numpy as np


def periodic_delta(xa, xb, nm: float):
    """Component-wise shortest separation xa - xb on a periodic box of side nm, in [-nm/2, nm/2)."""
    return np.mod(np.asarray(xa, dtype=np.float64) - np.asarray(xb, dtype=np.float64) + 0.5 * nm, nm) - 0.5 * nm


def offsets(xa, xb, nm: float):
    """Delta Psi for positions xa, xb of shape (N, 3) (the same particle in row i of both)."""
    d = periodic_delta(xa, xb, nm)
    return np.sqrt((d * d).sum(axis=1))


def lattice_positions(np_side: int, nm_side: int):
    """Lagrangian positions q (N, 3) in fine cells of lattice particle i = x + N_p (y + N_p z)."""
    i = np.arange(np_side)
    qz, qy, qx = np.meshgrid(i, i, i, indexing="ij")
    return (np.stack([qx.reshape(-1), qy.reshape(-1), qz.reshape(-1)], axis=1) + 0.5) * (nm_side / np_side)


def cdf(values, grid):
    """Fraction of values at or below each grid point (the CDF of Fig. dsp)."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    return np.searchsorted(v, np.asarray(grid, dtype=np.float64), side="right") / float(len(v))
