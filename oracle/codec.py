"""FP64 reference of CUBE's compressed particle storage (Sec. 2.1 and 2.2).

Test infrastructure only (see ``oracle/__init__``).

Conventions (readings of the paper, each listed in the design notes):
* Coarse cells are 0-based (the paper's n_c is 1-based), so Eq. (x) reads
  x_d = n_c + 2^{-8 n_chi} (chi_d + 2^{8 n_chi - 1} + 1/2)   in coarse-cell units.
* [ ] in Eq. (chi) is floor after periodic wrap into [0, N_c); the bin index is clamped to
  2^{8 n_chi} - 1 so that a value that rounds up to the cell edge stays in its cell.
* Eq. (nu): the bracket is round-to-nearest and the constant under the root is pi/(2 sigma^2),
  the exact inverse of Eq. (v). Codes run over -(M-1)/2 .. (M-1)/2 with M = 2^{8 n_nu} - 1.
* Storage order is cell order (cell id c = x + N_c (y + N_c z)); a stable sort keeps the
  incoming order inside a cell (the worked example under Eq. (x) shows an unsorted cell).

Pins (tests/test_oracle_codec.py): the worked 1-D example printed under Eq. (x);
encode(decode(chi)) = chi for every code; |x - decode(encode(x))| <= 2^{-8 n_chi - 1};
encode(decode(nu)) = nu for every velocity code; odd symmetry; the Cauchy/Gaussian peak match
at nu = 0 stated after Eq. (v); the 1-byte count export (Sec. 2.1: 255 marks a cell whose
true count, 255 or more, goes to a separate list of 4-byte integers) round-trips and puts every
count below 255 in its byte.
"""
from __future__ import annotations

import math

import numpy as np


def chi_range(nchi: int):
    half = 1 << (8 * nchi - 1)
    return -half, half - 1


def encode_position(x_coarse, n_c: int, nchi: int):
    """Eq. (chi). x_coarse: positions in coarse-cell units, any shape (..., 3).
    Returns (cell, chi): integer coarse cell per dimension (wrapped) and signed chi."""
    x = np.mod(np.asarray(x_coarse, dtype=np.float64), n_c)
    cell = np.floor(x).astype(np.int64)
    cell = np.where(cell >= n_c, cell - n_c, cell)  # x == n_c after mod rounding
    nb = 1 << (8 * nchi)
    frac = x - cell
    b = np.minimum(np.floor(nb * frac).astype(np.int64), nb - 1)
    b = np.maximum(b, 0)
    return cell, b - (nb >> 1)


def decode_position(cell, chi, nchi: int):
    """Eq. (x) with 0-based cells: the centre of the chi bin, in coarse-cell units."""
    nb = 1 << (8 * nchi)
    return np.asarray(cell, dtype=np.float64) + (np.asarray(chi, dtype=np.float64) + (nb >> 1) + 0.5) / nb


def decode_position_1d_from_counts(chi, rho_c, nchi: int):
    """Worked example under Eq. (x): positions from chi plus per-cell counts in storage order."""
    cell = np.repeat(np.arange(len(rho_c)), rho_c)
    return decode_position(cell, chi, nchi)


def vel_m(nnu: int) -> int:
    return (1 << (8 * nnu)) - 1


def encode_velocity(v, vc, sigma, nnu: int):
    """Eq. (nu): nu = nint( M/pi * atan( (v - v_c) sqrt(pi / (2 sigma^2)) ) ), M = 2^{8 n_nu} - 1.
    sigma is the per-dimension dispersion."""
    m = vel_m(nnu)
    u = (np.asarray(v, np.float64) - vc) * np.sqrt(np.pi / (2.0 * np.asarray(sigma, np.float64) ** 2))
    return np.rint(m / np.pi * np.arctan(u)).astype(np.int64)


def decode_velocity(nu, vc, sigma, nnu: int):
    """Eq. (v): v = v_c + tan(pi nu / M) sqrt(2 sigma^2 / pi)."""
    m = vel_m(nnu)
    return vc + np.tan(np.pi * np.asarray(nu, np.float64) / m) * np.sqrt(2.0 * np.asarray(sigma, np.float64) ** 2 / np.pi)


def cell_id(cell, n_c: int):
    cell = np.asarray(cell, dtype=np.int64)
    return cell[..., 0] + n_c * (cell[..., 1] + n_c * cell[..., 2])


def cell_order(cid, n_cells: int):
    """Counts per cell and the stable cell-ordered permutation (np.argsort, kind='stable')."""
    counts = np.bincount(cid, minlength=n_cells)
    order = np.argsort(cid, kind="stable")
    return counts, order


def counts_to_u8(counts):
    """1-byte coarse density of Sec. 2.1: min(count, 255) per cell, and the true counts of the
    cells marked 255, in cell order, as 4-byte integers."""
    c = np.asarray(counts, dtype=np.int64)
    rho1 = np.minimum(c, 255).astype(np.uint8)
    overflow = c[c >= 255].astype(np.uint32)
    return rho1, overflow


def counts_from_u8(rho1, overflow):
    """Inverse of counts_to_u8."""
    c = np.asarray(rho1, dtype=np.uint8).astype(np.uint32)
    mark = np.nonzero(c == 255)[0]
    if len(mark) != len(overflow):
        raise ValueError("overflow list does not match the cells marked 255")
    c[mark] = np.asarray(overflow, dtype=np.uint32)
    return c


def cauchy_peak_density(sigma: float) -> float:
    """Density at zero of the Eq. (v) code distribution when codes are uniform: the velocity
    is Cauchy with scale sigma sqrt(2/pi), so the peak is 1 / (pi s)."""
    s = sigma * math.sqrt(2.0 / math.pi)
    return 1.0 / (math.pi * s)
