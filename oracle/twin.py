"""FP32 step-by-step reference of the compressed PM step (numpy float32/int64 only).

Test infrastructure only (see ``oracle/__init__``).

CUBE is a lossy compression of plain PM (oracle.pm). The lossy part -- encoding, cell counts,
storage order, integer density -- has to be reproduced bit-exactly by the GPU from identical
inputs, so this module spells out one fixed sequence of IEEE operations for it, written from
the paper's equations. Every FP32 operation is a separate numpy float32 operation
(round-to-nearest) except the fused multiply-adds named below, which round once (fma32, computed
exactly); every FP64 operation likewise in float64.

State (cell-ordered storage, Sec. 2.1):
  cnt[c]      particles per coarse cell, c = x + N_c (y + N_c z)
  chi[d, i]   stored position code chi + 2^{8 n_chi - 1} (unsigned, 1 or 2 bytes)
  nu[d, i]    velocity code, signed, |nu| <= (M-1)/2, M = 2^{8 n_nu} - 1
  vc[d, c]    coarse-cell mean velocity (FP32), Eq. (deltav)
  vs[c]       decode scale sigma sqrt(2/pi) (FP32), Eq. (v)
Units: fine-mesh cells, ratio R = N_m / N_c = 4, H0 = 1, momentum p = a^2 dx/dt.

Definitions (the device contract):
* position decode, Eq. (x): local offset in fine cells l = (2 chi_u + 1) 2^{1 - 8 n_chi}, chi_u
  the stored unsigned code; global fine position 4 c + l.
* velocity decode, Eq. (v): v = fma(vs, T[nu], vc) with T[nu] = FP32(tan(pi nu / M)).
* integer CIC (Sec. 3 CIC, cell centres at i + 1/2): in units of 2^{1-8 n_chi} fine cells the
  particle sits at P = c 2^{8 n_chi + 1} + 2 chi_u + 1; Q = P - 2^{8 n_chi - 2};
  i0 = Q >> (8 n_chi - 1), f = Q mod 2^{8 n_chi - 1}; weights (2^{8 n_chi-1} - f, f), the mass
  of a particle is 2^{3 (8 n_chi - 1)}; sums are exact int64.
  delta = FP32( FP64(rho) * (N_m^3 / (N_p 2^{3(8 n_chi - 1)})) - 1 ).
* gradient, 4-point: D = 8 (phi[i+1] - phi[i-1]) - (phi[i+2] - phi[i-2]) (FP32, force -D/12).
* interpolation: r = fma(wx1, D(1), wx0*D(0)) along x, then y, then z (FP32, exact dyadic
  weights).
* kick: v' = fma(t, kf, v), kf = FP32(-K/12); drift: l' = fma(v', df, l), df = FP32(Delta).
* new cell: k = -1 if l' < 0, +1 if l' >= 4, else 0 (|l'| beyond one cell is a CFL error);
  l'' = l' - 4k; chi_u' = clamp(floor(l'' 2^{8 n_chi - 2}), 0, 2^{8 n_chi} - 1).
* moments per new cell (int64): n, S1_d = sum rint(v'_d 2^32), S2 = sum_d rint(v'_d^2 2^24).
* per-cell statistics in FP64 (cell_stats), then Eq. (nu) through an edge table:
  u = (v' - vc) * inv (FP32), nu = -(M-1)/2 + #{edges e_j <= u}, e_j = tan(pi (j - 1/2) / M)
  rounded up to FP32 (so u >= e_j in FP32 iff u >= the exact edge), i.e. round-to-nearest of
  M atan(u) / pi, Eq. (nu).
* order: by new cell, then by the source cell's offset from the new cell (z, y, x each in
  -1, 0, +1 order), then by previous storage order -- a counting sort that is stable for every
  particle whose move does not cross the periodic boundary and is translation invariant.

Parity status: pinned. The codec parts reduce to oracle.codec (the FP64 plain definitions) within
one FP32 rounding (tests/test_oracle_twin.py); the integer CIC equals oracle.pm.cic_deposit
exactly; the move agrees with an FP64 evaluation of the same formulas to FP32 rounding.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import numpy as np

R = 4
F32 = np.float32


def fma32(a, b, c):
    """a * b + c rounded once to FP32 (the device's fused multiply-add), elementwise.

    The product of two FP32 values is exact in FP64; the FP64 sum is rounded to odd (the exact
    error of the sum, from TwoSum, tells whether it was inexact and on which side), and rounding an
    odd-rounded value with at least two extra bits to FP32 gives the correctly rounded result."""
    a = np.asarray(a, np.float32).astype(np.float64)
    b = np.asarray(b, np.float32).astype(np.float64)
    c = np.asarray(c, np.float32).astype(np.float64)
    p = a * b
    s = p + c
    bb = s - p
    e = (p - (s - bb)) + (c - bb)
    step = (e != 0) & ((s.view(np.int64) & 1) == 0)
    s = np.where(step, np.nextafter(s, np.where(e > 0, np.inf, -np.inf)), s)
    return s.astype(np.float32)
SQ2PI = math.sqrt(2.0 / math.pi)
SIGMA_GLOBAL = 0
SIGMA_PER_CELL = 1


def vel_m(nnu: int) -> int:
    return (1 << (8 * nnu)) - 1


@functools.lru_cache(maxsize=None)
def decode_table(nnu: int) -> np.ndarray:
    """T[nu + (M-1)/2] = FP32(tan(pi nu / M)), computed with the C library tan in FP64 (read-only,
    computed once per code width)."""
    m = vel_m(nnu)
    half = (m - 1) // 2
    t = np.array([math.tan(math.pi * float(nu) / float(m)) for nu in range(-half, half + 1)],
                 dtype=np.float64).astype(np.float32)
    t.flags.writeable = False
    return t


@functools.lru_cache(maxsize=None)
def edge_table(nnu: int) -> np.ndarray:
    """Bin edges of Eq. (nu) rounded up to FP32 (M - 1 entries, ascending; read-only, computed once
    per code width)."""
    m = vel_m(nnu)
    half = (m - 1) // 2
    out = np.empty(m - 1, dtype=np.float32)
    for i, j in enumerate(range(-(half - 1), half + 1)):
        e = math.tan(math.pi * (float(j) - 0.5) / float(m))
        f = np.float32(e)
        if float(f) < e:
            f = np.nextafter(f, np.float32(np.inf))
        out[i] = f
    out.flags.writeable = False
    return out


@dataclass
class State:
    nc: int
    nchi: int
    nnu: int
    cnt: np.ndarray   # uint32 [nc^3]
    chi: np.ndarray   # uint8/uint16 [3, N]
    nu: np.ndarray    # int8/int16 [3, N]
    vc: np.ndarray    # float32 [3, nc^3]
    vs: np.ndarray    # float32 [nc^3]

    @property
    def n(self) -> int:
        return int(self.chi.shape[1])

    def cell_of_particle(self) -> np.ndarray:
        return np.repeat(np.arange(self.nc**3, dtype=np.int64), self.cnt.astype(np.int64))

    def copy(self):
        return State(self.nc, self.nchi, self.nnu, self.cnt.copy(), self.chi.copy(), self.nu.copy(),
                     self.vc.copy(), self.vs.copy())


def _coords(cid, nc):
    return cid % nc, (cid // nc) % nc, cid // (nc * nc)


def chi_dtype(nchi):
    return np.uint8 if nchi == 1 else np.uint16


def nu_dtype(nnu):
    return np.int8 if nnu == 1 else np.int16


# ---------------------------------------------------------------------------------------
# per-cell statistics (FP64 from exact integer moments)
# ---------------------------------------------------------------------------------------
def moments(cid_new, v32, n_cells):
    """Integer moments (n, S1[3], S2) per cell from FP32 velocities v32 (3, N)."""
    n = np.bincount(cid_new, minlength=n_cells).astype(np.int64)
    v64 = v32.astype(np.float64)
    s1 = np.empty((3, n_cells), dtype=np.int64)
    s2 = np.zeros(n_cells, dtype=np.int64)
    for d in range(3):
        t1 = np.rint(v64[d] * 4294967296.0).astype(np.int64)
        s1[d] = _int_bincount(cid_new, t1, n_cells)
        t2 = np.rint(v64[d] * v64[d] * 16777216.0).astype(np.int64)
        s2 += _int_bincount(cid_new, t2, n_cells)
    return n, s1, s2


def _int_bincount(idx, vals, n):
    out = np.zeros(n, dtype=np.int64)
    np.add.at(out, idx, vals)
    return out


def cell_stats(n, s1, s2, n_total, sigma_mode):
    """vc (3, C) FP32, vs (C,) FP32, inv (C,) FP32 and sigma_g^2 from the integer moments."""
    nd = n.astype(np.float64)
    ok = n > 0
    safe = np.where(ok, nd, 1.0)
    d1 = safe * 4294967296.0
    m = [np.where(ok, s1[d].astype(np.float64) / d1, 0.0) for d in range(3)]
    d2 = safe * 16777216.0
    e2 = np.where(ok, s2.astype(np.float64) / d2, 0.0)
    mm = m[0] * m[0]
    mm = mm + m[1] * m[1]
    mm = mm + m[2] * m[2]
    dev = e2 - mm
    dev = np.where(ok & (dev > 0.0), dev, 0.0)
    # global dispersion: per-cell fixed-point terms n dev 2^20 (each below 2^54, beyond which the
    # step reports an overflow), summed exactly (Python integers) and rounded once to FP64
    term = (dev * nd) * 1048576.0
    if np.any(term >= 2.0**54):
        raise OverflowError("a cell's n x dispersion term reaches 2^54")
    q = np.rint(term).astype(np.int64)
    qsum = int(q.astype(object).sum())
    sg2 = float(qsum) / ((3.0 * float(n_total)) * 1048576.0)
    if not sg2 > 0.0:
        sg2 = 2.0**-60
    if sigma_mode == SIGMA_PER_CELL:
        s2c = dev / 3.0
        use_g = (n < 2) | (s2c < sg2 * 9.5367431640625e-07)
        s2c = np.where(use_g, sg2, s2c)
    else:
        s2c = np.full(n.shape, sg2)
    sc = np.sqrt(s2c) * SQ2PI
    vc = np.stack([mi.astype(np.float32) for mi in m])
    return vc, sc.astype(np.float32), (1.0 / sc).astype(np.float32), sg2


def encode_nu(v32, vc32, inv32, nnu):
    """Eq. (nu) via the FP32 edge table: u = (v - vc) * inv, nu = -(M-1)/2 + #{e <= u}."""
    e = edge_table(nnu)
    half = (vel_m(nnu) - 1) // 2
    u = (v32 - vc32) * inv32
    return (np.searchsorted(e, u, side="right").astype(np.int64) - half).astype(nu_dtype(nnu))


# ---------------------------------------------------------------------------------------
# load path: uncompressed FP64 particles -> encoded state (stable sort by cell)
# ---------------------------------------------------------------------------------------
def load(x64, v64, nc: int, nchi: int, nnu: int, sigma_mode: int = SIGMA_PER_CELL) -> State:
    """x64 (N,3) fine-mesh positions, v64 (N,3) momenta -> State. Positions follow Eq. (chi) in FP64;
    velocities are rounded to FP32 and encoded with the statistics of their cell."""
    x64 = np.asarray(x64, np.float64)
    xc = x64 * 0.25
    bad = (xc < 0.0) | (xc >= nc)
    xc = np.where(bad, xc - nc * np.floor(xc / nc), xc)
    cell = np.floor(xc).astype(np.int64)
    cell = np.where(cell >= nc, cell - nc, cell)
    nb = 1 << (8 * nchi)
    b = np.floor((xc - cell) * float(nb)).astype(np.int64)
    b = np.clip(b, 0, nb - 1)
    cid = cell[:, 0] + nc * (cell[:, 1] + nc * cell[:, 2])
    order = np.argsort(cid, kind="stable")
    cid_s = cid[order]
    v32 = np.asarray(v64, np.float64).astype(np.float32)[order].T.copy()
    n_cells = nc**3
    n, s1, s2 = moments(cid_s, v32, n_cells)
    vc, vs, inv, _ = cell_stats(n, s1, s2, len(cid), sigma_mode)
    nu = np.stack([encode_nu(v32[d], vc[d][cid_s], inv[cid_s], nnu) for d in range(3)])
    chi = b[order].T.astype(chi_dtype(nchi))
    return State(nc, nchi, nnu, n.astype(np.uint32), chi, nu, vc, vs)


# ---------------------------------------------------------------------------------------
# decode
# ---------------------------------------------------------------------------------------
def decode(st: State):
    """FP32 local offsets l (3,N) in fine cells, velocities v (3,N), cell ids (N,)."""
    cid = st.cell_of_particle()
    unit = F32(2.0 ** (1 - 8 * st.nchi))
    l = (st.chi.astype(np.int64) * 2 + 1).astype(np.float32) * unit
    t = decode_table(st.nnu)
    half = (vel_m(st.nnu) - 1) // 2
    tv = t[st.nu.astype(np.int64) + half]
    v = fma32(st.vs[cid][None, :], tv, st.vc[:, cid])
    return l, v, cid


def positions_fine(st: State):
    """Global fine-mesh positions (FP64, exact) of every particle, shape (N,3)."""
    cid = st.cell_of_particle()
    cx, cy, cz = _coords(cid, st.nc)
    unit = 2.0 ** (1 - 8 * st.nchi)
    c = np.stack([cx, cy, cz], axis=1).astype(np.float64)
    return 4.0 * c + (st.chi.T.astype(np.float64) * 2 + 1) * unit


# ---------------------------------------------------------------------------------------
# integer CIC deposit
# ---------------------------------------------------------------------------------------
def _cic_int(st: State):
    cid = st.cell_of_particle()
    cc = _coords(cid, st.nc)
    sh = 8 * st.nchi - 1
    i0, f = [], []
    for d in range(3):
        p = cc[d] * (1 << (sh + 2)) + 2 * st.chi[d].astype(np.int64) + 1
        q = p - (1 << (sh - 1))
        i0.append(q >> sh)
        f.append(q & ((1 << sh) - 1))
    return i0, f, sh


def deposit_int(st: State, nm: int) -> np.ndarray:
    """Exact integer CIC density rho[z, y, x] (int64, particle mass 2^{3(8 n_chi - 1)})."""
    i0, f, sh = _cic_int(st)
    one = 1 << sh
    rho = np.zeros(nm**3, dtype=np.int64)
    for cz in (0, 1):
        wz = f[2] if cz else one - f[2]
        iz = (i0[2] + cz) % nm
        for cy in (0, 1):
            wy = f[1] if cy else one - f[1]
            iy = (i0[1] + cy) % nm
            for cx in (0, 1):
                wx = f[0] if cx else one - f[0]
                ix = (i0[0] + cx) % nm
                np.add.at(rho, ix + nm * (iy + nm * iz), wx * wy * wz)
    return rho.reshape(nm, nm, nm)


def delta_from_rho(rho, n_particles: int, nchi: int) -> np.ndarray:
    nm3 = rho.size
    inv_mean = float(nm3) / (float(n_particles) * 2.0 ** (3 * (8 * nchi - 1)))
    return (rho.astype(np.float64) * inv_mean - 1.0).astype(np.float32)


# ---------------------------------------------------------------------------------------
# move: interpolate force from phi, kick, drift, re-encode, counting-sort order
# ---------------------------------------------------------------------------------------
def move(st: State, phi32: np.ndarray, kfac32, dfac32, sigma_mode: int = SIGMA_PER_CELL,
         return_info: bool = False):
    """One fused kick+drift+encode pass with a given potential phi32 [z,y,x] (float32).

    kfac32 = FP32(-K/12), dfac32 = FP32(Delta). Returns the new State (and optionally the
    per-particle displacement codes and the CFL flag)."""
    kf = F32(kfac32)
    df = F32(dfac32)
    nm = phi32.shape[0]
    phi = np.asarray(phi32, np.float32).reshape(-1)
    l, v, cid = decode(st)
    i0, f, sh = _cic_int(st)
    wunit = F32(2.0 ** -sh)
    one = 1 << sh
    w = [[(one - f[d]).astype(np.float32) * wunit, f[d].astype(np.float32) * wunit] for d in range(3)]

    def at(ix, iy, iz):
        return phi[(ix % nm) + nm * ((iy % nm) + nm * (iz % nm))]

    def dgrad(d, ix, iy, iz):
        e = [0, 0, 0]
        e[d] = 1
        p1 = at(ix + e[0], iy + e[1], iz + e[2])
        m1 = at(ix - e[0], iy - e[1], iz - e[2])
        p2 = at(ix + 2 * e[0], iy + 2 * e[1], iz + 2 * e[2])
        m2 = at(ix - 2 * e[0], iy - 2 * e[1], iz - 2 * e[2])
        a = p1 - m1
        b = p2 - m2
        return F32(8) * a - b

    vnew = np.empty_like(v)
    tgrad = np.empty_like(v)
    for d in range(3):
        s = []
        for cz in (0, 1):
            r = []
            for cy in (0, 1):
                d0 = dgrad(d, i0[0], i0[1] + cy, i0[2] + cz)
                d1 = dgrad(d, i0[0] + 1, i0[1] + cy, i0[2] + cz)
                r.append(fma32(w[0][1], d1, w[0][0] * d0))
            s.append(fma32(w[1][1], r[1], w[1][0] * r[0]))
        t = fma32(w[2][1], s[1], w[2][0] * s[0])
        tgrad[d] = t
        vnew[d] = fma32(t, kf, v[d])
    lnew = fma32(vnew, df, l)
    cfl = bool(np.any(~np.isfinite(lnew)) or np.any(lnew < F32(-4)) or np.any(lnew >= F32(8)))
    k = np.where(lnew < F32(0), -1, np.where(lnew >= F32(4), 1, 0)).astype(np.int64)
    lw = np.where(k == 1, lnew - F32(4), np.where(k == -1, lnew + F32(4), lnew)).astype(np.float32)
    nb = 1 << (8 * st.nchi)
    chi_new = np.clip(np.floor(lw * F32(2.0 ** (8 * st.nchi - 2))).astype(np.int64), 0, nb - 1)
    nc = st.nc
    cx, cy, cz = _coords(cid, nc)
    ncx, ncy, ncz = (cx + k[0]) % nc, (cy + k[1]) % nc, (cz + k[2]) % nc
    cnew = ncx + nc * (ncy + nc * ncz)
    code = 26 - ((k[2] + 1) * 9 + (k[1] + 1) * 3 + (k[0] + 1))
    old = np.arange(st.n, dtype=np.int64)
    perm = np.lexsort((old, code, cnew))
    cnew_s = cnew[perm]
    v_s = vnew[:, perm]
    n_cells = nc**3
    n, s1, s2 = moments(cnew_s, v_s, n_cells)
    vc, vs, inv, _ = cell_stats(n, s1, s2, st.n, sigma_mode)
    nu = np.stack([encode_nu(v_s[d], vc[d][cnew_s], inv[cnew_s], st.nnu) for d in range(3)])
    chi = chi_new[:, perm].astype(chi_dtype(st.nchi))
    new = State(nc, st.nchi, st.nnu, n.astype(np.uint32), chi, nu, vc, vs)
    if return_info:
        dcode = (k[2] + 1) * 9 + (k[1] + 1) * 3 + (k[0] + 1)
        return new, dict(cfl=cfl, dcode=dcode, perm=perm, v=vnew, l=lnew, t=tgrad)
    return new
