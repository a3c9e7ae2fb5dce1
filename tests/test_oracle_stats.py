"""Pins of the per-cell velocity statistics of oracle.twin (moments, cell_stats) against plain FP64
definitions: v_c is the mean velocity of the particles in the coarse cell (Eq. (deltav)); the
dispersion is the per-dimension variance of v - v_c, one third of the 3-D one (Sec. 2.2, the
equipartition reading); the decode scale of Eq. (v) is sigma sqrt(2/pi); cells with fewer than two
particles or a vanishing dispersion take the global value, which is the same variance over all
particles (the paper's single sigma, Sec. 2.2, last paragraph)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import twin


def plain_stats(cid, v64, n_cells):
    """Per-cell count, mean velocity (3, C), per-dimension variance about the mean (C,), and the
    same variance over all particles: two passes, FP64, no fixed point."""
    n = np.bincount(cid, minlength=n_cells)
    mean = np.stack([np.bincount(cid, weights=v64[d], minlength=n_cells) for d in range(3)]) / np.maximum(n, 1)
    dv = v64 - mean[:, cid]
    ss = np.bincount(cid, weights=(dv**2).sum(axis=0), minlength=n_cells)
    var = ss / np.maximum(n, 1) / 3.0
    var_g = ss.sum() / (3.0 * len(cid))
    return n, mean, var, var_g


def cloud(seed=31, n=20000, nm=32, nc=8):
    """A clumped cloud with a bulk flow, plus hand-made cells: one particle, two identical
    velocities (no dispersion), a tiny dispersion (below 2^-20 of the global one)."""
    x, v = synth.particle_cloud(seed, n, nm, vscale=0.7)
    cell = (np.floor(x / (nm // nc)).astype(np.int64)) % nc
    cid = cell[:, 0] + nc * (cell[:, 1] + nc * cell[:, 2])
    v32 = v.T.astype(np.float32)
    n_cells = nc**3
    # empty out three cells and refill them by hand
    special = np.array([5, 77, 300])
    keep = ~np.isin(cid, special)
    cid, v32 = cid[keep], v32[:, keep]
    extra_c = np.array([5, 77, 77, 300, 300, 300])
    extra_v = np.array([[0.3, -0.2, 0.1], [1.5, 1.5, -0.5], [1.5, 1.5, -0.5],
                        [0.25, 0.5, 0.75], [0.25 + 2**-12, 0.5, 0.75], [0.25, 0.5 - 2**-12, 0.75]],
                       np.float32).T
    cid = np.concatenate([cid, extra_c])
    v32 = np.concatenate([v32, extra_v], axis=1)
    order = np.argsort(cid, kind="stable")
    return cid[order], v32[:, order], n_cells


@pytest.mark.parametrize("mode", [twin.SIGMA_PER_CELL, twin.SIGMA_GLOBAL])
def test_cell_stats_match_plain_fp64(mode):
    cid, v32, n_cells = cloud()
    n_i, s1, s2 = twin.moments(cid, v32, n_cells)
    vc, vs, inv, sg2 = twin.cell_stats(n_i, s1, s2, len(cid), mode)
    n, mean, var, var_g = plain_stats(cid, v32.astype(np.float64), n_cells)
    assert np.array_equal(n_i, n)
    # Eq. (deltav): v_c is the per-cell mean (FP32 of the FP64 mean of fixed-point sums)
    assert np.all(vc[:, n == 0] == 0.0)
    assert np.allclose(vc.astype(np.float64), mean, rtol=2e-7, atol=1e-9)
    # the global dispersion: per-dimension variance over every particle
    assert sg2 == pytest.approx(var_g, rel=1e-6)
    # which cells fall back to the global value
    use_g = (n < 2) | (var < var_g * 2.0**-20)
    assert use_g[5] and use_g[77] and use_g[300] and use_g[n == 0].all()
    assert not use_g[(n >= 2) & (var > 1e-3 * var_g)].any()
    sigma2 = np.full(n_cells, var_g) if mode == twin.SIGMA_GLOBAL else np.where(use_g, var_g, var)
    # Eq. (v): the decode scale is sigma sqrt(2/pi), the encode scale its inverse
    expect = np.sqrt(sigma2) * math.sqrt(2.0 / math.pi)
    assert np.allclose(vs.astype(np.float64), expect, rtol=2e-6)
    assert np.allclose(inv.astype(np.float64), 1.0 / expect, rtol=2e-6)


def test_decode_scale_of_a_known_cell():
    """Two particles at +-(a, a, a) about a mean m: the per-dimension variance is a^2, so the
    decode scale is a sqrt(2/pi) exactly (a sqrt(pi/2), or the 3-D variance, would not be)."""
    a, m = 0.375, np.array([0.5, -1.25, 2.0])
    v32 = np.stack([m + a, m - a]).T.astype(np.float32)
    cid = np.array([0, 0])
    n, s1, s2 = twin.moments(cid, v32, 1)
    vc, vs, inv, sg2 = twin.cell_stats(n, s1, s2, 2, twin.SIGMA_PER_CELL)
    assert np.array_equal(vc[:, 0], m.astype(np.float32))
    assert sg2 == a * a
    assert vs[0] == np.float32(a * math.sqrt(2.0 / math.pi))
    assert inv[0] == np.float32(1.0 / (a * math.sqrt(2.0 / math.pi)))


def test_global_dispersion_sum_exact_beyond_int64():
    """The global dispersion sums per-cell fixed-point terms n dev 2^20; their total can exceed 2^63
    (at 2^33 particles a mean 3-D dispersion above 1024), so it is summed exactly. Cells with
    n dev near the 2^34 limit: the result equals the plain FP64 mean, and an int64 sum would have
    wrapped."""
    cells = 4096
    g = np.random.default_rng(5)
    n = g.integers(1 << 16, 1 << 17, cells).astype(np.int64)
    dev = (2.0**33.9 / n) * g.uniform(0.5, 1.0, cells)  # 3-D variance, n dev < 2^34
    s1 = np.zeros((3, cells), np.int64)
    s2 = np.rint(dev * n * 2.0**24).astype(np.int64)
    vc, vs, inv, sg2 = twin.cell_stats(n, s1, s2, int(n.sum()), twin.SIGMA_GLOBAL)
    dev_used = s2.astype(np.float64) / (n * 2.0**24)
    q = [int(x) for x in np.rint(dev_used * n * 2.0**20)]
    assert sum(q) >= 2**63  # beyond int64
    exact = Fraction(sum(q)) / (3 * int(n.sum()) * 2**20)
    assert sg2 == pytest.approx(float(exact), rel=1e-15)
    assert sg2 == pytest.approx((dev_used * n).sum() / (3.0 * n.sum()), rel=1e-12)
    # a single cell past the limit is refused (the device raises its overflow flag)
    s2[0] = np.int64(2**62)
    n[0] = 1
    with pytest.raises(OverflowError):
        twin.cell_stats(n, s1, s2, int(n.sum()), twin.SIGMA_GLOBAL)
