"""Pins of oracle.twolevel (the two-level potential: short-range fine part, compensating coarse part)."""
import math

import numpy as np
import pytest

from oracle import ewald, pm, twolevel


def test_band_limited_density_gives_single_level_potential():
    """Without power at or beyond the coarse Nyquist frequency the restriction has no aliasing, and
    the fine and coarse parts add up to the single-level potential exactly."""
    nm, nc = 64, 16
    i = np.arange(nm)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    g = np.random.default_rng(4)
    delta = np.zeros((nm, nm, nm))
    for _ in range(10):
        n = g.integers(-7, 8, size=3)
        delta += g.normal() * np.cos(2 * np.pi * (n[0] * x + n[1] * y + n[2] * z) / nm + g.uniform(0, 6.3))
    for r_s in (4.0, 6.0, 8.0):
        phi = twolevel.potential(delta, nc, 0.3, r_s)
        ref = pm.poisson(delta, 0.3)
        assert np.abs(phi - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("q", [1, 5, 7, 9, 16, 23, 33])
def test_restriction_transfer_of_single_modes(q):
    """restrict() of one fine Fourier mode exp(2 pi i q j / N_m) is transfer(q) times the same mode
    sampled at the coarse cells' first fine cells, for every q (including aliased ones)."""
    nm, nc = 64, 16
    R = nm // nc
    j = np.arange(nm)
    mode = np.exp(2j * np.pi * q * j / nm)
    field = np.broadcast_to(mode[None, None, :], (nm, nm, nm))
    got = twolevel.restrict(field.real, nc) + 1j * twolevel.restrict(field.imag, nc)
    c = np.arange(nc)
    expect = twolevel.transfer([q], nm, R)[0] * np.exp(2j * np.pi * q * R * c / nm)
    # the other axes: a constant restricts to itself (weights sum to one)
    assert np.allclose(got, expect[None, None, :], atol=1e-13)
    assert abs(twolevel.transfer([0], nm, R)[0] - 1.0) < 1e-15


def test_fine_part_is_short_range():
    """Around a point mass the fine part carries the force near the mass and falls off beyond a few
    r_s: at r = 4 r_s it is below 10% of the whole, and from 6 r_s on below 3%. (The continuous split
    alone would leave erfc(u) + 2u exp(-u^2)/sqrt(pi) with u = r/(2 r_s), 4e-4 at 6 r_s; the rest is
    the lattice kernel 1/k^2's tail, which the single-level force has too. A tile-by-tile solve with
    a buffer of 6 r_s would drop it; the library solves the fine part over the whole mesh.)"""
    nm, nc, r_s = 64, 16, 4.0
    delta = np.zeros((nm, nm, nm))
    delta[0, 0, 0] = nm**3
    delta -= 1.0
    phi, fine, coarse = twolevel.potential(delta, nc, 1.0, r_s, parts=True)
    gx_all = pm.gradient4(phi)[0][0, 0]
    gx_fine = pm.gradient4(fine)[0][0, 0]
    assert abs(gx_fine[2] - gx_all[2]) < 0.01 * abs(gx_all[2])
    assert abs(gx_fine[int(4 * r_s)]) < 0.1 * abs(gx_all[int(4 * r_s)])
    for r in range(int(6 * r_s), nm // 2 - 4):
        assert abs(gx_fine[r]) <= 0.03 * abs(gx_all[r]), (r, gx_fine[r], gx_all[r])


@pytest.mark.parametrize("r_s", [6.0, 8.0])
@pytest.mark.parametrize("r", [4.5, 6.0, 9.0, 14.0])
def test_two_level_force_matches_direct_sum(r, r_s):
    """Pair forces at 4.5 - 14 fine cells against the periodic direct sum, with the single-level
    force's tolerances (radial within 3% per orientation and 1% on average, tangential below 3%)."""
    nm, nc, om = 64, 16, 1.0
    g = np.random.default_rng(int(r * 10))
    rad, tan = [], []
    for _ in range(12):
        n = g.normal(size=3)
        n /= np.linalg.norm(n)
        x0 = g.uniform(20, 44, size=3)
        x = np.stack([x0, x0 + r * n])
        acc = twolevel.accel(x, nm, nc, om, r_s)[1]
        ew = ewald.ewald_accel(x, nm, om)[1]
        fr, er = acc @ n, ew @ n
        rad.append(fr / er)
        tan.append(np.linalg.norm(acc - fr * n) / abs(er))
    rad = np.array(rad)
    assert np.all(np.abs(rad - 1) < 0.03), rad
    assert abs(rad.mean() - 1) < 0.01, rad.mean()
    assert max(tan) < 0.03, max(tan)


def test_two_level_force_close_to_single_level_on_a_cloud():
    """On a clumped cloud the two-level force differs from the single-level one by the coarse
    restriction's aliasing only: rms difference below 1% of the rms force."""
    import synth
    nm, nc = 64, 16
    x, _ = synth.particle_cloud(3, 20000, nm)
    a2 = twolevel.accel(x, nm, nc, 0.3, 6.0)
    a1 = pm.pm_accel(x, nm, 0.3)
    assert np.sqrt(((a2 - a1) ** 2).mean()) < 0.01 * np.sqrt((a1**2).mean())
