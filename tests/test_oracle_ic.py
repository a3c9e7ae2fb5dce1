"""Pins of oracle.ic: amplitude and units of the Zel'dovich initial conditions."""
import numpy as np

from oracle import ic, pm, power
from oracle.cosmology import Cosmology


def test_ic_density_tracks_linear_spectrum():
    c = Cosmology(0.3, 0.7, h=0.7, sigma8=0.8)
    np_side, nm, box, a = 64, 64, 200.0, 0.1
    x, p, q = ic.zeldovich(np_side, nm, box, c, a, seed=5)
    delta = pm.density_contrast(pm.cic_deposit(x, nm), np_side**3)
    k, pk, nmodes = power.power_spectrum(delta, box)
    # CIC window: divide by sinc^4 of the shell mean wavenumber (approximate deconvolution)
    kc = k * box / nm / 2.0
    w = (np.sin(kc) / kc) ** 4
    sel = slice(2, 12)
    ratio = pk[sel] / w[sel] / c.pk_linear(k[sel], a)
    assert np.all(np.abs(ratio - 1.0) < 4.0 * np.sqrt(2.0 / nmodes[sel]) + 0.05), ratio
    assert abs(np.average(ratio, weights=nmodes[sel]) - 1.0) < 0.05


def test_ic_velocity_is_growing_mode_eds():
    c = Cosmology(1.0, 0.0, h=0.7, sigma8=0.8)
    np_side, nm, box, a = 16, 32, 100.0, 0.02
    x, p, q = ic.zeldovich(np_side, nm, box, c, a, seed=9)
    disp = (x - q + nm / 2) % nm - nm / 2
    # EdS: p = a^2 E f Psi(a) with E = a^{-3/2}, f = 1, so p = a^{1/2} Psi(a) = a^{3/2} Psi_1
    assert np.allclose(p, a**0.5 * disp, rtol=1e-10, atol=1e-14)
    # displacements at a = 0.02 are a small fraction of a coarse cell
    assert np.abs(disp).max() < 1.0


def _band_limited_at(noise, points, cut):
    """(1/N^3) sum over the modes with every |n_i| < cut of W(n) exp(2 pi i n.x / N), by direct
    summation (no FFT), at the given lattice coordinates x (in cells of this lattice)."""
    n = noise.shape[0]
    idx = np.arange(n)
    out = np.zeros(len(points))
    modes = [(a, b, c) for a in range(-cut + 1, cut) for b in range(-cut + 1, cut) for c in range(-cut + 1, cut)]
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    for (mz, my, mx) in modes:
        w = np.sum(noise * np.exp(-2j * np.pi * (mx * xx + my * yy + mz * zz) / n))
        ph = np.exp(2j * np.pi * (mx * points[:, 0] + my * points[:, 1] + mz * points[:, 2]) / n)
        out += (w * ph).real
    return out / n**3


def test_refined_noise_holds_the_parent_field_on_its_scales():
    from oracle import philox
    seed, n, parent = 5, 8, 4
    child = ic.refined_noise(seed, n, parent)
    par = philox.white_noise_grid(seed, parent)
    # the band-limited fields (every |n_i| < parent/2) agree everywhere up to the white-noise
    # normalisation: unit variance per cell, so the finer lattice's field is (parent/n)^{3/2}
    # times the coarser one's; compare them at random points
    g = np.random.default_rng(0)
    pts_parent = g.uniform(0, parent, size=(6, 3))
    got = _band_limited_at(child, pts_parent * (n / parent), parent // 2)
    want = _band_limited_at(par, pts_parent, parent // 2) * (parent / n) ** 1.5
    assert np.allclose(got, want, rtol=1e-10, atol=1e-12)
    # the small scales are the run's own noise: not the unrefined run's, and of unit variance
    own = philox.white_noise_grid(seed, n)
    assert not np.allclose(child, own)
    big = ic.refined_noise(seed, 32, 16)
    assert abs(big.var() - 1) < 0.05 and abs(big.mean()) < 0.05
