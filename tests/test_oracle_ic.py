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
