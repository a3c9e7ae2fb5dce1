"""The whole oracle PM chain (CIC, Poisson, gradient, interpolation, DKD) against the exact 1-D
Zel'dovich plane wave before shell crossing (EdS, crossing at a = 1.5, C1 lattice)."""
import numpy as np

from oracle import pm, zeldovich
from oracle.cosmology import Cosmology


def test_plane_wave_to_a1():
    c = Cosmology(1.0, 0.0)
    np_side, nm = 32, 64
    x, p, q, psi1 = zeldovich.plane_wave(np_side, nm, c, 0.02, 1.5)
    run = pm.PMRun(x, p, nm, c, 0.02, 1.0, 50)
    xf, pf = run.run()
    xe, pe, _, _ = zeldovich.plane_wave(np_side, nm, c, 1.0, 1.5)
    amp = np.abs(psi1).max()
    dx = (xf[:, 0] - xe[:, 0] + nm / 2) % nm - nm / 2
    assert np.sqrt((dx**2).mean()) <= 0.01 * amp
    assert np.abs(dx).max() <= 0.02 * amp
    pamp = np.abs(pe[:, 0]).max()
    dp = pf[:, 0] - pe[:, 0]
    assert np.sqrt((dp**2).mean()) <= 0.01 * pamp
    assert np.abs(dp).max() <= 0.02 * pamp
    # transverse motion stays zero
    assert np.abs(pf[:, 1:]).max() < 1e-10 * pamp
