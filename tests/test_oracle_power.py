"""Pins of oracle.power: single mode, white-noise level, mode counting."""
import numpy as np
import pytest

from oracle import power


def test_single_cosine_mode():
    nm, box = 32, 100.0
    i = np.arange(nm)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    delta = 0.1 * np.cos(2 * np.pi * (3 * x + 4 * y) / nm)  # |n| = 5
    k, pk, nmodes = power.power_spectrum(delta, box)
    # |delta_k|^2 = (0.1 N^3 / 2)^2 on the 4 modes +-(3,4,0) and +-(3,-4,0)... here only (3,4),(-3,-4)
    # appear as two half-space entries with weight 2 each: total power sum_k P = <delta^2> L^3
    total = (pk * nmodes).sum()
    assert total == pytest.approx(0.1**2 / 2 * box**3, rel=1e-12)
    assert np.nonzero(pk * nmodes > 1e-12 * total)[0].tolist() == [4]  # shell b = 5
    assert k[4] == pytest.approx(2 * np.pi / box * 5, rel=0.05)


def test_white_noise_flat():
    nm, box = 64, 50.0
    g = np.random.default_rng(2)
    delta = g.normal(size=(nm, nm, nm))
    k, pk, nmodes = power.power_spectrum(delta, box)
    expect = box**3 / nm**3
    sel = nmodes > 200
    scatter = np.sqrt(2.0 / nmodes[sel])  # chi^2 scatter of a shell mean
    assert np.all(np.abs(pk[sel] / expect - 1) < 5 * scatter)


def test_mode_counts():
    nm = 16
    k, pk, nmodes = power.power_spectrum(np.zeros((nm, nm, nm)), 1.0)
    f = np.fft.fftfreq(nm) * nm
    n2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    b = np.floor(np.sqrt(n2) + 0.5)
    expect = np.array([(b == s).sum() for s in range(1, nm // 2 + 1)])
    assert np.array_equal(nmodes, expect)
