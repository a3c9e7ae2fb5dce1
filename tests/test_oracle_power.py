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


def _grid(nm):
    i = np.arange(nm)
    return np.meshgrid(i, i, i, indexing="ij")  # z, y, x


def test_cross_of_a_field_with_itself_and_its_negative():
    g = np.random.default_rng(7)
    delta = g.normal(size=(32, 32, 32))
    k, paa, pbb, pab, nmodes = power.cross_spectrum(delta, delta, 80.0)
    assert np.allclose(paa, pbb, rtol=0) and np.allclose(pab, paa, rtol=1e-12)
    assert np.allclose(power.correlation(paa, pbb, pab), 1.0, rtol=1e-12)
    _, _, _, pneg, _ = power.cross_spectrum(delta, -delta, 80.0)
    assert np.allclose(power.correlation(paa, pbb, pneg), -1.0, rtol=1e-12)


@pytest.mark.parametrize("theta", [0.3, 1.2, 2.5])
def test_cross_of_phase_shifted_cosines_is_cos_theta(theta):
    nm, box, amp = 32, 60.0, 0.2
    z, y, x = _grid(nm)
    ph = 2 * np.pi * (2 * x - 5 * y + 3 * z) / nm  # |n|^2 = 38: shell 6
    a = amp * np.cos(ph)
    b = amp * np.cos(ph + theta)
    k, paa, pbb, pab, nmodes = power.cross_spectrum(a, b, box)
    live = np.nonzero(paa * nmodes > 1e-20)[0]
    assert live.tolist() == [5]
    # all of <a^2> L^3 sits in the one shell; the cross power carries cos(theta) of it
    assert (paa * nmodes).sum() == pytest.approx(amp**2 / 2 * box**3, rel=1e-12)
    assert (pab * nmodes).sum() == pytest.approx(np.cos(theta) * amp**2 / 2 * box**3, rel=1e-10)
    assert power.correlation(paa, pbb, pab)[5] == pytest.approx(np.cos(theta), rel=1e-10)


def test_cross_of_independent_noise_is_zero_within_scatter():
    g = np.random.default_rng(8)
    a, b = g.normal(size=(2, 48, 48, 48))
    k, paa, pbb, pab, nmodes = power.cross_spectrum(a, b, 100.0)
    xi = power.correlation(paa, pbb, pab)
    sel = nmodes > 100
    assert np.all(np.abs(xi[sel]) < 5 / np.sqrt(nmodes[sel]))


@pytest.mark.parametrize("small", [16, 24])
def test_cross_between_mesh_sizes_uses_the_common_modes(small):
    box, amp = 70.0, 0.1
    waves = [(3, -5, 2), (-1, 4, 6), (7, 0, -3)]  # (n_x, n_y, n_z), every |n_i| < 8
    if small == 24:
        waves += [(-10, 3, -5), (11, -2, 1)]  # |n_i| up to 11 < 12, shells 12 and 11

    def field(nm):
        z, y, x = _grid(nm)
        return sum(amp * np.cos(2 * np.pi * (nx * x + ny * y + nz * z) / nm + 0.4 * j)
                   for j, (nx, ny, nz) in enumerate(waves))

    a, b = field(small), field(2 * small)
    k, paa, pbb, pab, nmodes = power.cross_spectrum(a, b, box)
    assert len(k) == small // 2
    shells = sorted({int(np.floor(np.sqrt(nx * nx + ny * ny + nz * nz) + 0.5)) for nx, ny, nz in waves})
    live = np.nonzero(paa * nmodes > 1e-20)[0] + 1
    assert live.tolist() == shells
    for p in (paa, pbb, pab):  # the same band-limited field on both meshes: one spectrum
        assert (p * nmodes).sum() == pytest.approx(len(waves) * amp**2 / 2 * box**3, rel=1e-10)
    assert np.allclose(power.correlation(paa, pbb, pab)[live - 1], 1.0, rtol=1e-10)
    # the mode counts: integer vectors with every |n_i| < small/2, shell floor(|n| + 1/2), brute force
    h = small // 2
    f = np.arange(-h + 1, h)
    n2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    sh = np.floor(np.sqrt(n2) + 0.5)
    assert np.array_equal(nmodes, [(sh == s).sum() for s in range(1, h + 1)])
    # a scaled copy on the same mesh size keeps xi = 1 and scales P_ab linearly
    _, _, _, pab2, _ = power.cross_spectrum(field(small), 3.0 * field(small), box)
    _, p16, _, _, _ = power.cross_spectrum(field(small), field(small), box)
    assert np.allclose(pab2, 3.0 * p16, rtol=1e-12)
