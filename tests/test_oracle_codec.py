"""Pins of oracle.codec: the paper's worked example and closed-form codec identities."""
import math

import numpy as np
import pytest

from oracle import codec


def test_worked_example_under_eq_x():
    # n_chi = 1, N_c = 4 (1-D): chi = (-128, 127, 0, 60), rho_c = (1, 0, 2, 1)
    x = codec.decode_position_1d_from_counts(np.array([-128, 127, 0, 60]), np.array([1, 0, 2, 1]), 1)
    assert np.array_equal(x, [0.001953125, 2.998046875, 2.501953125, 3.736328125])


@pytest.mark.parametrize("nchi", [1, 2])
def test_position_roundtrip_every_code(nchi):
    lo, hi = codec.chi_range(nchi)
    chi = np.arange(lo, hi + 1)
    cell = np.full(chi.shape, 3)
    x = codec.decode_position(cell, chi, nchi)
    c2, chi2 = codec.encode_position(x, 8, nchi)
    assert np.array_equal(chi2, chi) and np.all(c2 == 3)


@pytest.mark.parametrize("nchi", [1, 2])
def test_position_quantisation_bound(nchi):
    g = np.random.default_rng(0)
    x = g.uniform(0, 16, size=200000)
    cell, chi = codec.encode_position(x, 16, nchi)
    xr = codec.decode_position(cell, chi, nchi)
    err = np.abs(x - xr)
    assert err.max() <= 2.0 ** (-8 * nchi - 1) + 1e-12
    # the resolution statement: bins of width 2^{-8 n_chi} coarse cells
    assert err.max() > 0.9 * 2.0 ** (-8 * nchi - 1)


def test_position_wrap_and_edge_clamp():
    c, chi = codec.encode_position(np.array([-0.25, 4.0, 3.9999999999999996]), 4, 1)
    assert list(c) == [3, 0, 3]
    assert chi[0] == 64 and chi[1] == -128 and chi[2] == 127


@pytest.mark.parametrize("nnu", [1, 2])
def test_velocity_roundtrip_every_code(nnu):
    m = codec.vel_m(nnu)
    nu = np.arange(-(m - 1) // 2, (m - 1) // 2 + 1)
    v = codec.decode_velocity(nu, 0.3, 1.7, nnu)
    assert np.array_equal(codec.encode_velocity(v, 0.3, 1.7, nnu), nu)
    # odd symmetry about v_c
    assert np.allclose(v - 0.3, -(v[::-1] - 0.3), rtol=0, atol=1e-12)


def test_velocity_angle_error_bound():
    g = np.random.default_rng(1)
    v = g.normal(0, 2.0, size=100000)
    nu = codec.encode_velocity(v, 0.0, 2.0, 1)
    u = v * math.sqrt(math.pi / 8.0)
    ang = np.arctan(u) - np.pi * nu / 255
    assert np.abs(ang).max() <= math.pi / (2 * 255) + 1e-12


def test_cauchy_gaussian_peak_match():
    # the tan codec (uniform codes) and a Gaussian with the same sigma have the same density at
    # the centre (stated after Eq. (v))
    s = 1.3
    assert codec.cauchy_peak_density(s) == pytest.approx(1.0 / (math.sqrt(2 * math.pi) * s), rel=1e-14)


def test_cell_order_is_stable():
    cid = np.array([2, 0, 2, 1, 0, 2])
    counts, order = codec.cell_order(cid, 4)
    assert list(counts) == [2, 1, 3, 0]
    assert list(order) == [1, 4, 3, 0, 2, 5]


def test_one_byte_count_export():
    counts = np.array([0, 3, 254, 255, 256, 7, 1000, 12], dtype=np.uint32)
    rho1, over = codec.counts_to_u8(counts)
    assert rho1.tolist() == [0, 3, 254, 255, 255, 7, 255, 12]
    assert over.dtype == np.uint32 and over.tolist() == [255, 256, 1000]  # cell order
    assert np.array_equal(codec.counts_from_u8(rho1, over), counts)
    with pytest.raises(ValueError):
        codec.counts_from_u8(rho1, over[:2])
