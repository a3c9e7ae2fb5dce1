"""Pins of oracle.displacement (Eq. (offset))."""
import itertools

import numpy as np
import pytest

import synth
from oracle import displacement, ic
from oracle.cosmology import Cosmology


def test_minimal_image_equals_brute_force_over_images():
    g = np.random.default_rng(3)
    nm = 16.0
    xa, xb = g.uniform(0, nm, size=(2, 500, 3))
    got = displacement.offsets(xa, xb, nm)
    shifts = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.float64) * nm
    brute = np.min(np.linalg.norm(xa[:, None, :] - xb[:, None, :] - shifts[None, :, :], axis=2), axis=1)
    assert np.allclose(got, brute, rtol=0, atol=1e-12)


def test_identical_runs_and_edge_pairs():
    x = np.array([[0.1, 5.0, 15.9], [3.0, 3.0, 3.0]])
    assert np.all(displacement.offsets(x, x, 16.0) == 0.0)
    a = np.array([[0.1, 0.0, 0.0]])
    b = np.array([[15.9, 0.0, 0.0]])
    assert displacement.offsets(a, b, 16.0)[0] == pytest.approx(0.2, abs=1e-12)
    assert displacement.periodic_delta(a, b, 16.0)[0, 0] == pytest.approx(0.2, abs=1e-12)


def test_lattice_positions_are_the_initial_conditions_q():
    cfg = synth.WORKLOADS["c1_pm32"]
    cosmo = Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])
    _, _, q = ic.zeldovich(16, 32, cfg["box"], cosmo, cfg["a_init"], 1, noise=np.zeros((16, 16, 16)))
    assert np.array_equal(displacement.lattice_positions(16, 32), q)


def test_cdf():
    v = np.array([0.3, 0.1, 0.2, 0.2])
    assert np.allclose(displacement.cdf(v, [0.0, 0.1, 0.2, 0.25, 1.0]), [0.0, 0.25, 0.75, 0.75, 1.0])
