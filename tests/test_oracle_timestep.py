"""Pins of oracle.timestep: closed-form steps in Einstein-de Sitter and an adaptive Zel'dovich run."""
import math

import numpy as np
import pytest

from oracle import timestep, zeldovich
from oracle.cosmology import Cosmology

EDS = Cosmology(1.0, 0.0)


def test_expansion_limited_steps_are_geometric():
    a = timestep.schedule_from_maxima(EDS, 0.02, 1.0, [0.0] * 200, [0.0] * 200, 1.0, 1.0, 0.05)
    m = int(np.argmax(a >= 1.0))
    want = 0.02 * 1.05 ** np.arange(m)
    assert np.allclose(a[:m], want, rtol=1e-13) and a[m] == 1.0 and want[-1] * 1.05 >= 1.0


@pytest.mark.parametrize("a0,vmax,eta_v", [(0.02, 3.0, 0.5), (0.3, 20.0, 1.0), (0.8, 7.0, 0.25)])
def test_velocity_limited_step_in_eds(a0, vmax, eta_v):
    # Delta = 2 (a0^-1/2 - a1^-1/2) = eta_v / vmax
    want = (a0**-0.5 - eta_v / (2.0 * vmax)) ** -2
    got = timestep.next_a(EDS, a0, vmax, 0.0, eta_v, 1e9, 10.0, 10.0)
    assert got == pytest.approx(want, rel=1e-9)


@pytest.mark.parametrize("a0,gmax,eta_a", [(0.02, 50.0, 0.5), (0.4, 5.0, 0.2)])
def test_acceleration_limited_step_in_eds(a0, gmax, eta_a):
    # 4 g (x - x0)^2 / (x0 x) = eta_a with x = sqrt(a1): x = x0 ((2 + c) + sqrt(c^2 + 4c)) / 2, c = eta_a / (4 g)
    x0, c = math.sqrt(a0), eta_a / (4.0 * gmax)
    want = (x0 * ((2.0 + c) + math.sqrt(c * c + 4.0 * c)) / 2.0) ** 2
    got = timestep.next_a(EDS, a0, 0.0, gmax, 1e9, eta_a, 10.0, 10.0)
    assert got == pytest.approx(want, rel=1e-9)


def test_adaptive_run_follows_the_zeldovich_wave():
    np_side, nm = 32, 64
    x, p, q, psi1 = zeldovich.plane_wave(np_side, nm, EDS, 0.02, 1.5)
    run = timestep.AdaptivePMRun(x, p, nm, EDS, 0.02, 1.0, 0.5, 0.5, 0.08)
    xf, pf = run.run()
    assert run.done and run.a[run.j] == 1.0 and 20 < run.j < 200
    xe, pe, _, _ = zeldovich.plane_wave(np_side, nm, EDS, 1.0, 1.5)
    amp = np.abs(psi1).max()
    dx = (xf[:, 0] - xe[:, 0] + nm / 2) % nm - nm / 2
    assert np.sqrt((dx**2).mean()) <= 0.01 * amp
    pamp = np.abs(pe[:, 0]).max()
    assert np.sqrt(((pf[:, 0] - pe[:, 0]) ** 2).mean()) <= 0.01 * pamp
    # the log reproduces the schedule
    a = timestep.schedule_from_maxima(EDS, 0.02, 1.0, run.vmax, run.gmax, 0.5, 0.5, 0.08)
    assert np.array_equal(a[: len(run.a)], np.array(run.a))
