"""The 2048^3-particle workload at full size, in the launch configuration the benchmark times
(two warm-up steps, then the autotuned kernel variants). The FP64 oracle cannot run 8.6e9
particles, so the checks are properties that hold at any size:

* mass: the coarse-cell counts sum to N exactly, after the initial conditions and after steps;
* initial conditions: P(k) of the lowest shells follows the linear spectrum at a_init (Sec. 2.3.2,
  BBKS + sigma_8), within the cosmic variance of those shells;
* growth: over the steps the lowest shells grow as the linear growing mode integrated with the
  simulation's own kick and drift factors (for a long-wavelength mode the PM force is
  3/2 Omega_m times the displacement, so the leapfrog of one mode can be followed exactly); the
  same modes are compared, so there is no cosmic variance in the ratio.
"""
import math

import numpy as np
import pytest

import synth
from oracle.cosmology import Cosmology

pytestmark = pytest.mark.gpu

NAME = "c3_pm2048"


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_06121_amd as m
    return m


def linear_leapfrog_growth(cosmo, a0, drift0, kicks, drifts, n):
    """Amplitude of one long-wavelength displacement mode after the initial half drift and n
    kick-drift steps, relative to its value at a0 (Zel'dovich start: p = a^2 E f Psi)."""
    psi = 1.0
    p = a0 * a0 * cosmo.E(a0) * cosmo.f(a0) * psi
    psi += p * drift0
    for j in range(n):
        p += 1.5 * cosmo.omega_m * psi * kicks[j]
        psi += p * drifts[j]
    return psi


def test_full_size_mass_spectrum_and_growth(lib):
    import torch
    torch.cuda.empty_cache()
    cfg = synth.WORKLOADS[NAME]
    need = lib.footprint(**cfg) + (40 << 30)  # plus the z-contiguous FFT scratch the autotuner may pick
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    n = cfg["np_side"] ** 3
    cosmo = Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])
    nb = 16
    with lib.Sim(**cfg) as sim:
        sim.init_ic()
        assert sim.get_counts().sum(dtype=np.int64) == n
        k0, p0, m0 = sim.get_power(nb)
        drift0, kicks, drifts = sim.get_schedule()
        sim.step(2)
        sim.autotune()
        sim.step(1)
        steps = sim.steps_done
        a1 = sim.a
        assert sim.get_counts().sum(dtype=np.int64) == n
        k1, p1, m1 = sim.get_power(nb)
    assert np.array_equal(m0, m1) and np.allclose(k0, k1)
    # initial conditions against the linear spectrum: shells 2..16 together (~2e4 modes, so the
    # mean ratio has a cosmic-variance error of about 1%)
    sel = slice(1, nb)
    ratio = p0[sel] / cosmo.pk_linear(k0[sel], cfg["a_init"])
    mean = np.sum(ratio * m0[sel]) / np.sum(m0[sel])
    print(f"IC P/P_lin over shells 2..{nb}: mean {mean:.4f}; per shell {np.round(ratio, 3)}")
    assert abs(mean - 1) < 0.05
    assert np.all(np.abs(ratio - 1) < 5 * np.sqrt(2 / m0[sel]) + 0.02)
    # growth of the lowest shells over the steps, against the leapfrog of the linear mode
    g = linear_leapfrog_growth(cosmo, cfg["a_init"], drift0, kicks, drifts, steps)
    growth = p1[1:8] / p0[1:8]
    print(f"a = {a1:.4f} after {steps} steps: P ratio {np.round(growth, 4)}, linear leapfrog {g * g:.4f}, "
          f"(D(a)/D(a0))^2 {(cosmo.D(a1) / cosmo.D(cfg['a_init'])) ** 2:.4f}")
    assert np.all(np.abs(growth / (g * g) - 1) < 0.01)


@pytest.mark.parametrize("variant", [dict(fft_z_layout=0), dict(fft_col_width=8, fft_z_layout=1, fft_z_width=4)])
def test_full_size_poisson_on_plane_waves(lib, variant):
    """The 2048^3 Poisson solve (the five FFT passes with the Green's function, in the mesh layout and
    in the z-contiguous layout the autotuner picks at this size) on a density of plane waves, whose
    potential is known exactly: phi_k = -(3/2) Omega_m delta_k / |k|^2 with k = 2 pi n / N_m per
    fine cell (Sec. 2.3.3). Checked on 2e5 sampled cells."""
    import torch
    torch.cuda.empty_cache()
    cfg = synth.WORKLOADS[NAME]
    need = lib.footprint(**cfg) + (40 << 30)
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    nm, om = cfg["nm_side"], cfg["omega_m"]
    # (n_x, n_y, n_z), amplitude, phase: low, intermediate and near-Nyquist modes, one off-axis
    waves = [((3, 0, 0), 0.5, 0.3), ((0, 517, 0), 0.2, 1.1), ((0, 0, 1023), 0.1, -0.7), ((5, -7, 0), 0.3, 2.0)]
    i = torch.arange(nm, dtype=torch.float64)

    def c1(n, amp, ph):
        return (amp * torch.cos(2 * math.pi * n * i / nm + ph)).float()

    delta = torch.empty((nm, nm, nm), dtype=torch.float32)  # [z, y, x], host memory
    delta.copy_(c1(3, 0.5, 0.3)[None, None, :].expand(nm, nm, nm))
    delta += c1(517, 0.2, 1.1)[None, :, None]
    delta += c1(1023, 0.1, -0.7)[:, None, None]
    # cos(a x + b y + ph) = cos(a x) cos(b y + ph) - sin(a x) sin(b y + ph)
    ax, by = 2 * math.pi * 5 * i / nm, 2 * math.pi * -7 * i / nm + 2.0
    delta += (0.3 * (torch.cos(ax)[None, :] * torch.cos(by)[:, None] - torch.sin(ax)[None, :] * torch.sin(by)[:, None])).float()[None]
    with lib.Sim(**cfg) as sim:
        sim.set_variant(**variant)
        sim.set_mesh(delta.numpy())
        del delta
        sim.stage_solve()
        phi = torch.from_numpy(sim.get_mesh())
    g = np.random.default_rng(31)
    z, y, x = (g.integers(0, nm, size=200000) for _ in range(3))
    want = np.zeros(len(x))
    for (nx, ny, nz), amp, ph in waves:
        k2 = (2 * math.pi / nm) ** 2 * (nx * nx + ny * ny + nz * nz)
        want += -1.5 * om * amp * np.cos(2 * math.pi * (nx * x + ny * y + nz * z) / nm + ph) / k2
    got = phi[torch.from_numpy(z), torch.from_numpy(y), torch.from_numpy(x)].double().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"variant {variant}: max |phi - exact| / max |phi| = {err:.2e}")
    assert err < 1e-5
