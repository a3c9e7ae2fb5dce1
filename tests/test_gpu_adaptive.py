"""Adaptive time steps (Sec. 2.3.3): the step maxima the count pass measures are bit-exact with the
FP32 twin, the schedule follows the oracle's rule from the logged maxima, and an adaptive run
agrees with the oracle's adaptive FP64 run."""
import numpy as np
import pytest

import synth
from oracle import power, timestep, twin
from oracle.cosmology import Cosmology

pytestmark = pytest.mark.gpu

ETA = (0.5, 0.05, 0.04)  # eta_v, eta_a (fine cells), eta_e: expansion, then acceleration bind in C1


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_06121_amd as m
    return m


def cosmo_of(cfg):
    return Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])


def f32_norm2(a):
    a = np.asarray(a, np.float32)
    return (a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]


@pytest.mark.parametrize("nchi,nnu,nm,n,variant", [(1, 1, 64, 40000, 0), (2, 2, 64, 25000, 0),
                                                    (1, 1, 32, 20000, 1), (2, 1, 64, 160000, 1)])
def test_step_maxima_bit_exact_with_twin(lib, nchi, nnu, nm, n, variant):
    nc = nm // 4
    x, v = synth.particle_cloud(41 + nm + nchi, n, nm, vscale=1.0, clump_frac=0.5, clump_radius=1.0)
    st = twin.load(x, v, nc, nchi, nnu, 1)
    phi = synth.smooth_potential(7 + nm, nm, amp=2.0 if nm >= 64 else 0.5)
    kf, df = np.float32(-1.3 / 12.0), np.float32(0.5)
    _, info = twin.move(st, phi, kf, df, return_info=True)
    vmax = float(np.sqrt(np.float64(f32_norm2(info["v"]).max())))
    gmax = float(np.sqrt(np.float64(f32_norm2(info["t"]).max())) / 12.0)
    np_side = next(p for p in (32, 48, 64, 96, 128) if p % nc == 0)
    with lib.Sim(np_side, nm, 100.0, x_bytes=nchi, v_bytes=nnu, capacity=n) as sim:
        sim.set_adaptive(*ETA)
        sim.set_state(st.cnt, st.chi, st.nu, st.vc, st.vs)
        sim.set_variant(move_variant=variant)
        sim.set_mesh(phi)
        sim.stage_move(kf, df)
        got = sim.get_last_maxima()
    assert got == (vmax, gmax)


def adaptive_cfg():
    return dict(synth.WORKLOADS["c1_pm32"], x_bytes=2, v_bytes=2, n_steps=400)


@pytest.mark.parametrize("eta,limits", [(ETA, ("expansion", "acceleration")),
                                        ((0.2, 1.0, 0.04), ("expansion", "velocity"))])
def test_adaptive_schedule_follows_the_rule(lib, eta, limits):
    cfg = adaptive_cfg()
    with lib.Sim(**cfg) as sim:
        sim.set_adaptive(*eta)
        sim.init_ic()
        assert sim.step(10) == lib.CUBE_OK
        a_mid = sim.a
        while sim.step(50) == lib.CUBE_OK:
            pass
        assert sim.a == pytest.approx(1.0)
        a_int, vmax, gmax = sim.get_adaptive_log()
        steps = sim.steps_done
        drift0, kicks, drifts = sim.get_schedule()
    cosmo = cosmo_of(cfg)
    want = timestep.schedule_from_maxima(cosmo, cfg["a_init"], cfg["a_final"], vmax, gmax, *eta)
    print(f"{steps} adaptive steps; a after 10 steps {a_mid:.4f}; vmax {vmax[0]:.3g} .. {vmax.max():.3g}, "
          f"gmax up to {gmax.max():.3g}")
    assert a_int[steps] == 1.0 and np.all(a_int[:steps] < 1.0) and np.all(np.diff(a_int[: steps + 1]) > 0)
    assert np.allclose(a_int, want[: len(a_int)], rtol=1e-12)
    # the kick factors used are those of the chosen intervals
    assert np.allclose(kicks[:steps], [cosmo.kick_factor(a_int[j], a_int[j + 1]) for j in range(steps)], rtol=1e-8)
    # every criterion holds for every interval (with the maxima that chose it); count which binds
    binds = {"expansion": 0, "velocity": 0, "acceleration": 0, "end": 0}
    for i in range(1, steps + 1):
        m = max(i - 2, 0)
        d = cosmo.drift_factor(a_int[i - 1], a_int[i])
        g = gmax[m] * cosmo.kick_factor(a_int[i - 1], a_int[i]) * d
        assert a_int[i] <= a_int[i - 1] * (1 + eta[2]) * (1 + 1e-12)
        assert vmax[m] * d <= eta[0] * (1 + 1e-9) and g <= eta[1] * (1 + 1e-9)
        if a_int[i] == 1.0:
            binds["end"] += 1
        elif a_int[i] == a_int[i - 1] * (1 + eta[2]):
            binds["expansion"] += 1
        elif vmax[m] * d > eta[0] * (1 - 1e-6):
            binds["velocity"] += 1
        else:
            assert g > eta[1] * (1 - 1e-6)
            binds["acceleration"] += 1
    print("binding criterion per interval:", binds)
    assert all(binds[c] > 0 for c in limits)


def test_adaptive_run_matches_the_oracle_adaptive_run(lib):
    from oracle import ic, pm
    cfg = adaptive_cfg()
    nm = cfg["nm_side"]
    with lib.Sim(**cfg) as sim:
        sim.set_adaptive(*ETA)
        sim.init_ic()
        while sim.step(50) == lib.CUBE_OK:
            pass
        a_gpu, _, _ = sim.get_adaptive_log()
        steps = sim.steps_done
        k, pk, _ = sim.get_power()
    cosmo = cosmo_of(cfg)
    x, p, _ = ic.zeldovich(cfg["np_side"], nm, cfg["box"], cosmo, cfg["a_init"], cfg["seed"])
    run = timestep.AdaptivePMRun(x, p, nm, cosmo, cfg["a_init"], cfg["a_final"], *ETA)
    run.run()
    k0, p0, _ = power.power_spectrum(pm.density_contrast(pm.cic_deposit(run.x, nm), cfg["np_side"] ** 3), cfg["box"])
    a_or = np.array(run.a)
    n = min(steps, run.j) + 1
    print(f"steps: GPU {steps}, oracle {run.j}; max |a_gpu/a_oracle - 1| {np.abs(a_gpu[:n] / a_or[:n] - 1).max():.2e}")
    assert abs(steps - run.j) <= 1
    assert np.allclose(a_gpu[:n], a_or[:n], rtol=1e-3)
    kny = np.pi * nm / cfg["box"]
    dev = np.abs(pk / p0 - 1)[k < kny / 2]
    print(f"max |P_gpu/P_oracle - 1| below k_Ny/2: {dev.max():.4f}")
    assert dev.max() < 0.01


def test_adaptive_validation_and_switching_off(lib):
    cfg = dict(synth.WORKLOADS["c1_pm32"], n_steps=12)
    with lib.Sim(**cfg) as sim:
        for bad in ((0.0, 1.0, 0.1), (-1.0, 1.0, 0.1), (1.0, float("inf"), 0.1)):
            with pytest.raises(lib.CubeError):
                sim.set_adaptive(*bad)
        sim.set_adaptive(*ETA)
        sim.set_adaptive(0.0, 0.0, 0.0)  # back to the fixed schedule
        sim.init_ic()
        sim.step(3)
        with pytest.raises(lib.CubeError):
            sim.set_adaptive(*ETA)  # only before the first step
        with pytest.raises(lib.CubeError):
            sim.get_adaptive_log()
        got = sim.get_state()
    with lib.Sim(**cfg) as ref:
        ref.init_ic()
        ref.step(3)
        want = ref.get_state()
    for key in ("cnt", "chi", "nu", "vc", "vs"):
        assert np.array_equal(got[key], want[key]), key
    with lib.Batch([cfg, dict(cfg, seed=5)]) as b:
        b.boxes[0].set_adaptive(*ETA)
        b.init_ic()
        with pytest.raises(lib.CubeError) as e:
            b.step(1)
        assert "adaptive" in str(e.value)
