"""The two-level force (cube_set_two_level) against oracle.twolevel: the Poisson solve from one
density, and whole runs."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import pm, power, twin, twolevel

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def Sim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_06121_amd import Sim as S
    return S


def np_for(nm):
    return next(p for p in (32, 48, 64, 96, 128, 192, 256) if p % (nm // 4) == 0)


@pytest.mark.parametrize("nm,r_s", [(64, 4.0), (64, 6.0), (128, 8.0), (256, 6.0)])
def test_two_level_solve_matches_oracle(Sim, nm, r_s):
    """GPU (FP32) two-level potential from a clumped particle density within 1e-5 (relative L2) of
    the FP64 oracle's, and its 4-point gradient too; switched off, the single-level solve again."""
    nc = nm // 4
    n = nm**3 // 8
    x, v = synth.particle_cloud(17 + nm, n, nm, clump_frac=0.3)
    st = twin.load(x, v, nc, 1, 1)
    delta = twin.delta_from_rho(twin.deposit_int(st, nm), st.n, 1)
    with Sim(np_for(nm), nm, 100.0, omega_m=0.3, capacity=n) as sim:
        sim.set_two_level(r_s)
        sim.set_mesh(delta)
        sim.stage_solve()
        phi = sim.get_mesh()
        sim.set_two_level(0)
        sim.set_mesh(delta)
        sim.stage_solve()
        phi1 = sim.get_mesh()
    ref = twolevel.potential(delta.astype(np.float64), nc, 0.3, r_s)
    assert np.linalg.norm(phi - ref) / np.linalg.norm(ref) < 1e-5
    g, gr = pm.gradient4(phi.astype(np.float64)), pm.gradient4(ref)
    num = np.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(g, gr)))
    assert num / np.sqrt(sum((b**2).sum() for b in gr)) < 1e-5
    ref1 = pm.poisson(delta.astype(np.float64), 0.3)
    assert np.linalg.norm(phi1 - ref1) / np.linalg.norm(ref1) < 1e-5
    # the two forces differ by the coarse restriction's aliasing only
    assert np.linalg.norm(ref - ref1) / np.linalg.norm(ref1) < 0.01


def test_two_level_validation(Sim):
    with Sim(**synth.WORKLOADS["c1_pm32"]) as sim:
        for bad in (2.0, 100.0):
            with pytest.raises(Exception):
                sim.set_two_level(bad)
        sim.set_two_level(5.0)
        sim.set_two_level(0.0)


@pytest.mark.parametrize("name", ["c1_pm32", "c2_pm128"])
def test_two_level_full_run_power(Sim, name):
    """A whole run with the two-level force (r_s = 6 fine cells) against the single-level FP64 oracle's
    P(k) at a = 1: the same tolerances as the single-level GPU run (1% below 0.2 k_Nyquist), and within
    0.5% of the single-level GPU run below k_Nyquist/2."""
    ref = json.load(open(os.path.join(HERE, "golden", f"{name}_pk.json")))
    cfg = synth.WORKLOADS[name]
    out = []
    for r_s in (6.0, 0.0):
        with Sim(**cfg) as sim:
            sim.set_two_level(r_s)
            sim.init_ic()
            sim.step(cfg["n_steps"])
            out.append(sim.get_power())
    (k, p2, _), (_, p1, _) = out
    kny = np.pi * cfg["nm_side"] / cfg["box"]
    dev = np.abs(p2 / np.array(ref["pk"]) - 1)
    rel = np.abs(p2 / p1 - 1)
    print(name, f"two-level vs oracle: k<0.2k_Ny {dev[k < 0.2 * kny].max():.4f}, k<k_Ny/2 {dev[k < kny / 2].max():.4f}; "
          f"vs single-level GPU k<k_Ny/2 {rel[k < kny / 2].max():.4f}")
    assert dev[k < 0.2 * kny].max() < 0.01
    assert rel[k < kny / 2].max() < 0.005
