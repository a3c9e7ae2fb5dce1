"""GPU path vs the oracle through the C ABI: bit-exact codes, counts, order and density from
identical inputs; Poisson solve within 1e-5; full runs within the P(k) tolerance."""
import numpy as np
import pytest

import synth
from oracle import pm, twin

pytestmark = pytest.mark.gpu

KEYS = ("cnt", "chi", "nu", "vc", "vs")


@pytest.fixture(scope="module")
def Sim():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_06121_amd import Sim as S
    return S


def assert_state_equal(got: dict, ref: twin.State, tag=""):
    for key in KEYS:
        a, b = got[key], getattr(ref, key)
        assert a.shape == b.shape, (tag, key, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            raise AssertionError(f"{tag} {key}: {len(bad)} mismatches, first {bad[:5].tolist()}")


def twin_state(d: dict, nc, nchi, nnu) -> twin.State:
    return twin.State(nc, nchi, nnu, d["cnt"], d["chi"], d["nu"], d["vc"], d["vs"])


CODECS = [(1, 1, 1), (2, 1, 1), (1, 2, 0), (2, 2, 1)]


@pytest.mark.parametrize("nchi,nnu,mode", CODECS)
def test_load_bit_exact(Sim, nchi, nnu, mode):
    nm, nc, n = 64, 16, 30011
    x, v = synth.particle_cloud(21 + nchi + 2 * nnu, n, nm)
    ref = twin.load(x, v, nc, nchi, nnu, mode)
    with Sim(np_for(nm), nm, 100.0, x_bytes=nchi, v_bytes=nnu, sigma_mode=mode, capacity=n) as sim:
        sim.load_particles(x, v)
        assert_state_equal(sim.get_state(), ref, f"load x{nchi}v{nnu}")


def test_load_many_tiles_bit_exact(Sim):
    """The load path's stable sort by cell over many tiles of 4096 and three 8-bit digit passes
    (2^18 coarse cells), with crowded cells whose particles span tiles."""
    nm, nc, n = 256, 64, 600011
    x, v = synth.particle_cloud(29, n, nm, clump_frac=0.5, n_clumps=20, clump_radius=2.0)
    ref = twin.load(x, v, nc, 1, 1, 1)
    assert ref.cnt.max() > 4096
    with Sim(np_for(nm), nm, 100.0, capacity=n) as sim:
        sim.load_particles(x, v)
        assert_state_equal(sim.get_state(), ref, "load, many tiles")


def test_tables_match(Sim):
    for nnu in (1, 2):
        with Sim(32, 64, 100.0, v_bytes=nnu) as sim:
            dec, edg = sim.get_tables()
        assert np.array_equal(dec, twin.decode_table(nnu))
        assert np.array_equal(edg, twin.edge_table(nnu))


def np_for(nm):
    """Smallest valid lattice side for a mesh: an FFT size, at least 32, a multiple of nm / 4."""
    return next(p for p in (32, 48, 64, 96, 128, 192, 256) if p % (nm // 4) == 0)


DEPOSIT_VARIANTS = [3, 0]  # the default (interleaved order, 512 threads); storage order, 256 threads


@pytest.mark.parametrize("variant", DEPOSIT_VARIANTS)
@pytest.mark.parametrize("clumps", [0.4, 0.0])
@pytest.mark.parametrize("nchi", [1, 2])
@pytest.mark.parametrize("nm", [32, 64, 96, 128])
def test_deposit_bit_exact(Sim, nchi, nm, clumps, variant):
    # clumped clouds put hundreds to thousands of particles in a coarse cell (64-bit LDS sums);
    # without clumps every cell holds fewer than 255 (the 32-bit sums of 1-byte codes)
    nc = nm // 4
    n = 5 * nm**3 // 16 + 7
    x, v = synth.particle_cloud(31 + nm, n, nm, clump_frac=clumps)
    ref = twin.load(x, v, nc, nchi, 1)
    with Sim(np_for(nm), nm, 100.0, x_bytes=nchi, capacity=n) as sim:
        sim.set_state(ref.cnt, ref.chi, ref.nu, ref.vc, ref.vs)
        sim.set_variant(deposit_variant=variant)
        sim.stage_deposit()
        got = sim.get_mesh()
    exp = twin.delta_from_rho(twin.deposit_int(ref, nm), ref.n, nchi)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("variant", DEPOSIT_VARIANTS)
@pytest.mark.parametrize("n", [1, 37, 900])
def test_deposit_sparse_bit_exact(Sim, n, variant):
    # layers with no particle at all and layers with fewer particles than a workgroup has threads
    # (the deposit's software pipeline clamps its look-ahead to the layer's last particle)
    nm = 64
    x, v = synth.particle_cloud(77 + n, n, nm, clump_frac=0.0)
    ref = twin.load(x, v, nm // 4, 1, 1)
    with Sim(np_for(nm), nm, 100.0, capacity=n) as sim:
        sim.set_state(ref.cnt, ref.chi, ref.nu, ref.vc, ref.vs)
        sim.set_variant(deposit_variant=variant)
        sim.stage_deposit()
        got = sim.get_mesh()
    exp = twin.delta_from_rho(twin.deposit_int(ref, nm), ref.n, 1)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("variant", DEPOSIT_VARIANTS)
def test_deposit_dense_layers_bit_exact(Sim, variant):
    """Many chunks of z layers per workgroup column (a 256^3 mesh: interior layers with no plane
    tests) and ring cells with many particles, some at the very edge of their cell."""
    nm = 256
    n = 600000
    x, v = synth.particle_cloud(91, n, nm, clump_frac=0.3, n_clumps=40, clump_radius=3.0)
    x[:5000] = np.floor(x[:5000] / 4.0) * 4.0 + np.where(np.arange(5000)[:, None] % 2 == 0, 1e-6, 4.0 - 1e-6)
    x = np.mod(x, nm)
    ref = twin.load(x, v, nm // 4, 1, 1)
    with Sim(np_for(nm), nm, 100.0, capacity=n) as sim:
        sim.set_state(ref.cnt, ref.chi, ref.nu, ref.vc, ref.vs)
        sim.set_variant(deposit_variant=variant)
        sim.stage_deposit()
        got = sim.get_mesh()
    exp = twin.delta_from_rho(twin.deposit_int(ref, nm), ref.n, 1)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("nm", [32, 64, 96, 192, 256])
def test_solve_within_tolerance(Sim, nm):
    nc = nm // 4
    rng = np.random.default_rng(nm)
    delta = rng.normal(size=(nm, nm, nm)).astype(np.float32)
    with Sim(np_for(nm), nm, 100.0, omega_m=0.3) as sim:
        sim.set_mesh(delta)
        sim.stage_solve()
        phi = sim.get_mesh()
    ref = pm.poisson(delta.astype(np.float64), 0.3)
    assert np.linalg.norm(phi - ref) / np.linalg.norm(ref) < 1e-5
    g = pm.gradient4(phi.astype(np.float64))
    gr = pm.gradient4(ref)
    num = np.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(g, gr)))
    den = np.sqrt(sum((b**2).sum() for b in gr))
    assert num / den < 1e-5


def test_solve_plane_wave_exact(Sim):
    nm, om = 128, 0.3
    i = np.arange(nm)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    kv = 2 * np.pi * np.array([3, -5, 7]) / nm
    arg = kv[0] * x + kv[1] * y + kv[2] * z
    with Sim(32, nm, 100.0, omega_m=om) as sim:
        sim.set_mesh(np.cos(arg).astype(np.float32))
        sim.stage_solve()
        phi = sim.get_mesh()
    exact = -1.5 * om * np.cos(arg) / (kv**2).sum()
    assert np.abs(phi - exact).max() < 1e-5 * np.abs(exact).max()


MOVE_CASES = [
    (1, 1, 1, 64, 40000, 2.0),
    (2, 1, 1, 64, 30000, 1.0),
    (1, 2, 0, 32, 9000, 1.0),
    (2, 2, 1, 64, 25000, 0.5),
    (1, 1, 1, 128, 150000, 1.5),
    # at least half as many particles as fine cells: the gradient tile is precomputed in LDS
    (1, 1, 1, 32, 20000, 1.0),
    (2, 1, 0, 64, 160000, 1.0),
    (1, 1, 1, 64, 300000, 0.7),
    # a 3 * 2^k mesh (radix-3 FFT sizes), generic and dense paths
    (1, 1, 1, 96, 200000, 0.7),
    (1, 1, 1, 96, 460000, 0.7),
]


@pytest.mark.parametrize("nchi,nnu,mode,nm,n,vscale", MOVE_CASES)
def test_move_bit_exact(Sim, nchi, nnu, mode, nm, n, vscale):
    nc = nm // 4
    x, v = synth.particle_cloud(41 + nm + nchi, n, nm, vscale=vscale, clump_frac=0.5, clump_radius=1.0)
    st = twin.load(x, v, nc, nchi, nnu, mode)
    phi = synth.smooth_potential(7 + nm, nm, amp=2.0 if nm >= 64 else 0.5)
    kf, df = np.float32(-1.3 / 12.0), np.float32(0.5)
    exp, info = twin.move(st, phi, kf, df, sigma_mode=mode, return_info=True)
    assert not info["cfl"]
    moved = (info["dcode"] != 13).mean()
    assert moved > 0.02  # many particles change cell, some cross the periodic boundary
    with Sim(np_for(nm), nm, 100.0, x_bytes=nchi, v_bytes=nnu, sigma_mode=mode, capacity=n) as sim:
        sim.set_state(st.cnt, st.chi, st.nu, st.vc, st.vs)
        sim.set_mesh(phi)
        sim.stage_move(kf, df)
        got = sim.get_state()
        assert_state_equal(got, exp, f"move x{nchi}v{nnu}")
        # a second move from the GPU's own output stays bit-exact
        sim.stage_move(kf, df)
        got2 = sim.get_state()
    exp2, info2 = twin.move(exp, phi, kf, df, sigma_mode=mode, return_info=True)
    assert not info2["cfl"]
    assert_state_equal(got2, exp2, "second move")


@pytest.mark.parametrize("move_variant", [1, 0])
def test_move_crowded_cell_bit_exact(Sim, move_variant):
    """One coarse cell holding most of the particles (about 1400 chunks of 64, taken by all the
    wavefronts of its tile in turn): the ranks inside the new cells still follow storage order."""
    nm, n = 32, 100000
    x, v = synth.particle_cloud(17, n, nm, vscale=0.5, clump_frac=0.9, n_clumps=1, clump_radius=0.7)
    st = twin.load(x, v, nm // 4, 1, 1, 1)
    assert st.cnt.max() > 40000
    phi = synth.smooth_potential(9, nm, amp=0.5)
    kf, df = np.float32(-1.3 / 12.0), np.float32(0.5)
    exp, info = twin.move(st, phi, kf, df, sigma_mode=1, return_info=True)
    assert not info["cfl"]
    assert (info["dcode"] != 13).mean() > 0.05
    with Sim(np_for(nm), nm, 100.0, sigma_mode=1, capacity=n) as sim:
        sim.set_state(st.cnt, st.chi, st.nu, st.vc, st.vs)
        sim.set_variant(move_variant=move_variant)
        sim.set_mesh(phi)
        sim.stage_move(kf, df)
        got = sim.get_state()
    assert_state_equal(got, exp, f"crowded cell, move variant {move_variant}")


def test_scatter_wait_limit_raises_error(Sim):
    """The gradient-tile scatter's ordered section is a bounded wait: with the bound forced down
    to one poll, chunks of a crowded tile give up waiting, the move reports the count error and
    is not applied, and with the default bound the same move is bit-exact."""
    from paper_1712_06121_amd import CubeError
    nm, n = 32, 100000
    x, v = synth.particle_cloud(17, n, nm, vscale=0.5, clump_frac=0.9, n_clumps=1, clump_radius=0.7)
    st = twin.load(x, v, nm // 4, 1, 1, 1)
    phi = synth.smooth_potential(9, nm, amp=0.5)
    kf, df = np.float32(-1.3 / 12.0), np.float32(0.5)
    exp = twin.move(st, phi, kf, df, sigma_mode=1)
    with Sim(np_for(nm), nm, 100.0, sigma_mode=1, capacity=n) as sim:
        sim.set_state(st.cnt, st.chi, st.nu, st.vc, st.vs)
        sim.set_variant(move_variant=1)
        sim.set_mesh(phi)
        sim.debug_set_turn_limit(1)
        with pytest.raises(CubeError) as e:
            sim.stage_move(kf, df)
        assert e.value.code == -8  # CUBE_E_STATE: the count changed during the move
        assert_state_equal(sim.get_state(), st, "state after the failed move")
        sim.debug_set_turn_limit(1 << 22)
        sim.set_mesh(phi)
        sim.stage_move(kf, df)
        assert_state_equal(sim.get_state(), exp, "move after the failed one")


def test_cfl_violation_reported(Sim):
    from paper_1712_06121_amd import CubeError
    nm, nc, n = 64, 16, 5000
    x, v = synth.particle_cloud(5, n, nm, vscale=1.0)
    with Sim(32, nm, 100.0, capacity=n) as sim:
        sim.load_particles(x, v)
        sim.set_mesh(np.zeros((nm,) * 3, np.float32))
        with pytest.raises(CubeError) as e:
            sim.stage_move(0.0, 50.0)
        assert e.value.code == -5


@pytest.mark.parametrize("nchi", [1, 2])
def test_get_density_host_and_device(Sim, nchi):
    """cube_get_density into host memory and into device memory equals the FP32 density of the
    exact integer CIC of the same state, element by element."""
    nm, nc, n = 64, 16, 30011
    x, v = synth.particle_cloud(61 + nchi, n, nm)
    ref = twin.load(x, v, nc, nchi, 1)
    exp = twin.delta_from_rho(twin.deposit_int(ref, nm), ref.n, nchi)
    with Sim(np_for(nm), nm, 100.0, x_bytes=nchi, capacity=n) as sim:
        sim.load_particles(x, v)
        host = sim.get_density()
        dev = sim.get_density(device=True)
        assert dev.device.type == "cuda" and dev.dtype.is_floating_point
        dev = dev.cpu().numpy()
    assert np.array_equal(host, exp)
    assert np.array_equal(dev, exp)


def test_get_density_after_steps(Sim):
    cfg = synth.WORKLOADS["c1_pm32"]
    with Sim(**cfg) as sim:
        sim.init_ic()
        sim.step(10)
        got = sim.get_density(device=True).cpu().numpy()
        st = sim.get_state()
    tw = twin_state(st, cfg["nc_side"], cfg["x_bytes"], cfg["v_bytes"])
    assert np.array_equal(got, twin.delta_from_rho(twin.deposit_int(tw, cfg["nm_side"]), tw.n, tw.nchi))


def test_failed_step_is_not_applied(Sim):
    """A step whose move raises an error flag (a CFL error raised from the host before the move of
    step 2 of step(5)) and every later step of the call are not applied: the call reports the step,
    the state and the step count are those after 2 steps, and the run continues from there."""
    from paper_1712_06121_amd import CubeError
    cfg = synth.WORKLOADS["c1_pm32"]
    with Sim(**cfg) as ref:
        ref.init_ic()
        ref.step(2)
        s2, a2 = ref.get_state(), ref.a
        ref.step(3)
        s5 = ref.get_state()
    with Sim(**cfg) as sim:
        sim.init_ic()
        sim.debug_inject_flag(2, 1)
        with pytest.raises(CubeError) as e:
            sim.step(5)
        assert e.value.code == -5 and "step 2" in str(e.value)
        assert sim.steps_done == 2 and sim.a == a2
        got = sim.get_state()
        for key in KEYS:
            assert np.array_equal(got[key], s2[key]), key
        sim.debug_inject_flag(-1, 0)
        sim.step(3)
        got = sim.get_state()
    for key in KEYS:
        assert np.array_equal(got[key], s5[key]), key
