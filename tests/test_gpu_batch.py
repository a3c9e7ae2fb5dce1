"""Ensembles of boxes stepped together (cube_batch_*) and the equivalent kernel variants.

Every box of a batch must evolve exactly as it does alone, whatever kernel variants the
autotuner picks: states are compared bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS = ("cnt", "chi", "nu", "vc", "vs")


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_06121_amd as m
    return m


def small_ensemble():
    base = dict(omega_m=0.3, omega_l=0.7, h=0.7, a_init=0.02, a_final=1.0, n_steps=12, spacing=1, x_bytes=1,
                v_bytes=1)
    return [
        dict(base, np_side=32, nm_side=64, box=50.0, sigma8=0.8, n_s=0.95, seed=11),
        dict(base, np_side=48, nm_side=96, box=75.0, sigma8=0.75, n_s=0.92, seed=12),
        dict(base, np_side=64, nm_side=128, box=100.0, sigma8=0.85, n_s=0.99, seed=13),
        dict(base, np_side=32, nm_side=64, box=50.0, sigma8=0.7, n_s=0.9, seed=14, x_bytes=2),
    ]


def run_alone(lib, cfg, k, variant=None):
    with lib.Sim(**cfg) as s:
        s.init_ic()
        if variant is not None:
            s.set_variant(**variant)
        s.step(k)
        return s.get_state()


def assert_same(a, b, what):
    for key in KEYS:
        assert np.array_equal(a[key], b[key]), f"{what}: {key}"


def test_batch_equals_each_box_alone(lib):
    cfgs = small_ensemble()
    with lib.Batch(cfgs) as b:
        b.init_ic()
        b.step(3)
        b.step(4)  # two calls: the graph for each state parity, the device step counter re-synced
        got = [box.get_state() for box in b.boxes]
        assert all(box.steps_done == 7 for box in b.boxes)
    for i, cfg in enumerate(cfgs):
        assert_same(got[i], run_alone(lib, cfg, 7), f"box {i}")


def test_batch_stream_mode_equals_alone(lib):
    cfgs = small_ensemble()[:3]
    with lib.Batch(cfgs) as b:
        b.init_ic()
        b.set_mode(b.STREAMS)
        b.step(2)
        b.set_mode(b.GRAPH)  # the modes can be mixed: both keep the boxes at the same step
        b.step(1)
        b.set_mode(b.STREAMS)
        b.step(2)
        got = [box.get_state() for box in b.boxes]
    for i, cfg in enumerate(cfgs):
        assert_same(got[i], run_alone(lib, cfg, 5), f"box {i}")


def test_ensemble_launches_equal_alone(lib):
    """Mode 2: every stage one launch over all boxes (three mesh sizes, a 2-byte position box)."""
    cfgs = small_ensemble()
    with lib.Batch(cfgs) as b:
        b.init_ic()
        b.set_mode(b.ENSEMBLE)
        b.step(3)
        b.step(4)  # both state parities
        b.set_mode(b.GRAPH)  # the modes can be mixed
        b.step(1)
        b.set_mode(b.ENSEMBLE)
        b.step(2)
        got = [box.get_state() for box in b.boxes]
        assert all(box.steps_done == 10 for box in b.boxes)
    for i, cfg in enumerate(cfgs):
        assert_same(got[i], run_alone(lib, cfg, 10), f"box {i}")


# per-box kernel variants: boxes of one stage then take different kernels (one launch each)
ENSEMBLE_VARIANTS = [dict(move_variant=1, deposit_variant=0), dict(move_variant=2, fft_z_layout=1, deposit_variant=1),
                     dict(move_variant=3, deposit_variant=2, fft_z_order=1), dict(move_variant=0, fft_col_width=8)]


def test_ensemble_launches_with_mixed_variants(lib):
    cfgs = small_ensemble()
    with lib.Batch(cfgs) as b:
        b.init_ic()
        for box, v in zip(b.boxes, ENSEMBLE_VARIANTS):
            box.set_variant(**v)
        b.boxes[2].enable_pids(4)
        b.set_mode(b.ENSEMBLE)
        b.step(5)
        got = [box.get_state() for box in b.boxes]
        pids = b.boxes[2].get_pids()
    for i, cfg in enumerate(cfgs):
        with lib.Sim(**cfg) as s:
            s.init_ic()
            s.set_variant(**ENSEMBLE_VARIANTS[i])
            if i == 2:
                s.enable_pids(4)
            s.step(5)
            assert_same(got[i], s.get_state(), f"box {i}")
            if i == 2:
                assert np.array_equal(pids, s.get_pids())


def test_ensemble_launches_need_single_level_solves(lib):
    cfgs = [small_ensemble()[i] for i in (0, 3)]  # 16^3 coarse meshes: the two-level force is available
    with lib.Batch(cfgs) as b:
        b.init_ic()
        b.boxes[1].set_two_level(6.0)
        with pytest.raises(lib.CubeError) as e:
            b.set_mode(b.ENSEMBLE)
        assert e.value.code == -1 and "box 1" in str(e.value)  # CUBE_E_INVALID
        b.boxes[1].set_two_level(0.0)
        b.set_mode(b.ENSEMBLE)
        b.boxes[0].set_two_level(6.0)  # switched on after the mode: the step refuses
        with pytest.raises(lib.CubeError) as e:
            b.step(1)
        assert e.value.code == -1
        assert [box.steps_done for box in b.boxes] == [0, 0]


def test_batch_autotune_keeps_results(lib):
    cfgs = small_ensemble()[:3]
    with lib.Batch(cfgs) as b:
        b.init_ic()
        b.step(2)
        b.autotune()
        variants = [box.variant for box in b.boxes]
        b.step(3)
        got = [box.get_state() for box in b.boxes]
    print("variants", variants)
    for i, cfg in enumerate(cfgs):
        assert_same(got[i], run_alone(lib, cfg, 5), f"box {i}")


VARIANTS = [dict(move_variant=0, fft_col_width=8), dict(move_variant=1, fft_col_width=8),
            dict(move_variant=2), dict(move_variant=3), dict(move_variant=-1),
            dict(move_variant=0, fft_col_width=16, fft_z_order=1), dict(move_variant=1, fft_col_width=16),
            dict(deposit_variant=1), dict(deposit_variant=2), dict(deposit_variant=3, fft_z_order=1),
            dict(fft_z_layout=1), dict(fft_z_layout=1, fft_col_width=16),
            dict(fft_z_layout=1, fft_col_width=16, fft_z_width=8)]


@pytest.mark.parametrize("variant", VARIANTS)
def test_variants_are_bit_identical(lib, variant):
    cfg = dict(synth.WORKLOADS["c1_pm32"], n_steps=12)
    ref = run_alone(lib, cfg, 6)
    assert_same(run_alone(lib, cfg, 6, variant), ref, f"variant {variant}")


@pytest.mark.parametrize("nm", [192, 384, 512])
def test_fft_variants_bit_identical_at_ensemble_sizes(lib, nm):
    """Every column width, z layout, z width and z order of the Poisson solve gives the same
    potential bit for bit at the mesh sizes of the ensembles (radix-3 sizes included): the FFT
    kernels write their fused multiply-adds out, so no instantiation rounds differently."""
    cfg = dict(synth.WORKLOADS["c1_pm32"], np_side=nm // 2, nm_side=nm, nc_side=nm // 4, box=1.5625 * nm / 2,
               omega_m=0.3, omega_l=0.7, seed=21)
    pots = {}
    with lib.Sim(**cfg) as s:
        s.init_ic()
        for v in (dict(fft_col_width=16, fft_z_layout=0, fft_z_order=0), dict(fft_col_width=8, fft_z_layout=0),
                  dict(fft_col_width=16, fft_z_layout=0, fft_z_order=1),
                  dict(fft_col_width=16, fft_z_layout=1, fft_z_width=16),
                  dict(fft_col_width=16, fft_z_layout=1, fft_z_width=8),
                  dict(fft_col_width=8, fft_z_layout=1, fft_z_width=8)):
            s.set_variant(**v)
            s.stage_deposit()
            s.stage_solve()
            pots[str(v)] = s.get_mesh().copy()
    ref = next(iter(pots.values()))
    for k, p in pots.items():
        assert np.array_equal(p, ref), f"{k}: {int(np.sum(p != ref))} values differ"


def test_variant_validation(lib):
    with lib.Sim(**synth.WORKLOADS["c1_pm32"]) as s:
        before = s.variant
        for bad in (dict(move_variant=4), dict(fft_col_width=4), dict(fft_z_order=3), dict(deposit_variant=4),
                    dict(fft_z_layout=2), dict(fft_col_width=8, fft_z_width=16)):
            with pytest.raises(lib.CubeError):
                s.set_variant(**bad)
        assert s.variant == before


def test_batch_runs_to_the_end(lib):
    # steps fine enough that no particle crosses more than one coarse cell per step
    cfgs = [dict(c, n_steps=40) for c in small_ensemble()[:2]]
    with lib.Batch(cfgs) as b:
        b.init_ic()
        assert b.step(30) == lib.CUBE_OK
        assert b.step(15) == lib.CUBE_DONE
        assert all(box.steps_done == 40 and box.a == pytest.approx(1.0) for box in b.boxes)
        k, pk, nmodes = b.boxes[1].get_power()
        assert np.all(np.isfinite(pk)) and pk[0] > 0


def test_batch_refuses_boxes_out_of_step(lib):
    cfgs = small_ensemble()[:2]
    with lib.Batch(cfgs) as b:
        b.init_ic()
        b.boxes[0].step(1)  # a box stepped alone leaves the batch out of step
        with pytest.raises(lib.CubeError) as e:
            b.step(1)
        assert "same step" in str(e.value)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_failed_box_stops_at_its_step(lib, mode):
    """A box whose step fails (a CFL error raised from the host before the move of step 2) stays at
    the state before that step; the other boxes complete their steps."""
    cfgs = small_ensemble()[:3]
    with lib.Batch(cfgs) as b:
        b.set_mode(mode)
        b.init_ic()
        b.boxes[1].debug_inject_flag(2, 1)
        with pytest.raises(lib.CubeError) as e:
            b.step(4)
        assert e.value.code == -5 and "box 1" in str(e.value) and "step 2" in str(e.value)
        assert [box.steps_done for box in b.boxes] == [4, 2, 4]
        got = [box.get_state() for box in b.boxes]
    assert_same(got[0], run_alone(lib, cfgs[0], 4), "box 0")
    assert_same(got[1], run_alone(lib, cfgs[1], 2), "box 1")
    assert_same(got[2], run_alone(lib, cfgs[2], 4), "box 2")
