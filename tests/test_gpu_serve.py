"""The continuous-batching simulation server (cube_server_*): jobs that join while others run
give exactly the results they give alone; admission keeps to the memory budget."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KEYS = ("cnt", "chi", "nu", "vc", "vs")


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_06121_amd as m
    return m


def job(side, seed, sigma8=0.8, n_steps=9):
    return dict(np_side=side, nm_side=2 * side, nc_side=side // 2, box=1.5625 * side, omega_m=0.3, omega_l=0.7,
                h=0.7, sigma8=sigma8, n_s=1.0, a_init=0.02, a_final=1.0, n_steps=n_steps, spacing=1, seed=seed)


def alone(lib, cfg):
    with lib.Sim(**cfg) as s:
        s.init_ic()
        s.step(cfg["n_steps"])
        return s.get_state(), s.get_power()


def drain(srv, pending, results, on_finish=None, deadline=60.0):
    t0 = time.time()
    while pending:
        assert time.time() - t0 < deadline, f"jobs {sorted(pending)} did not finish"
        for i in srv.poll():
            st, rc = srv.status(i)
            assert st == srv.FINISHED, (i, rc, srv.job_error(i))
            if on_finish:
                on_finish(i)
            sim = srv.job(i)
            results[i] = (sim.get_state(), sim.get_power())
            srv.release(i)
            pending.discard(i)
        time.sleep(0.001)


def test_jobs_in_the_mix_equal_alone(lib):
    cfgs = {1: job(32, 101), 2: job(48, 102, 0.75), 3: job(64, 103, 0.85), 4: job(32, 104, 0.7),
            5: job(48, 105, 0.9), 6: job(32, 106)}
    results = {}
    with lib.Server(8 << 30, max_active=3, slice_steps=2) as srv:
        # jobs arrive while others are running
        for i in (1, 2):
            srv.submit(cfgs[i], i)
        srv.poll()
        srv.poll()
        for i in (3, 4):
            srv.submit(cfgs[i], i)
        for _ in range(3):
            srv.poll()
        for i in (5, 6):
            srv.submit(cfgs[i], i)
        drain(srv, set(cfgs), results)
        assert srv.stats() == (0, 0, 0)
    for i, cfg in cfgs.items():
        st, (k, pk, nm) = results[i]
        st0, (k0, pk0, nm0) = alone(lib, cfg)
        for key in KEYS:
            assert np.array_equal(st[key], st0[key]), (i, key)
        # shell sums use floating-point atomics: equal up to the order of the additions
        assert np.allclose(pk, pk0, rtol=1e-12, atol=0) and np.array_equal(nm, nm0)


def test_admission_keeps_to_the_budget(lib):
    cfgs = {i: job(48, 200 + i, n_steps=30) for i in range(4)}
    fp = lib.footprint(**cfgs[0])
    results, seen = {}, []
    with lib.Server(fp + fp // 2, max_active=4, slice_steps=1) as srv:
        with pytest.raises(lib.CubeError):
            srv.submit(job(96, 299), 99)  # alone larger than the budget
        for i, c in cfgs.items():
            srv.submit(c, i)

        def check(_i):
            q, a, b = srv.stats()
            seen.append(a)
            assert b <= fp + fp // 2

        drain(srv, set(cfgs), results, on_finish=check)
    assert max(seen) <= 1  # only one job fits at a time


def test_failed_job_is_reported_and_others_finish(lib):
    with lib.Server(8 << 30, max_active=2, slice_steps=3) as srv:
        bad = job(32, 300)
        bad["nm_side"], bad["nc_side"] = 40, 10  # not an FFT size: cube_create refuses it at admission
        srv.submit(bad, 1)
        srv.submit(job(32, 301, n_steps=30), 2)
        done, t0 = {}, time.time()
        while len(done) < 2 and time.time() - t0 < 30:
            for i in srv.poll():
                done[i] = srv.status(i)
            time.sleep(0.001)
        assert done[1][0] == srv.FAILED and done[1][1] == -1 and "nm_side" in srv.job_error(1)
        assert done[2][0] == srv.FINISHED
        srv.release(1)
        srv.release(2)


def test_footprint_bounds_device_bytes(lib):
    for cfg in (job(32, 1), job(48, 2), job(64, 3)):
        fp = lib.footprint(**cfg)
        with lib.Sim(**cfg) as s:
            s.init_ic()
            assert 0.5 * fp < s.device_bytes <= fp
